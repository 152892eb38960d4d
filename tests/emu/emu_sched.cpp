// Fiber scheduler of the host workgroup emulation (see emu_sched.hpp).
#include "emu_sched.hpp"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#endif
#endif
#ifdef EMU_ASAN
#include <sanitizer/common_interface_defs.h>
#endif

extern "C" void emu_ctx_switch(void** save_sp, void* new_sp);
extern "C" void emu_ctx_entry();

// x86-64 System V: save the callee-saved registers on the current stack,
// store the stack pointer, load the other one and restore its registers.
// A new fiber starts in emu_ctx_entry with r12 = argument, r13 = function.
asm(R"(
  .text
  .globl emu_ctx_switch
  .type emu_ctx_switch,@function
emu_ctx_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_ctx_switch, .-emu_ctx_switch
  .globl emu_ctx_entry
  .type emu_ctx_entry,@function
emu_ctx_entry:
  movq %r12, %rdi
  callq *%r13
  ud2
  .size emu_ctx_entry, .-emu_ctx_entry
)");

namespace emu {

Group* g_group = nullptr;
Lane* g_cur = nullptr;

namespace {

constexpr size_t kStack = 512 * 1024;
struct LaneExtra {
  WaveFn fn;
  const char* name;
};
LaneExtra g_extra[kMaxThreads];
void* g_sched_fake = nullptr;

[[noreturn]] void die(const char* what, const char* name) {
  fprintf(stderr, "emu: %s%s%s\n", what, name ? ": " : "", name ? name : "");
  fflush(stderr);
  abort();
}

void start_switch(void** fake_save, const void* bottom, size_t size) {
#ifdef EMU_ASAN
  __sanitizer_start_switch_fiber(fake_save, bottom, size);
#else
  (void)fake_save; (void)bottom; (void)size;
#endif
}
void finish_switch(void* fake, const void** bottom_old, size_t* size_old) {
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(fake, bottom_old, size_old);
#else
  (void)fake; (void)bottom_old; (void)size_old;
#endif
}

void to_scheduler() {
  Lane* L = g_cur;
  start_switch(L->st == St::Done ? nullptr : &L->fake_stack, g_group->sched_stack_bottom,
               g_group->sched_stack_size);
  ++g_group->switches;
  emu_ctx_switch(&L->sp, g_group->sched_sp);
  finish_switch(L->fake_stack, nullptr, nullptr);
}

void to_lane(Lane* L) {
  g_cur = L;
  start_switch(&g_sched_fake, L->stack, L->stack_size);
  emu_ctx_switch(&g_group->sched_sp, L->sp);
  finish_switch(g_sched_fake, nullptr, nullptr);
  g_cur = nullptr;
}

extern "C" void fiber_main(void* arg) {
  Lane* L = static_cast<Lane*>(arg);
  finish_switch(nullptr, &g_group->sched_stack_bottom, &g_group->sched_stack_size);
  g_cur = L;
  g_group->body(g_group->body_arg);
  L->st = St::Done;
  to_scheduler();
  die("finished fiber resumed", nullptr);
}

}  // namespace

void syncthreads() {
  g_cur->st = St::Barrier;
  to_scheduler();
}

void wave_collective(WaveFn fn, const char* name, int arg) {
  const int t = (int)g_cur->idx.x;
  g_extra[t].fn = fn;
  g_extra[t].name = name;
  WaveOp& w = my_wave_op();
  w.fn = fn;
  w.name = name;
  w.arg = arg;
  g_cur->st = St::WaveOp;
  to_scheduler();
}

void run_group(int nthreads, unsigned bx, unsigned gx, void (*body)(void*), void* arg) {
  run_group2(nthreads, bx, 0, gx, 1, body, arg);
}

void run_group2(int nthreads, unsigned bx, unsigned by, unsigned gx, unsigned gy,
                void (*body)(void*), void* arg) {
  if (nthreads < 1 || nthreads > kMaxThreads || nthreads % kWave) die("bad workgroup size", nullptr);
  static Group* G = nullptr;
  if (!G) {
    G = static_cast<Group*>(calloc(1, sizeof(Group)));
    for (int t = 0; t < kMaxThreads; ++t) {
      void* p = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
      if (p == MAP_FAILED) die("mmap of a fiber stack failed", nullptr);
      mprotect(p, 4096, PROT_NONE);  // guard page below the stack
      G->lanes[t].stack = static_cast<unsigned char*>(p);
      G->lanes[t].stack_size = kStack;
    }
  }
  g_group = G;
  G->nthreads = nthreads;
  G->bidx = Dim3{bx, by, 0};
  G->bdim = Dim3{(unsigned)nthreads, 1, 1};
  G->gdim = Dim3{gx, gy, 1};
  G->body = body;
  G->body_arg = arg;
  for (int t = 0; t < nthreads; ++t) {
    Lane& L = G->lanes[t];
    L.idx = Dim3{(unsigned)t, 0, 0};
    L.st = St::Run;
    L.fake_stack = nullptr;
    // initial frame popped by emu_ctx_switch: r15 r14 r13 r12 rbx rbp, return
    // address; the stack is 16-byte aligned when emu_ctx_entry calls
    uintptr_t top = reinterpret_cast<uintptr_t>(L.stack + L.stack_size) & ~(uintptr_t)15;
    uint64_t* sp = reinterpret_cast<uint64_t*>(top - 72);
    memset(sp, 0, 72);
    sp[2] = reinterpret_cast<uint64_t>(&fiber_main);   // r13: function
    sp[3] = reinterpret_cast<uint64_t>(&L);            // r12: argument
    sp[6] = reinterpret_cast<uint64_t>(&emu_ctx_entry);
    L.sp = sp;
  }
  const int nw = nthreads / kWave;
  for (;;) {
    bool ran = false;
    for (int w = 0; w < nw; ++w) {
      for (int l = 0; l < kWave; ++l) {
        Lane& L = G->lanes[w * kWave + l];
        if (L.st == St::Run) {
          to_lane(&L);
          ran = true;
        }
      }
      int nop = 0;
      for (int l = 0; l < kWave; ++l) nop += G->lanes[w * kWave + l].st == St::WaveOp;
      if (nop == 0) continue;
      WaveOp& op = G->wops[w];
      if (nop != kWave) die("wave collective not reached by the whole wave", op.name);
      for (int l = 0; l < kWave; ++l)
        if (g_extra[w * kWave + l].fn != op.fn) die("lanes of one wave in different collectives", op.name);
      op.fn(op);
      for (int l = 0; l < kWave; ++l) G->lanes[w * kWave + l].st = St::Run;
      ran = true;
    }
    if (ran) continue;
    int nbar = 0, ndone = 0;
    for (int t = 0; t < nthreads; ++t) {
      nbar += G->lanes[t].st == St::Barrier;
      ndone += G->lanes[t].st == St::Done;
    }
    if (ndone == nthreads) break;
    if (nbar != nthreads) die("barrier reached by only part of the workgroup", nullptr);
    for (int t = 0; t < nthreads; ++t) G->lanes[t].st = St::Run;
  }
  g_group = nullptr;
}

}  // namespace emu
