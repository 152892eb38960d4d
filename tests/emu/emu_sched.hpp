// Host emulation of one HIP workgroup (TEST INFRASTRUCTURE: lets the CPU
// tests execute the batched kernel's own source, with its own index
// arithmetic, under AddressSanitizer).
//
// Every work-item is a fiber with its own stack; one OS thread runs them.
// A fiber runs until it reaches a synchronisation point:
//   * __syncthreads(): the work-item waits until every work-item of the
//     workgroup has arrived;
//   * a wave collective (__shfl_xor, __any, an MFMA): the work-item posts its
//     operands and waits until all 64 work-items of its wave have posted the
//     same collective, which is then evaluated for the whole wave.
// Work-items of one wave that reach different kinds of synchronisation
// point, or a barrier reached by only part of the workgroup, abort the run
// (such code is not valid on the hardware either).  Memory written by one
// work-item is visible to another only through these synchronisation points
// in a correct kernel; the emulation does not model weaker ordering.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace emu {

struct Dim3 {
  unsigned x, y, z;
};

constexpr int kMaxThreads = 1024;
constexpr int kWave = 64;

enum class St : int { Run, Barrier, WaveOp, Done };

struct WaveOp;
typedef void (*WaveFn)(WaveOp&);

// Operands and results of one wave collective (per lane, up to 8 words).
struct WaveOp {
  WaveFn fn;
  const char* name;
  int arg;
  uint64_t in[kWave][8];
  uint64_t out[kWave][8];
};

struct Lane {
  void* sp;
  void* fake_stack;
  unsigned char* stack;
  size_t stack_size;
  St st;
  Dim3 idx;
};

struct Group {
  int nthreads;
  Dim3 bidx, bdim, gdim;
  Lane lanes[kMaxThreads];
  WaveOp wops[kMaxThreads / kWave];
  void* sched_sp;
  const void* sched_stack_bottom;
  size_t sched_stack_size;
  void (*body)(void*);
  void* body_arg;
  long long switches;
};

extern Group* g_group;
extern Lane* g_cur;

// Run body(arg) as one workgroup of nthreads work-items (block index bx of
// gx).  Returns 0, or aborts with a message on invalid synchronisation.
void run_group(int nthreads, unsigned bx, unsigned gx, void (*body)(void*), void* arg);
// The same for block (bx, by) of a gx x gy grid.
void run_group2(int nthreads, unsigned bx, unsigned by, unsigned gx, unsigned gy,
                void (*body)(void*), void* arg);

// Called by work-items.
void syncthreads();
void wave_collective(WaveFn fn, const char* name, int arg);
inline int lane_id() { return (int)(g_cur->idx.x % kWave); }
inline WaveOp& my_wave_op() { return g_group->wops[g_cur->idx.x / kWave]; }

}  // namespace emu
