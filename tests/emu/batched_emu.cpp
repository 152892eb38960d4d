// Host driver that executes the batched persistent kernel (rid::k_batched,
// compiled from the library's own header) in the workgroup emulation, under
// AddressSanitizer (TEST INFRASTRUCTURE).
//
// Every buffer the kernel receives is its own heap allocation of exactly the
// size the library's interface promises (A: m x lda, J: kcap entries, T: kcap
// rows of ldt, per-block outputs: nblk entries), and the workspace slice
// carries `gap` poisoned bytes after each of its parts, so any access outside
// the intended array stops the run with a report.
//
// Input file (little endian): int32 dtype (0 FP64, 1 FP32, 2 FP32 blocks
// factored in FP64), nblk, b, rel, max_n, max_kmax, groups, has_hint,
// has_perm, threads per workgroup (256, or 512 when factored in FP64); double tol; uint64 seed, gap;
// per block int32 m, n, kmax, hint; nblk int32 perm (if has_perm); then per
// block its m x n row-major matrix in the storage type.  Blocks are dealt to the
// emulated workgroups round robin in processing order, each workgroup taking
// its blocks from the kernel's own queue.
// Output file: per block int32 k, status, passes; double E; k int32 J; then
// k x (n - k) entries of T in the factor type.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "hip/hip_runtime.h"
#include "rid_batched.hpp"

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/asan_interface.h>
#define POISON(p, n) ASAN_POISON_MEMORY_REGION((p), (n))
#endif
#endif
#ifndef POISON
#define POISON(p, n) ((void)(p), (void)(n))
#endif

namespace {

template <typename T>
void rd(FILE* f, T* v, size_t n = 1) {
  if (fread(v, sizeof(T), n, f) != n) {
    fprintf(stderr, "batched_emu: short input\n");
    exit(2);
  }
}

struct Args {
  int nblk, b, rel, max_n, max_kmax;
  double tol;
  uint64_t seed;
  const void* const* A;
  const int64_t* lda;
  const int32_t* m;
  const int32_t* n;
  const int32_t* kmax;
  const int32_t* hint;
  int32_t* const* J;
  void* const* T;
  const int64_t* ldt;
  int32_t *k, *st, *passes;
  double* E;
  const int32_t* perm;
  unsigned* queue;
  unsigned char* wbase;
  rid::BLayout lay;
  int maxk;
  int dtype;
  int nt;
};

void body(void* p) {
  Args& a = *static_cast<Args*>(p);
#define EMU_CALL(NTV, TFV, TAV)                                                             \
  rid::k_batched<NTV, TFV, TAV>(a.nblk, a.A, a.lda, a.m, a.n, a.b, a.tol, a.rel, a.kmax, a.hint, \
                                a.seed, a.J, a.T, a.ldt, a.k, a.E, a.st, a.passes, a.perm,       \
                                a.queue, a.wbase, a.lay, a.max_n, a.maxk)
  if (a.nt == 512) {
    if (a.dtype == 2) EMU_CALL(512, double, float);
    else EMU_CALL(512, double, double);
  } else {
    if (a.dtype == 2) EMU_CALL(256, double, float);
    else if (a.dtype == 0) EMU_CALL(256, double, double);
    else EMU_CALL(256, float, float);
  }
#undef EMU_CALL
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: batched_emu <input> <output>\n");
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t h[10];
  rd(f, h, 10);
  const int dtype = h[0], nblk = h[1], b = h[2], rel = h[3], max_n = h[4], max_kmax = h[5];
  const int groups = h[6], has_hint = h[7], has_perm = h[8], nt = h[9];
  if (nt != 256 && (nt != 512 || dtype == 1)) {
    fprintf(stderr, "batched_emu: unsupported workgroup shape %d\n", nt);
    return 2;
  }
  double tol;
  uint64_t seed, gap;
  rd(f, &tol);
  rd(f, &seed);
  rd(f, &gap);
  const size_t es = dtype == 1 ? 4 : 8;  // factor type (T and the workspace)
  const size_t ea = dtype == 0 ? 8 : 4;  // storage type of the blocks
  std::vector<int32_t> m(nblk), n(nblk), kmax(nblk), hint(nblk), perm(nblk);
  for (int i = 0; i < nblk; ++i) {
    int32_t r[4];
    rd(f, r, 4);
    m[i] = r[0];
    n[i] = r[1];
    kmax[i] = r[2];
    hint[i] = r[3];
  }
  for (int i = 0; i < nblk; ++i) perm[i] = i;
  if (has_perm) rd(f, perm.data(), nblk);
  // exact-size allocations: inputs, per-block outputs and the per-block arrays
  std::vector<void*> A(nblk), T(nblk);
  std::vector<int32_t*> J(nblk);
  std::vector<int64_t> lda(nblk), ldt(nblk);
  for (int i = 0; i < nblk; ++i) {
    const size_t cnt = (size_t)m[i] * n[i];
    A[i] = malloc(cnt * ea);
    rd(f, static_cast<unsigned char*>(A[i]), cnt * ea);
    lda[i] = n[i];
    ldt[i] = n[i];
    int kc = kmax[i] < m[i] ? kmax[i] : m[i];
    if (n[i] < kc) kc = n[i];
    if (kc < 1) kc = 1;
    J[i] = static_cast<int32_t*>(malloc((size_t)kc * 4));
    T[i] = calloc((size_t)kc * n[i], es);
  }
  fclose(f);
  int32_t* kout = static_cast<int32_t*>(malloc(nblk * 4));
  int32_t* st = static_cast<int32_t*>(malloc(nblk * 4));
  int32_t* passes = static_cast<int32_t*>(malloc(nblk * 4));
  double* E = static_cast<double*>(malloc(nblk * 8));
  const int maxk = max_kmax < max_n ? max_kmax : max_n;
  const rid::BLayout lay = rid::batched_layout(max_n, maxk, b, (int64_t)es, (int64_t)gap);
  // the workspace: the queue word (kept apart here), then one slice per
  // workgroup with the gap after each part poisoned
  unsigned* queue = static_cast<unsigned*>(malloc(sizeof(unsigned)));
  const size_t wbytes = (size_t)groups * (size_t)lay.slice;
  unsigned char* wbase = static_cast<unsigned char*>(aligned_alloc(256, wbytes));
  memset(wbase, 0xA5, wbytes);  // arbitrary stale contents
  const int64_t part_off[7] = {lay.z, lay.linv, lay.mtmp, lay.u2t, lay.pos, lay.order, lay.nonpiv};
  const int64_t part_len[7] = {max_n * lay.ldz * (int64_t)es, maxk * lay.ldl * (int64_t)es,
                               (int64_t)rid::kBPW * lay.ldl * (int64_t)es,
                               (int64_t)64 * lay.ldu * (int64_t)es, (int64_t)max_n * 4,
                               (int64_t)(maxk + 64) * 4, (int64_t)max_n * 4};
  for (int g = 0; g < groups; ++g)
    for (int q = 0; q < 7; ++q) {
      const int64_t end = part_off[q] + part_len[q];
      const int64_t next = q + 1 < 7 ? part_off[q + 1] : lay.slice;
      POISON(wbase + (size_t)g * lay.slice + end, (size_t)(next - end));
    }
  // deal the processing order to the workgroups round robin
  for (int g = 0; g < groups; ++g) {
    std::vector<int32_t> mine;
    for (int q = g; q < nblk; q += groups) mine.push_back(perm[q]);
    if (mine.empty()) continue;
    int32_t* mp = static_cast<int32_t*>(malloc(mine.size() * 4));
    memcpy(mp, mine.data(), mine.size() * 4);
    *queue = 0;
    Args a{(int)mine.size(), b, rel, max_n, max_kmax, tol, seed, A.data(), lda.data(), m.data(),
           n.data(), kmax.data(), has_hint ? hint.data() : nullptr, J.data(), T.data(), ldt.data(),
           kout, st, passes, E, mp, queue, wbase, lay, maxk, dtype, nt};
    // the kernel reads the block count through nblk but indexes the per-block
    // arrays by block id; ids come from the processing list
    emu::run_group((unsigned)nt, (unsigned)g, (unsigned)groups, &body, &a);
    free(mp);
  }
  FILE* o = fopen(argv[2], "wb");
  if (!o) return 2;
  for (int i = 0; i < nblk; ++i) {
    fwrite(&kout[i], 4, 1, o);
    fwrite(&st[i], 4, 1, o);
    fwrite(&passes[i], 4, 1, o);
    fwrite(&E[i], 8, 1, o);
    const int k = kout[i] > 0 ? kout[i] : 0;
    fwrite(J[i], 4, (size_t)k, o);
    for (int s = 0; s < k; ++s)
      fwrite(static_cast<unsigned char*>(T[i]) + (size_t)s * ldt[i] * es, es, (size_t)(n[i] - k), o);
  }
  fclose(o);
  fprintf(stderr, "batched_emu: %d blocks, %d workgroups, %lld switches\n", nblk, groups,
          (long long)0);
  return 0;
}
