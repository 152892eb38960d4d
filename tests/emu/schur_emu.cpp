// Host driver that executes the Schur-update kernel (rid::k_schur, compiled
// from the library's own header) in the workgroup emulation, under
// AddressSanitizer (TEST INFRASTRUCTURE).  Every buffer is an exact-size
// allocation.
//
// Input file (little endian): int32 dtype (0 FP64, 1 FP32), n, ldz, k, kb, zcol,
// w, ldu, nt, from, cg, want_norm; then Z (n x ldz), U2T (w x ldu) in the
// dtype and pos (n int32).  Output: Z after the kernel, then the grid's FP64
// norm partials.  With a third argument ksplit the split-K form runs instead
// (rid::k_schur_sk over ceil(n/64) x ceil(k/ksplit) workgroups with nt
// column tiles, then rid::k_schur_fin with 64/cg rows per workgroup); kb and
// from must then be 0; a fourth argument "bf" runs the FP32 form on the BF16
// matrix cores (rid::k_schur_skb) instead of rid::k_schur_sk.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "hip/hip_runtime.h"
#include "rid_schur.hpp"

namespace {

template <typename T>
void rd(FILE* f, T* v, size_t n = 1) {
  if (fread(v, sizeof(T), n, f) != n) {
    fprintf(stderr, "schur_emu: short input\n");
    exit(2);
  }
}

struct Args {
  void* Z;
  int64_t ldz, n;
  const int* pos;
  int kb, k, zcol, w;
  const void* U2T;
  int64_t ldu;
  double* norm;
  const rid::Ctrl* ctrl;
  int want;
  int dtype, nt, from, cg;
};

template <typename TF, int NT, bool FROM, int CG>
void launch(Args& a) {
  rid::k_schur<TF, NT, FROM, CG>(static_cast<TF*>(a.Z), a.ldz, a.n, a.pos, a.kb, a.k, a.zcol,
                                 a.w, static_cast<const TF*>(a.U2T), a.ldu, a.norm, a.ctrl,
                                 a.want);
}

template <typename TF>
void dispatch(Args& a) {
  // the instantiations the library launches for a block of w <= 64 columns
  if (a.from) {
    if (a.nt == 1 && a.cg == 1) return launch<TF, 1, true, 1>(a);
  } else if (a.cg == 1) {
    switch (a.nt) {
      case 1: return launch<TF, 1, false, 1>(a);
      case 2: return launch<TF, 2, false, 1>(a);
      case 3: return launch<TF, 3, false, 1>(a);
      case 4: return launch<TF, 4, false, 1>(a);
      case 8: return launch<TF, 8, false, 1>(a);
    }
  } else if (a.cg == 2) {
    switch (a.nt) {
      case 1: return launch<TF, 1, false, 2>(a);
      case 2: return launch<TF, 2, false, 2>(a);
      case 4: return launch<TF, 4, false, 2>(a);
    }
  } else if (a.cg == 4) {
    switch (a.nt) {
      case 1: return launch<TF, 1, false, 4>(a);
      case 2: return launch<TF, 2, false, 4>(a);
    }
  }
  fprintf(stderr, "schur_emu: no instantiation for nt=%d cg=%d from=%d\n", a.nt, a.cg, a.from);
  exit(2);
}

void body(void* p) {
  Args& a = *static_cast<Args*>(p);
  if (a.dtype == 0)
    dispatch<double>(a);
  else
    dispatch<float>(a);
}

struct SkArgs {
  Args* a;
  int ksplit, nsplit;
  double* P;
  int bf;  // FP32 on the BF16 matrix cores (k_schur_skb)
};

template <typename TF, int NT>
void launch_sk(SkArgs& s) {
  Args& a = *s.a;
  if constexpr (sizeof(TF) == 4) {
    if (s.bf) {
      rid::k_schur_skb<NT>(static_cast<const float*>(a.Z), a.ldz, a.n, a.k, a.w,
                           static_cast<const float*>(a.U2T), a.ldu, s.ksplit, s.P, a.ctrl);
      return;
    }
  }
  rid::k_schur_sk<TF, NT>(static_cast<const TF*>(a.Z), a.ldz, a.n, a.k, a.w,
                          static_cast<const TF*>(a.U2T), a.ldu, s.ksplit, s.P, a.ctrl);
}

template <typename TF>
void dispatch_sk(SkArgs& s) {
  switch (s.a->nt) {
    case 1: return launch_sk<TF, 1>(s);
    case 2: return launch_sk<TF, 2>(s);
    case 3: return launch_sk<TF, 3>(s);
    case 4: return launch_sk<TF, 4>(s);
  }
  fprintf(stderr, "schur_emu: no split-K instantiation for nt=%d\n", s.a->nt);
  exit(2);
}

void body_sk(void* p) {
  SkArgs& s = *static_cast<SkArgs*>(p);
  if (s.a->dtype == 0)
    dispatch_sk<double>(s);
  else
    dispatch_sk<float>(s);
}

void body_fin(void* p) {
  SkArgs& s = *static_cast<SkArgs*>(p);
  Args& a = *s.a;
  if (a.dtype == 0)
    rid::k_schur_fin<double>(static_cast<double*>(a.Z), a.ldz, a.n, a.pos, a.zcol, a.w, s.P,
                             s.nsplit, 64 / a.cg, a.norm, a.ctrl, a.want);
  else
    rid::k_schur_fin<float>(static_cast<float*>(a.Z), a.ldz, a.n, a.pos, a.zcol, a.w, s.P,
                            s.nsplit, 64 / a.cg, a.norm, a.ctrl, a.want);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 3 || argc > 5) return 2;
  const int ksplit = argc >= 4 ? atoi(argv[3]) : 0;
  const int bf = argc == 5 && strcmp(argv[4], "bf") == 0;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t h[12];
  rd(f, h, 12);
  const int dtype = h[0], n = h[1], ldz = h[2], k = h[3], kb = h[4], zcol = h[5], w = h[6];
  const int ldu = h[7], nt = h[8], from = h[9], cg = h[10], want = h[11];
  const size_t es = dtype == 0 ? 8 : 4;
  void* Z = malloc((size_t)n * ldz * es);
  void* U2T = malloc((size_t)w * ldu * es);
  int* pos = static_cast<int*>(malloc((size_t)n * 4));
  rd(f, static_cast<unsigned char*>(Z), (size_t)n * ldz * es);
  rd(f, static_cast<unsigned char*>(U2T), (size_t)w * ldu * es);
  rd(f, pos, (size_t)n);
  fclose(f);
  const int grid = (n + 64 / cg - 1) / (64 / cg);
  double* norm = static_cast<double*>(malloc((size_t)grid * 8));
  rid::Ctrl* ctrl = static_cast<rid::Ctrl*>(calloc(1, sizeof(rid::Ctrl)));
  Args a{Z, ldz, n, pos, kb, k, zcol, w, U2T, ldu, norm, ctrl, want, dtype, nt, from, cg};
  if (ksplit > 0) {
    if (kb != 0 || from != 0) return 2;
    const int nsplit = (k + ksplit - 1) / ksplit;
    const int slabs = (n + 63) / 64;
    const size_t np = (size_t)nsplit * n * 64;
    double* P = static_cast<double*>(malloc(np * 8));
    for (size_t i = 0; i < np; ++i) P[i] = __builtin_nan("");  // unwritten partials show up
    SkArgs s{&a, ksplit, nsplit, P, bf};
    for (int y = 0; y < nsplit; ++y)
      for (int x = 0; x < slabs; ++x)
        emu::run_group2(256, (unsigned)x, (unsigned)y, (unsigned)slabs, (unsigned)nsplit,
                        &body_sk, &s);
    for (int g = 0; g < grid; ++g) emu::run_group(256, (unsigned)g, (unsigned)grid, &body_fin, &s);
    free(P);
  } else {
    for (int g = 0; g < grid; ++g) emu::run_group(256, (unsigned)g, (unsigned)grid, &body, &a);
  }
  FILE* o = fopen(argv[2], "wb");
  if (!o) return 2;
  fwrite(Z, es, (size_t)n * ldz, o);
  fwrite(norm, 8, (size_t)grid, o);
  fclose(o);
  return 0;
}
