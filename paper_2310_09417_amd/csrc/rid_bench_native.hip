// Native driver for profiling the library without Python: runs, through the
// C ABI, the sketch of one block and the whole adaptive decomposition on an
// m x n FP32 matrix resident in HBM, plus one plain device copy of a known
// size (the reference for hardware traffic counters).
//
// usage: rid_bench_native [m n b kmax iters fmt [libs]]
//        (defaults 50000 20000 64 2048 3 0)
// fmt 0: A in FP32; 1: A stored as BF16; 2: A stored as FP8-e4m3 (scale 1 per
// 128-column tile; the Gaussian entries fit the format unscaled); 3: the three
// in turn, in one process.  With a seventh argument "libs" the driver lists the
// executable address ranges of every loaded object before it returns (to place
// the addresses of stack traces printed at process exit by tools).
// The matrix holds Gaussian entries produced by rid_debug_gaussian; traffic
// and timing of the kernels do not depend on the values.
#include <hip/hip_runtime.h>

#include <link.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <vector>

#include "../../include/rid.h"

#define CHECK(x)                                                             \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) {                                                  \
      std::fprintf(stderr, "%s:%d %s\n", __FILE__, __LINE__, hipGetErrorString(e_)); \
      return 1;                                                              \
    }                                                                        \
  } while (0)

__global__ void calib_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Streaming read of n4 16-byte words (four independent loads in flight per
// thread); one value per thread is written so the loads are kept.
__global__ void calib_read(const float4* __restrict__ src, size_t n4, float* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  float4 a = {0.f, 0.f, 0.f, 0.f}, b = a, c = a, d = a;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const float4 x = src[i], y = src[i + stride], z = src[i + 2 * stride], w = src[i + 3 * stride];
    a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
    b.x += y.x; b.y += y.y; b.z += y.z; b.w += y.w;
    c.x += z.x; c.y += z.y; c.z += z.z; c.w += z.w;
    d.x += w.x; d.y += w.y; d.z += w.z; d.w += w.w;
  }
  for (; i < n4; i += stride) {
    const float4 x = src[i];
    a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] =
      (a.x + a.y + a.z + a.w) + (b.x + b.y + b.z + b.w) + (c.x + c.y + c.z + c.w) +
      (d.x + d.y + d.z + d.w);
}

// FP32 -> BF16 bits (nearest even) or e4m3 codes, one entry per thread.
__global__ void to_format(const float* __restrict__ src, unsigned char* __restrict__ dst,
                          size_t count, int fmt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float x = src[i];
  if (fmt == 1) {
    const unsigned u = __float_as_uint(x);
    reinterpret_cast<unsigned short*>(dst)[i] = (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  } else {
    dst[i] = (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xff);
  }
}

__global__ void fill_ones(float* p, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 1.0f;
}

static int print_segments(struct dl_phdr_info* info, size_t, void*) {
  const char* name = (info->dlpi_name && info->dlpi_name[0]) ? info->dlpi_name : "(main program)";
  for (int i = 0; i < info->dlpi_phnum; ++i) {
    const ElfW(Phdr)& ph = info->dlpi_phdr[i];
    if (ph.p_type == PT_LOAD && (ph.p_flags & PF_X))
      std::printf("[native] text 0x%lx-0x%lx %s\n", (unsigned long)(info->dlpi_addr + ph.p_vaddr),
                  (unsigned long)(info->dlpi_addr + ph.p_vaddr + ph.p_memsz), name);
  }
  return 0;
}

// Plain device copy of a known size: the reference for the traffic counters.
static int calibrate(hipStream_t st) {
  // calibration copy: 1 GiB read, 1 GiB written
  const size_t cbytes = (size_t)1 << 30;
  float *csrc = nullptr, *cdst = nullptr;
  CHECK(hipMalloc(&csrc, cbytes));
  CHECK(hipMalloc(&cdst, cbytes));
  CHECK(hipMemsetAsync(csrc, 0, cbytes, st));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  CHECK(hipEventRecord(e0, st));
  hipLaunchKernelGGL(calib_copy, dim3(4096), dim3(256), 0, st, (const float4*)csrc, (float4*)cdst,
                     cbytes / 16);
  CHECK(hipEventRecord(e1, st));
  CHECK(hipStreamSynchronize(st));
  float ms_copy = 0.f;
  CHECK(hipEventElapsedTime(&ms_copy, e0, e1));
  std::printf("[native] calibration copy: %zu bytes read, %zu written, %.3f ms (%.0f GB/s)\n",
              cbytes, cbytes, ms_copy, 2.0 * cbytes / (ms_copy * 1e-3) / 1e9);
  // streaming read of 4 GiB (the two buffers twice), best of three
  CHECK(hipFree(cdst));
  const size_t rbytes = (size_t)4 << 30;
  float* rbuf = nullptr;
  float* rout = nullptr;
  CHECK(hipMalloc(&rbuf, rbytes));
  CHECK(hipMemsetAsync(rbuf, 0, rbytes, st));
  const unsigned rgrid = 256 * 16;
  CHECK(hipMalloc(&rout, (size_t)rgrid * 256 * sizeof(float)));
  float best = 0.f;
  for (int r = 0; r < 3; ++r) {
    CHECK(hipEventRecord(e0, st));
    hipLaunchKernelGGL(calib_read, dim3(rgrid), dim3(256), 0, st, (const float4*)rbuf, rbytes / 16,
                       rout);
    CHECK(hipEventRecord(e1, st));
    CHECK(hipStreamSynchronize(st));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (r == 0 || ms < best) best = ms;
  }
  std::printf("[native] streaming read: %zu bytes, %.3f ms (%.0f GB/s)\n", rbytes, best,
              rbytes / (best * 1e-3) / 1e9);
  CHECK(hipFree(rbuf));
  CHECK(hipFree(rout));
  CHECK(hipFree(csrc));
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  return 0;
}

static int run_format(int64_t m, int64_t n, int64_t b, int64_t kmax, int iters, int fmt,
                      hipStream_t st);

int main(int argc, char** argv) {
  std::setvbuf(stdout, nullptr, _IOLBF, 0);  // each line reaches the log at once
  const int64_t m = argc > 1 ? atoll(argv[1]) : 50000;
  const int64_t n = argc > 2 ? atoll(argv[2]) : 20000;
  const int64_t b = argc > 3 ? atoll(argv[3]) : 64;
  const int64_t kmax = argc > 4 ? atoll(argv[4]) : 2048;
  const int iters = argc > 5 ? atoi(argv[5]) : 3;
  const int fmt = argc > 6 ? atoi(argv[6]) : 0;
  const bool libs = argc > 7 && std::strcmp(argv[7], "libs") == 0;
  if (fmt < 0 || fmt > 3) return 5;
  hipStream_t st;
  CHECK(hipStreamCreate(&st));
  if (calibrate(st) != 0) return 1;
  for (int f = (fmt == 3 ? 0 : fmt); f <= (fmt == 3 ? 2 : fmt); ++f) {
    const int rc = run_format(m, n, b, kmax, iters, f, st);
    if (rc != 0) return rc;
  }
  CHECK(hipStreamSynchronize(st));
  CHECK(hipStreamDestroy(st));
  if (rid_release() != RID_OK) return 5;
  if (libs) dl_iterate_phdr(print_segments, nullptr);
  std::printf("[native] done\n");
  return 0;
}

static int run_format(int64_t m, int64_t n, int64_t b, int64_t kmax, int iters, int fmt,
                      hipStream_t st) {
  std::printf("[native] format %d (%s)\n", fmt, fmt == 0 ? "fp32" : fmt == 1 ? "bf16" : "fp8-e4m3");

  float* A = nullptr;
  CHECK(hipMalloc(&A, (size_t)m * n * sizeof(float)));
  if (rid_debug_gaussian(7, 0, m, n, RID_F32, A, st) != RID_OK) return 2;
  rid_config cfg{RID_F32, 1, 1, RID_F32, nullptr, 0};
  void* Aop = A;  // the matrix the calls read
  float* scale = nullptr;
  if (fmt != 0) {
    const size_t count = (size_t)m * n;
    unsigned char* Aq = nullptr;
    CHECK(hipMalloc(&Aq, count * (fmt == 1 ? 2 : 1)));
    hipLaunchKernelGGL(to_format, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, A, Aq,
                       count, fmt);
    const size_t ntile = (size_t)((n + 127) / 128);
    CHECK(hipMalloc(&scale, ntile * sizeof(float)));
    hipLaunchKernelGGL(fill_ones, dim3((unsigned)((ntile + 255) / 256)), dim3(256), 0, st, scale,
                       ntile);
    CHECK(hipStreamSynchronize(st));
    CHECK(hipFree(A));
    A = nullptr;
    Aop = Aq;
    cfg.a_type = fmt == 1 ? RID_BF16 : RID_FP8_E4M3;
    cfg.a_col_scale = fmt == 2 ? scale : nullptr;
  }
  const int64_t kcap = std::min<int64_t>(kmax, std::min(m, n));
  const size_t wb = rid_workspace_bytes(m, n, kmax, b, &cfg);
  void* work = nullptr;
  CHECK(hipMalloc(&work, wb));
  float *Yt = nullptr, *T = nullptr;
  int64_t* J = nullptr;
  int32_t *ko = nullptr, *so = nullptr;
  double* eo = nullptr;
  CHECK(hipMalloc(&Yt, (size_t)n * b * sizeof(float)));
  CHECK(hipMalloc(&T, (size_t)kcap * n * sizeof(float)));
  CHECK(hipMalloc(&J, (size_t)kcap * sizeof(int64_t)));
  CHECK(hipMalloc(&ko, 4));
  CHECK(hipMalloc(&so, 4));
  CHECK(hipMalloc(&eo, 8));
  const size_t wbs = rid_workspace_bytes(m, n, b, b, &cfg);
  void* works = nullptr;
  CHECK(hipMalloc(&works, wbs));

  for (int it = 0; it < iters; ++it) {
    auto t0 = std::chrono::steady_clock::now();
    if (rid_debug_sketch(Aop, m, n, n, b, b, &cfg, Yt, b, works, wbs, st) != RID_OK) return 3;
    CHECK(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    if (rid_lupp_adaptive(Aop, m, n, n, b, 1e-6, kmax, &cfg, J, T, n, ko, eo, so, work, wb, st) !=
        RID_OK)
      return 4;
    CHECK(hipStreamSynchronize(st));
    auto t2 = std::chrono::steady_clock::now();
    int32_t k = 0, s = 0;
    double e = 0;
    CHECK(hipMemcpy(&k, ko, 4, hipMemcpyDeviceToHost));
    CHECK(hipMemcpy(&s, so, 4, hipMemcpyDeviceToHost));
    CHECK(hipMemcpy(&e, eo, 8, hipMemcpyDeviceToHost));
    std::printf("[native] iter %d: sketch block %.3f ms, adaptive %.3f ms, k=%d status=%s E=%.3e\n",
                it, std::chrono::duration<double, std::milli>(t1 - t0).count(),
                std::chrono::duration<double, std::milli>(t2 - t1).count(), k,
                rid_status_string(s), e);
  }
  CHECK(hipFree(Aop));
  if (scale) CHECK(hipFree(scale));
  CHECK(hipFree(work));
  CHECK(hipFree(works));
  CHECK(hipFree(Yt));
  CHECK(hipFree(T));
  CHECK(hipFree(J));
  CHECK(hipFree(ko));
  CHECK(hipFree(so));
  CHECK(hipFree(eo));
  CHECK(hipStreamSynchronize(st));
  return 0;
}
