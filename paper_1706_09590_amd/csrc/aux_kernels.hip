// Pointwise and reduction kernels of the MS-QHFPE library: canonical <->
// packed conversion, dipole commutator, thermal initial state, level-0
// traces, norms and the spectral transforms of Sec. III.
#include <cmath>
#include <mutex>

#include "device_common.hpp"
#include "qhfpe_internal.hpp"

namespace qhfpe {

// Fixed device scratch of the allocation-free entry point (the t3 partial
// sums of the correlation spectrum): every GPU the library runs on holds its
// own copy until the process ends.  Host code never uses this name as an
// address: scratch_pointer() looks the device address up once per device.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_pointer(double** out) {
  static std::mutex mu;
  static double* ptr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = static_cast<double*>(p);
  }
  *out = ptr[dev];
  return hipSuccess;
}

namespace {

// Deterministic block sum / max of one double per thread (kBlock threads).
__device__ double block_sum(double x, double* sh) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) sh[tid >> 6] = x;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
  __syncthreads();
  return s;
}
__device__ double block_max(double x, double* sh) {
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) sh[tid >> 6] = x;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int w = 0; w < kBlock / 64; ++w) s = fmax(s, sh[w]);
  __syncthreads();
  return s;
}

// i^(-phase) * (re, im)
__device__ __forceinline__ cx<double> unphase(double re, double im, int phase) {
  switch (phase & 3) {
    case 0: return {re, im};
    case 1: return {im, -re};   // * (-i)
    case 2: return {-re, -im};
    default: return {-im, re};  // * i
  }
}
__device__ __forceinline__ cx<double> dophase(double re, double im, int phase) {
  return unphase(re, im, (4 - (phase & 3)) & 3);
}

// cells of one member: levels * nq * np
template <typename T, int NS>
__global__ void __launch_bounds__(kBlock)
    pack_kernel(GridDesc g, const double* __restrict__ canon, int phase, T* __restrict__ packed,
                int member_offset, double* red) {
  __shared__ double sh[kBlock / 64];
  constexpr int NC = NS * NS;
  const long long cells = (long long)g.levels * g.nq * g.np;
  const int b = blockIdx.y;
  const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dev = 0.0, mag = 0.0;
  if (cell < cells) {
    const long long gridn = (long long)g.nq * g.np;
    const int n = (int)(cell / gridn);
    const long long ia = cell % gridn;
    const double* src = canon + (long long)b * g.levels * NC * gridn * 2;
    cx<double> H[NS][NS];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const long long off = (((long long)(n * NS + j) * NS + k) * gridn + ia) * 2;
        H[j][k] = unphase(src[off], src[off + 1], phase);
        mag = fmax(mag, fabs(H[j][k].re) + fabs(H[j][k].im));
      }
    T* dst = packed + (long long)(member_offset + b) * g.member_stride + (long long)n * g.level_stride + ia;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      dev = fmax(dev, fabs(H[j][j].im));
      dst[j * g.comp_stride] = T(H[j][j].re);
#pragma unroll
      for (int k = j + 1; k < NS; ++k) {
        dev = fmax(dev, fabs(H[j][k].re - H[k][j].re) + fabs(H[j][k].im + H[k][j].im));
        const int c = Packing<NS>::re(j, k);
        dst[c * g.comp_stride] = T(0.5 * (H[j][k].re + H[k][j].re));
        dst[(c + 1) * g.comp_stride] = T(0.5 * (H[j][k].im - H[k][j].im));
      }
    }
  }
  const double d = block_max(dev, sh);
  const double m = block_max(mag, sh);
  if (threadIdx.x == 0) {
    const long long r = ((long long)b * gridDim.x + blockIdx.x) * 2;
    red[r] = d;
    red[r + 1] = m;
  }
}

template <typename T, int NS>
__global__ void __launch_bounds__(kBlock)
    unpack_kernel(GridDesc g, const T* __restrict__ packed, int phase, double* __restrict__ canon,
                  int member_offset) {
  constexpr int NC = NS * NS;
  const long long cells = (long long)g.levels * g.nq * g.np;
  const int b = blockIdx.y;
  const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (cell >= cells) return;
  const long long gridn = (long long)g.nq * g.np;
  const int n = (int)(cell / gridn);
  const long long ia = cell % gridn;
  const T* src = packed + (long long)(member_offset + b) * g.member_stride + (long long)n * g.level_stride + ia;
  T h[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) h[c] = src[c * g.comp_stride];
  double* dst = canon + (long long)b * g.levels * NC * gridn * 2;
#pragma unroll
  for (int j = 0; j < NS; ++j)
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const cx<T> e = herm_get<NS>(h, j, k);
      const cx<double> w = dophase((double)e.re, (double)e.im, phase);
      const long long off = (((long long)(n * NS + j) * NS + k) * gridn + ia) * 2;
      dst[off] = w.re;
      dst[off + 1] = w.im;
    }
}

// mu^x on packed H:  W = i^k H -> i^(k+1) H', H' = -i [mu, H]
template <typename T, int NS>
__global__ void __launch_bounds__(kBlock) dipole_kernel(GridDesc g, T* __restrict__ packed, DipoleMu mu) {
  constexpr int NC = NS * NS;
  const long long cells = (long long)g.levels * g.nq * g.np;
  const int b = blockIdx.y;
  const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (cell >= cells) return;
  const long long gridn = (long long)g.nq * g.np;
  const int n = (int)(cell / gridn);
  const long long ia = cell % gridn;
  T* p = packed + (long long)b * g.member_stride + (long long)n * g.level_stride + ia;
  T h[NC], o[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) h[c] = p[c * g.comp_stride];
  T A[NS][NS];
#pragma unroll
  for (int j = 0; j < NS; ++j)
#pragma unroll
    for (int k = 0; k < NS; ++k) A[j][k] = T(mu.m[j][k]);
  commutator_mi<NS, T>(A, h, o);
#pragma unroll
  for (int c = 0; c < NC; ++c) p[c * g.comp_stride] = o[c];
}

template <typename T, int NS>
__global__ void __launch_bounds__(kBlock)
    thermal_kernel(GridDesc g, T* __restrict__ packed, double q0, double dq, double p0, double dp,
                   const double* __restrict__ bath, double omega, double mass, double hbar,
                   const double* __restrict__ noise) {
  constexpr int NC = NS * NS;
  const long long gridn = (long long)g.nq * g.np;
  const long long cells = (long long)g.levels * gridn;
  const int b = blockIdx.y;
  const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (cell >= cells) return;
  const int n = (int)(cell / gridn);
  const long long ia = cell % gridn;
  T* p = packed + (long long)b * g.member_stride + (long long)n * g.level_stride + ia;
  double w = 0.0;
  if (n == 0) {
    // b = beta hbar omega / 2 with this member's beta
    const double tanh_b = tanh(0.5 * bath[kBathStride * b + 4] * hbar * omega);
    const int i = (int)(ia / g.np), a = (int)(ia % g.np);
    const double q = q0 + i * dq, pp = p0 + a * dp;
    w = (tanh_b / (M_PI * hbar)) *
        exp(-tanh_b * (pp * pp / (mass * hbar * omega) + mass * omega * q * q / hbar));
    if (noise) w += noise[ia];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) p[c * g.comp_stride] = T(c == 0 ? w : 0.0);
}

// Level-0 trace partials with the same tiling as the stage kernel.
template <typename T, int NS>
__global__ void __launch_bounds__(kBlock)
    trace_kernel(GridDesc g, const T* __restrict__ packed, DipoleMu mu, int tq, int ntiles,
                 double* __restrict__ partials, int slot) {
  __shared__ double sh[kBlock / 64];
  const int tile = blockIdx.x, b = blockIdx.y;
  const T* p = packed + (long long)b * g.member_stride;
  const int cells = tq * g.np;
  double tr = 0.0;
  for (int e = threadIdx.x; e < cells; e += kBlock) {
    const int q = tile * tq + e / g.np;
    if (q >= g.nq) continue;
    const long long ia = (long long)q * g.np + e % g.np;
#pragma unroll
    for (int j = 0; j < NS; ++j) tr += mu.m[j][j] * (double)p[j * g.comp_stride + ia];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int k = j + 1; k < NS; ++k)
        tr += 2.0 * mu.m[j][k] * (double)p[Packing<NS>::re(j, k) * g.comp_stride + ia];
  }
  const double s = block_sum(tr, sh);
  if (threadIdx.x == 0) partials[((long long)b * kRespSlots + slot) * ntiles + tile] = s;
}

__global__ void finalize_kernel(int batch, int ntiles, int nslots, const double* __restrict__ partials,
                                double scale, int phase, double* __restrict__ resp, long long resp_stride,
                                long long resp_offset, int* flag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (j >= nslots || b >= batch) return;
  const double* p = partials + ((long long)b * kRespSlots + j) * ntiles;
  double s = 0.0;
  for (int t = 0; t < ntiles; ++t) s += p[t];
  s *= scale;
  const cx<double> w = dophase(s, 0.0, phase);
  if (resp) {
    double* r = resp + (long long)b * resp_stride + (resp_offset + j) * 2;
    r[0] = w.re;
    r[1] = w.im;
  }
  if (!isfinite(s)) *flag = 1;
}

template <typename T, int NC>
__global__ void __launch_bounds__(kBlock)
    norm_kernel(GridDesc g, const T* __restrict__ packed, int ns, double* __restrict__ red) {
  __shared__ double sh[kBlock / 64];
  const long long gridn = (long long)g.nq * g.np;
  const long long cells = (long long)g.levels * gridn;
  const int b = blockIdx.y;
  double s = 0.0;
  for (long long cell = (long long)blockIdx.x * kBlock + threadIdx.x; cell < cells;
       cell += (long long)gridDim.x * kBlock) {
    const int n = (int)(cell / gridn);
    const long long ia = cell % gridn;
    const T* p = packed + (long long)b * g.member_stride + (long long)n * g.level_stride + ia;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double x = (double)p[c * g.comp_stride];
      // off-diagonal packed entries stand for two canonical entries
      s += (c < ns ? 1.0 : 2.0) * x * x;
    }
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) red[(long long)b * gridDim.x + blockIdx.x] = t;
}

__global__ void spectrum_abs_kernel(const double* __restrict__ series, long long n, double dt,
                                    const double* __restrict__ omega, int n_omega, double* __restrict__ out) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_omega) return;
  const double om = omega[w];
  double acc = 0.0;
  for (long long s = 0; s < n; ++s) {
    const double c = (s == 0 || s == n - 1) ? 0.5 : 1.0;
    double sn, cs;
    sincos(om * (double)s * dt, &sn, &cs);
    // Im(e^{i w t} R) = sin(wt) Re R + cos(wt) Im R
    acc += c * (sn * series[2 * s] + cs * series[2 * s + 1]);
  }
  out[w] = om * acc * dt;
}

// A[t1][w3] = sum_t3 c dt3 e^{i w3 t3} R3[t1][t3]
__global__ void spectrum_corr_t3_kernel(const double* __restrict__ r3, int n1, int n3, double dt3,
                                        const double* __restrict__ w3, int nw3, double* __restrict__ work) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int i1 = blockIdx.y;
  if (w >= nw3 || i1 >= n1) return;
  const double om = w3[w];
  const double* r = r3 + (long long)i1 * n3 * 2;
  double re = 0.0, im = 0.0;
  for (int s = 0; s < n3; ++s) {
    const double c = (s == 0 || s == n3 - 1) ? 0.5 : 1.0;
    double sn, cs;
    sincos(om * (double)s * dt3, &sn, &cs);
    re += c * (cs * r[2 * s] - sn * r[2 * s + 1]);
    im += c * (sn * r[2 * s] + cs * r[2 * s + 1]);
  }
  work[((long long)i1 * nw3 + w) * 2] = re * dt3;
  work[((long long)i1 * nw3 + w) * 2 + 1] = im * dt3;
}

// out[w3][w1] = sum_t1 c dt1 2 cos(w1 t1) Im A[t1][w3]
__global__ void spectrum_corr_t1_kernel(const double* __restrict__ work, int n1, double dt1,
                                        const double* __restrict__ w1, int nw1, int nw3, double* __restrict__ out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y;
  if (a >= nw1 || w >= nw3) return;
  const double om = w1[a];
  double acc = 0.0;
  for (int s = 0; s < n1; ++s) {
    const double c = (s == 0 || s == n1 - 1) ? 0.5 : 1.0;
    acc += c * 2.0 * cos(om * (double)s * dt1) * work[((long long)s * nw3 + w) * 2 + 1];
  }
  out[(long long)w * nw1 + a] = acc * dt1;
}

__global__ void clear_flag_kernel(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

// Streaming device copy: every lane moves kCopyUnroll 16-byte vectors, all
// loads issued before the first store, consecutive lanes on consecutive
// vectors (each load and store instruction of a wave covers 1 KiB).
constexpr int kCopyUnroll = 4;
__global__ void __launch_bounds__(kBlock)
    stream_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, long long n16) {
  const long long base = (long long)blockIdx.x * (kBlock * kCopyUnroll) + threadIdx.x;
  uint4 v[kCopyUnroll];
#pragma unroll
  for (int k = 0; k < kCopyUnroll; ++k) {
    const long long i = base + (long long)k * kBlock;
    if (i < n16) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < kCopyUnroll; ++k) {
    const long long i = base + (long long)k * kBlock;
    if (i < n16) dst[i] = v[k];
  }
}

// the bytes past the last whole 16-byte vector (fewer than 16)
__global__ void copy_tail_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int n) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = src[i];
}

inline dim3 cell_grid(const GridDesc& g, int nmembers) {
  const long long cells = (long long)g.levels * g.nq * g.np;
  return dim3((unsigned)((cells + kBlock - 1) / kBlock), (unsigned)nmembers);
}

}  // namespace

#define QHFPE_DISPATCH(g, F)                                  \
  do {                                                        \
    if ((g).precision == QHFPE_FP64) {                        \
      if ((g).ns == 2) { F(double, 2); } else { F(double, 3); } \
    } else {                                                  \
      if ((g).ns == 2) { F(float, 2); } else { F(float, 3); }   \
    }                                                         \
  } while (0)

hipError_t launch_pack(const GridDesc& g, const double* canon, int phase, void* packed, int member_offset,
                       int nmembers, double* red, int* nred_blocks, hipStream_t s) {
  const dim3 grid = cell_grid(g, nmembers);
  *nred_blocks = (int)grid.x;
#define F(T, NS) hipLaunchKernelGGL((pack_kernel<T, NS>), grid, dim3(kBlock), 0, s, g, canon, phase, \
                                    static_cast<T*>(packed), member_offset, red)
  QHFPE_DISPATCH(g, F);
#undef F
  return hipGetLastError();
}

hipError_t launch_unpack(const GridDesc& g, const void* packed, int phase, double* canon, int member_offset,
                         int nmembers, hipStream_t s) {
  const dim3 grid = cell_grid(g, nmembers);
#define F(T, NS) hipLaunchKernelGGL((unpack_kernel<T, NS>), grid, dim3(kBlock), 0, s, g, \
                                    static_cast<const T*>(packed), phase, canon, member_offset)
  QHFPE_DISPATCH(g, F);
#undef F
  return hipGetLastError();
}

hipError_t launch_dipole(const GridDesc& g, void* packed, const double mu[3][3], hipStream_t s) {
  const dim3 grid = cell_grid(g, g.batch);
  DipoleMu m;
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) m.m[j][k] = mu[j][k];
#define F(T, NS) hipLaunchKernelGGL((dipole_kernel<T, NS>), grid, dim3(kBlock), 0, s, g, static_cast<T*>(packed), m)
  QHFPE_DISPATCH(g, F);
#undef F
  return hipGetLastError();
}

hipError_t launch_thermal(const GridDesc& g, void* packed, double q0, double dq, double p0, double dp,
                          const double* bath, double omega, double mass, double hbar, const double* noise,
                          hipStream_t s) {
  const dim3 grid = cell_grid(g, g.batch);
#define F(T, NS) hipLaunchKernelGGL((thermal_kernel<T, NS>), grid, dim3(kBlock), 0, s, g, static_cast<T*>(packed), \
                                    q0, dq, p0, dp, bath, omega, mass, hbar, noise)
  QHFPE_DISPATCH(g, F);
#undef F
  return hipGetLastError();
}

hipError_t launch_trace_partials(const GridDesc& g, const void* packed, const double mu[3][3], int tq,
                                 int ntiles, double* partials, int slot, hipStream_t s) {
  DipoleMu m;
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) m.m[j][k] = mu[j][k];
  const dim3 grid(ntiles, g.batch);
#define F(T, NS) hipLaunchKernelGGL((trace_kernel<T, NS>), grid, dim3(kBlock), 0, s, g, \
                                    static_cast<const T*>(packed), m, tq, ntiles, partials, slot)
  QHFPE_DISPATCH(g, F);
#undef F
  return hipGetLastError();
}

hipError_t launch_finalize(int batch, int ntiles, int nslots, const double* partials, double scale, int phase,
                           double* resp, long long resp_stride, long long resp_offset, int* flag, hipStream_t s) {
  const dim3 grid((nslots + 63) / 64, batch);
  hipLaunchKernelGGL(finalize_kernel, grid, dim3(64), 0, s, batch, ntiles, nslots, partials, scale, phase, resp,
                     resp_stride, resp_offset, flag);
  return hipGetLastError();
}

hipError_t launch_norm_partials(const GridDesc& g, const void* packed, double* red, int* nblocks_per_member,
                                hipStream_t s) {
  const long long cells = (long long)g.levels * g.nq * g.np;
  int nb = (int)((cells + kBlock - 1) / kBlock);
  if (nb > 1024) nb = 1024;
  *nblocks_per_member = nb;
  const dim3 grid(nb, g.batch);
#define F(T, NS) hipLaunchKernelGGL((norm_kernel<T, NS * NS>), grid, dim3(kBlock), 0, s, g, \
                                    static_cast<const T*>(packed), NS, red)
  QHFPE_DISPATCH(g, F);
#undef F
  return hipGetLastError();
}

hipError_t launch_clear_flag(int* flag, hipStream_t s) {
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(64), 0, s, flag);
  return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16) return hipErrorInvalidValue;
  const long long n16 = (long long)(bytes / 16);
  const int tail = (int)(bytes % 16);
  if (n16 > 0) {
    const long long per_block = (long long)kBlock * kCopyUnroll;
    const long long blocks = (n16 + per_block - 1) / per_block;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (tail) {
    hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(64), 0, s, static_cast<const unsigned char*>(src) + 16 * n16,
                       static_cast<unsigned char*>(dst) + 16 * n16, tail);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_spectrum_abs(const double* series, long long n, double dt, const double* omega, int n_omega,
                               double* out, hipStream_t s) {
  hipLaunchKernelGGL(spectrum_abs_kernel, dim3((n_omega + 127) / 128), dim3(128), 0, s, series, n, dt, omega,
                     n_omega, out);
  return hipGetLastError();
}

hipError_t launch_spectrum_corr(const double* r3, int n1, int n3, double dt1, double dt3, const double* w1,
                                int nw1, const double* w3, int nw3, double* work, double* out, hipStream_t s) {
  hipLaunchKernelGGL(spectrum_corr_t3_kernel, dim3((nw3 + 127) / 128, n1), dim3(128), 0, s, r3, n1, n3, dt3, w3,
                     nw3, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(spectrum_corr_t1_kernel, dim3((nw1 + 127) / 128, nw3), dim3(128), 0, s, work, n1, dt1, w1,
                     nw1, nw3, out);
  return hipGetLastError();
}

}  // namespace qhfpe
