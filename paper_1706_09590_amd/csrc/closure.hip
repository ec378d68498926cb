// Learned hierarchy terminator: a linear convolution closure that predicts
// the truncated level W^(N+1) from W^(N) and replaces Eq. (GMFP) at n = N
// (two states).  The closure is a three-layer 5x5 convolution network over
// (q, p) without biases or activations (the hierarchy is linear, so is the
// closure); its input channels are the four packed components of W^(N) and
// the same four multiplied by p (the analytic terminator (zeta p + c0 d/dp)
// W^(N) is one such map).  The three layers compose exactly into one 13x13
// kernel, which is what the propagation applies.
//
//  - closure_apply_kernel: inference, BF16 inputs and weights on MFMA
//    (v_mfma_f32_16x16x16_bf16), FP32 accumulation;
//  - closure_stats_kernel: FP64 second-moment statistics of training pairs
//    (level n, level n + 1) of a propagated hierarchy;
//  - kernel-stack convolutions / correlations and Adam: gradient descent on
//    the three layers against the quadratic loss the statistics define.
#include <cstdint>

#include "device_common.hpp"
#include "qhfpe_internal.hpp"

namespace qhfpe {

namespace {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short to_bf16(float x) {
  const unsigned u = __builtin_bit_cast(unsigned, x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------------------
// Inference
// ---------------------------------------------------------------------------
// One task: 4 output q rows of one member over all p.  The 16 input rows
// (q0 - 6 .. q0 + 9) are staged in LDS as BF16, channel-last [row][p][8].
// MFMA tile: M = 16 consecutive p, N = 16 = 4 output rows x 4 components,
// K = 16 taps (dp, ci) of one input row: 13 dp x 8 ci = 104 taps in 7
// chunks per row, 16 rows.  The weights, already in this B layout
// [row][chunk][n][k] (closure_weights_kernel), are held in registers, each
// wave holding those of half the input rows.
constexpr int kRowsOut = 4;
constexpr int kRowsIn = kRowsOut + 2 * kClosureHalf;   // 16
constexpr int kChunks = 7;
constexpr int kTaps = (2 * kClosureHalf + 1) * kClosureIn;  // 104 per input row
// Eight waves: wave w takes the tile pairs w % 4 (+ 4 k) over the input rows
// (w / 4) * 8 .. + 7, holding those rows' weights in registers; the two
// halves of each sum meet in LDS.
constexpr int kApplyWaves = 8;
constexpr int kRowHalves = 2;
constexpr int kRowsPerWave = kRowsIn / kRowHalves;  // 8
constexpr int kTilesAtOnce = 2;  // tiles per wave at once
constexpr int kChains = 2;       // accumulators per tile (even and odd input rows): 4 independent MFMA chains
constexpr int kApplyThreads = 64 * kApplyWaves;

// The channels of one grid point as 8 BF16 values (16 bytes).
template <typename T>
__device__ __forceinline__ uint4 pack_channels(const float c[4], float pa) {
  unsigned short h[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h[k] = to_bf16(c[k]);
    h[4 + k] = to_bf16(pa * c[k]);
  }
  uint4 w4;
  w4.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
  w4.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
  w4.z = (unsigned)h[4] | ((unsigned)h[5] << 16);
  w4.w = (unsigned)h[6] | ((unsigned)h[7] << 16);
  return w4;
}

// Each workgroup walks a contiguous range of tasks in (member, q group)
// order.  The 16 input rows live in a ring of LDS row slots (row q in slot
// (q + 6) mod 16): the next group of the same member needs 4 new rows only,
// which are loaded into registers while the current group runs on the
// matrix cores, and written to the slots the current group no longer reads.
template <typename T, int NP>
__global__ void __launch_bounds__(kApplyThreads, 1)
    closure_apply_kernel(const T* __restrict__ v, int level, long long member_stride, long long level_stride,
                         long long comp_stride, int nq, int batch, double p0, double dp,
                         const unsigned short* __restrict__ wb, T* __restrict__ out, long long out_stride) {
  __shared__ __align__(16) unsigned short sx[kRowsIn * NP * kClosureIn];
  __shared__ f32x4_t sred[kApplyWaves / kRowHalves][kTilesAtOnce][64];  // second-half partial sums
  constexpr int kNewPer = kRowsOut * NP / kApplyThreads;  // new-row points per thread (1 or 2)
  static_assert(kRowsOut * NP % kApplyThreads == 0, "new rows split evenly over the threads");
  const int tid = threadIdx.x;
  const int groups = (nq + kRowsOut - 1) / kRowsOut;
  const long long ntasks = (long long)groups * batch;
  const long long per = (ntasks + gridDim.x - 1) / gridDim.x;
  const long long t_begin = (long long)blockIdx.x * per;
  const long long t_end = t_begin + per < ntasks ? t_begin + per : ntasks;
  const int lane = tid & 63, wid = tid >> 6;
  const int quad = lane >> 4, li = lane & 15;
  // the B fragments of this wave's input rows stay in its registers: they
  // are the same for every tile and task
  const int tg = wid % (kApplyWaves / kRowHalves), half = wid / (kApplyWaves / kRowHalves);
  bf16x4_t bw[kRowsPerWave][kChunks];
#pragma unroll
  for (int rr = 0; rr < kRowsPerWave; ++rr)
#pragma unroll
    for (int ch = 0; ch < kChunks; ++ch) {
      const int row = half * kRowsPerWave + rr;
      bw[rr][ch] = *reinterpret_cast<const bf16x4_t*>(wb + (((row * kChunks + ch) * 16 + li) * 16 + 4 * quad));
    }
  auto load_point = [&](const T* vb, int q, int a, float c[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = 0.f;
    if (q >= 0 && q < nq) {
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = (float)vb[k * comp_stride + (long long)q * NP + a];
    }
  };
  auto slot = [](int q) { return (q + kClosureHalf + kRowsIn) % kRowsIn; };
  float nxt[kNewPer][4];  // the next group's new rows, in flight during the MFMA phase
  bool have_next = false;
  for (long long task = t_begin; task < t_end; ++task) {
    const int b = (int)(task / groups), g = (int)(task % groups);
    const int q0 = g * kRowsOut;
    const T* vb = v + (long long)b * member_stride + (long long)level * level_stride;
    __syncthreads();  // the previous group's MFMA reads of sx are done
    if (!have_next) {
      // first group of a member in this range: all 16 rows
      for (int e = tid; e < kRowsIn * NP; e += kApplyThreads) {
        const int r = e / NP, a = e % NP;
        const int q = q0 - kClosureHalf + r;
        float c[4];
        load_point(vb, q, a, c);
        reinterpret_cast<uint4*>(sx)[slot(q) * NP + a] = pack_channels<T>(c, (float)(p0 + a * dp));
      }
    } else {
      // rows q0 + 6 .. q0 + 9 arrived during the previous group
#pragma unroll
      for (int j = 0; j < kNewPer; ++j) {
        const int e = tid + j * kApplyThreads;
        const int r = e / NP, a = e % NP;
        const int q = q0 + kClosureHalf + r;
        reinterpret_cast<uint4*>(sx)[slot(q) * NP + a] = pack_channels<T>(nxt[j], (float)(p0 + a * dp));
      }
    }
    __syncthreads();
    // the next group's new rows, if it is the same member's
    have_next = task + 1 < t_end && g + 1 < groups;
    if (have_next) {
#pragma unroll
      for (int j = 0; j < kNewPer; ++j) {
        const int e = tid + j * kApplyThreads;
        const int r = e / NP, a = e % NP;
        load_point(vb, q0 + kRowsOut + kClosureHalf + r, a, nxt[j]);
      }
    }
    constexpr int kGroups = kApplyWaves / kRowHalves;
    for (int t0 = tg * kTilesAtOnce; t0 < NP / 16; t0 += kGroups * kTilesAtOnce) {
      f32x4_t acc[kTilesAtOnce][kChains];
#pragma unroll
      for (int u = 0; u < kTilesAtOnce; ++u)
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[u][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int rr = 0; rr < kRowsPerWave; ++rr) {
        const int row = half * kRowsPerWave + rr;
        const unsigned short* xr = sx + slot(q0 - kClosureHalf + row) * NP * kClosureIn;
#pragma unroll
        for (int ch = 0; ch < kChunks; ++ch) {
          // A: lane holds taps k = 4 quad .. 4 quad + 3 of output p = 16 tile + li
          const int kk = ch * 16 + 4 * quad;
#pragma unroll
          for (int u = 0; u < kTilesAtOnce; ++u) {
            bf16x4_t av = {0, 0, 0, 0};
            if (kk < kTaps) {
              const int dpo = kk / kClosureIn, ci0 = kk % kClosureIn;
              const int pin = (16 * (t0 + u) + li + dpo - kClosureHalf + NP) % NP;
              av = *reinterpret_cast<const bf16x4_t*>(xr + pin * kClosureIn + ci0);
            }
            // B (registers): taps k = 4 quad .. 4 quad + 3 of output n = li
            acc[u][rr % kChains] =
                __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bw[rr][ch], acc[u][rr % kChains], 0, 0, 0);
          }
        }
      }
      // the second row half hands its partial sums to the first
      if (half == 1) {
#pragma unroll
        for (int u = 0; u < kTilesAtOnce; ++u) sred[tg][u][lane] = acc[u][0] + acc[u][1];
      }
      __syncthreads();
      if (half == 0) {
        // D: lane holds rows i = 4 quad .. 4 quad + 3 (p) of column n = li
        const int r = li >> 2, co = li & 3;
        const int q = q0 + r;
        if (q < nq) {
#pragma unroll
          for (int u = 0; u < kTilesAtOnce; ++u) {
            const f32x4_t sum = acc[u][0] + acc[u][1] + sred[tg][u][lane];
            T* o = out + (long long)b * out_stride + co * comp_stride + (long long)q * NP + 16 * (t0 + u) + 4 * quad;
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = (T)sum[j];
          }
        }
      }
      __syncthreads();  // sred is free again
    }
  }
}

// The 13x13 closure kernel K[dq][dp][ci][co] (FP32) in the B layout of
// closure_apply_kernel: wb[row][chunk][n][k] = K[row - n/4][kk/8][kk%8][n%4]
// with kk = 16 chunk + k, zero outside the kernel.
__global__ void closure_weights_kernel(const float* __restrict__ K, unsigned short* __restrict__ wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kClosureWeightElems) return;
  const int k = e % 16, n = (e / 16) % 16, ch = (e / 256) % kChunks, row = e / (256 * kChunks);
  const int kk = ch * 16 + k;
  const int r = n >> 2, co = n & 3, dq = row - r;
  float w = 0.f;
  if (kk < kTaps && dq >= 0 && dq <= 2 * kClosureHalf) {
    const int dpo = kk / kClosureIn, ci = kk % kClosureIn;
    w = K[((dq * (2 * kClosureHalf + 1) + dpo) * kClosureIn + ci) * kClosureOut + co];
  }
  wb[e] = to_bf16(w);
}

// ---------------------------------------------------------------------------
// Training statistics (FP64)
// ---------------------------------------------------------------------------
// Blocks 0..199: A[dq][.][ci][.] for dq = 0..24 (offset dq - 12), ci = 0..7;
// blocks 200..303: C[dq][.][ci][.] for dq = 0..12 (offset dq - 6);
// block 304: yy.  Each output belongs to one thread, which adds the sum over
// every member and grid row into stats (so repeated calls accumulate).
constexpr int kStatBlocksA = (4 * kClosureHalf + 1) * kClosureIn;
constexpr int kStatBlocksC = (2 * kClosureHalf + 1) * kClosureIn;
constexpr int kStatThreads = 256;

template <typename T, int NP>
__device__ __forceinline__ double channel(const T* lv, long long comp_stride, int c, int q, int a, double pa) {
  const double x = (double)lv[(c & 3) * comp_stride + (long long)q * NP + a];
  return c < 4 ? x : pa * x;
}

template <typename T, int NP>
__global__ void __launch_bounds__(kStatThreads)
    closure_stats_kernel(const T* __restrict__ v, int level, long long member_stride, long long level_stride,
                         long long comp_stride, int nq, int batch, double p0, double dp,
                         double* __restrict__ stats) {
  __shared__ double s1[NP];
  __shared__ double s2[kClosureIn * NP];
  const int tid = threadIdx.x;
  const int blk = blockIdx.x;
  constexpr int H2 = 2 * kClosureHalf, NA = 2 * H2 + 1, NCK = 2 * kClosureHalf + 1;
  double acc = 0.0;
  if (blk < kStatBlocksA) {
    const int dq = blk / kClosureIn, ci = blk % kClosureIn;
    const int dpo = tid / kClosureIn, cj = tid % kClosureIn;  // tid < 200
    for (int b = 0; b < batch; ++b) {
      const T* lv = v + (long long)b * member_stride + (long long)level * level_stride;
      for (int q = 0; q < nq; ++q) {
        const int q2 = q + dq - H2;
        if (q2 < 0 || q2 >= nq) continue;
        __syncthreads();
        for (int a = tid; a < NP; a += kStatThreads) s1[a] = channel<T, NP>(lv, comp_stride, ci, q, a, p0 + a * dp);
        for (int e = tid; e < kClosureIn * NP; e += kStatThreads) {
          const int c = e / NP, a = e % NP;
          s2[e] = channel<T, NP>(lv, comp_stride, c, q2, a, p0 + a * dp);
        }
        __syncthreads();
        if (tid < NA * kClosureIn) {
          const double* x2 = s2 + cj * NP;
          for (int a = 0; a < NP; ++a) acc += s1[a] * x2[(a + dpo - H2 + NP) % NP];
        }
      }
    }
    if (tid < NA * kClosureIn) stats[((dq * NA + dpo) * kClosureIn + ci) * kClosureIn + cj] += acc;
  } else if (blk < kStatBlocksA + kStatBlocksC) {
    const int e0 = blk - kStatBlocksA;
    const int dq = e0 / kClosureIn, ci = e0 % kClosureIn;
    const int dpo = tid / kClosureOut, co = tid % kClosureOut;  // tid < 52
    for (int b = 0; b < batch; ++b) {
      const T* lv = v + (long long)b * member_stride + (long long)level * level_stride;
      const T* ly = lv + level_stride;
      for (int q = 0; q < nq; ++q) {
        const int q2 = q + dq - kClosureHalf;
        if (q2 < 0 || q2 >= nq) continue;
        __syncthreads();
        for (int a = tid; a < NP; a += kStatThreads) s1[a] = channel<T, NP>(lv, comp_stride, ci, q2, a, p0 + a * dp);
        for (int e = tid; e < kClosureOut * NP; e += kStatThreads) {
          const int c = e / NP, a = e % NP;
          s2[e] = (double)ly[c * comp_stride + (long long)q * NP + a];
        }
        __syncthreads();
        if (tid < NCK * kClosureOut) {
          const double* y = s2 + co * NP;
          for (int a = 0; a < NP; ++a) acc += s1[(a + dpo - kClosureHalf + NP) % NP] * y[a];
        }
      }
    }
    if (tid < NCK * kClosureOut)
      stats[kClosureStatsA + ((dq * NCK + dpo) * kClosureIn + ci) * kClosureOut + co] += acc;
  } else {
    __shared__ double red[kStatThreads / 64];
    for (int b = 0; b < batch; ++b) {
      const T* ly = v + (long long)b * member_stride + (long long)(level + 1) * level_stride;
      for (long long e = tid; e < (long long)kClosureOut * nq * NP; e += kStatThreads) {
        const int c = (int)(e / ((long long)nq * NP));
        const long long r = e % ((long long)nq * NP);
        const double y = (double)ly[c * comp_stride + r];
        acc += y * y;
      }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kStatThreads / 64; ++w) s += red[w];
      stats[kClosureStatsA + kClosureStatsC] += s;
    }
  }
}

// ---------------------------------------------------------------------------
// Training: kernel stacks P[i][a][b] with a 2-D tap index i over an s x s
// square (offsets centred), composed and differentiated exactly.
// ---------------------------------------------------------------------------
// out[k][a][c] = sum_{i + j = k} sum_b P[i][a][b] Q[j][b][c]   (full convolution)
__global__ void stack_convolve_kernel(const float* __restrict__ P, int sp, const float* __restrict__ Q, int sq,
                                      int na, int nb, int nc, float* __restrict__ out) {
  const int so = sp + sq - 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= so * so * na * nc) return;
  const int c = e % nc, a = (e / nc) % na, k = e / (nc * na);
  const int kq = k / so, kp = k % so;
  double acc = 0.0;
  for (int iq = max(0, kq - sq + 1); iq <= min(sp - 1, kq); ++iq)
    for (int ip = max(0, kp - sq + 1); ip <= min(sp - 1, kp); ++ip) {
      const float* pr = P + ((iq * sp + ip) * na + a) * nb;
      const float* qr = Q + (((kq - iq) * sq + (kp - ip)) * nb) * nc + c;
      for (int b = 0; b < nb; ++b) acc += (double)pr[b] * (double)qr[b * nc];
    }
  out[e] = (float)acc;
}

// out[i][a][b] = sum_j sum_c G[i + j][a][c] Q[j][b][c]   (sizes sg, sq -> sg - sq + 1)
__global__ void stack_correlate_left_kernel(const float* __restrict__ G, int sg, const float* __restrict__ Q, int sq,
                                            int na, int nb, int nc, float* __restrict__ out) {
  const int so = sg - sq + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= so * so * na * nb) return;
  const int b = e % nb, a = (e / nb) % na, i = e / (nb * na);
  const int iq = i / so, ip = i % so;
  double acc = 0.0;
  for (int jq = 0; jq < sq; ++jq)
    for (int jp = 0; jp < sq; ++jp) {
      const float* gr = G + (((iq + jq) * sg + (ip + jp)) * na + a) * nc;
      const float* qr = Q + ((jq * sq + jp) * nb + b) * nc;
      for (int c = 0; c < nc; ++c) acc += (double)gr[c] * (double)qr[c];
    }
  out[e] = (float)acc;
}

// out[j][b][c] = sum_i sum_a P[i][a][b] G[i + j][a][c]   (sizes sp, sg -> sg - sp + 1)
__global__ void stack_correlate_right_kernel(const float* __restrict__ P, int sp, const float* __restrict__ G, int sg,
                                             int na, int nb, int nc, float* __restrict__ out) {
  const int so = sg - sp + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= so * so * nb * nc) return;
  const int c = e % nc, b = (e / nc) % nb, j = e / (nc * nb);
  const int jq = j / so, jp = j % so;
  double acc = 0.0;
  for (int iq = 0; iq < sp; ++iq)
    for (int ip = 0; ip < sp; ++ip) {
      const float* pr = P + ((iq * sp + ip) * na) * nb + b;
      const float* gr = G + (((iq + jq) * sg + (ip + jp)) * na) * nc + c;
      for (int a = 0; a < na; ++a) acc += (double)pr[a * nb] * (double)gr[a * nc];
    }
  out[e] = (float)acc;
}

// Gradient of the normalised loss L / yy with respect to the composite
// kernel K (13 x 13 taps):  g[k][ci][co] = 2 (sum_{k', cj} A[k' - k][ci][cj]
// K[k'][cj][co] - C[k][ci][co]) / yy, plus the ridge term 2 rho (K - K0)
// with rho = ridge * (mean zero-offset channel energy) / yy, and per-entry
// terms of the data loss K (R K - 2 C) / yy (summed by closure_loss_kernel).
__global__ void closure_grad_kernel(const double* __restrict__ stats, const float* __restrict__ K,
                                    const float* __restrict__ K0, double ridge, float* __restrict__ g,
                                    double* __restrict__ terms) {
  constexpr int NCK = 2 * kClosureHalf + 1, H2 = 2 * kClosureHalf, NA = 2 * H2 + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kClosureKernelElems) return;
  const int co = e % kClosureOut, ci = (e / kClosureOut) % kClosureIn, k = e / (kClosureOut * kClosureIn);
  const int kq = k / NCK, kp = k % NCK;
  const double yy = stats[kClosureStatsA + kClosureStatsC];
  const double* A = stats;
  const double* C = stats + kClosureStatsA;
  double rk = 0.0;
  for (int k2q = 0; k2q < NCK; ++k2q)
    for (int k2p = 0; k2p < NCK; ++k2p) {
      const double* ar = A + (((k2q - kq + H2) * NA + (k2p - kp + H2)) * kClosureIn + ci) * kClosureIn;
      const float* kr = K + ((k2q * NCK + k2p) * kClosureIn) * kClosureOut + co;
      for (int cj = 0; cj < kClosureIn; ++cj) rk += ar[cj] * (double)kr[cj * kClosureOut];
    }
  const double c = C[e];
  const double inv = yy > 0.0 ? 1.0 / yy : 0.0;
  double mean_diag = 0.0;
  for (int cc = 0; cc < kClosureIn; ++cc) mean_diag += A[((H2 * NA + H2) * kClosureIn + cc) * kClosureIn + cc];
  mean_diag /= kClosureIn;
  const double k0 = K0 ? (double)K0[e] : 0.0;
  g[e] = (float)(2.0 * (rk - c) * inv + 2.0 * ridge * mean_diag * inv * ((double)K[e] - k0));
  terms[e] = (double)K[e] * (rk - 2.0 * c) * inv;
}

// loss = 1 + sum(terms) (one block, fixed order)
__global__ void closure_loss_kernel(const double* __restrict__ terms, double* __restrict__ loss) {
  __shared__ double red[4];
  double s = 0.0;
  for (int e = threadIdx.x; e < kClosureKernelElems; e += 256) s += terms[e];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *loss = 1.0 + red[0] + red[1] + red[2] + red[3];
}

// Adam on n parameters: w -= lr mhat / (sqrt(vhat) + eps)
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ s, int n, float lr, float b1, float b2, float c1, float c2, float eps) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float si = b2 * s[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  s[e] = si;
  w[e] -= lr * (mi / c1) / (sqrtf(si / c2) + eps);
}

inline unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_closure_weights(const float* K, unsigned short* wb, hipStream_t s) {
  hipLaunchKernelGGL(closure_weights_kernel, dim3(blocks_for(kClosureWeightElems, 256)), dim3(256), 0, s, K, wb);
  return hipGetLastError();
}

template <typename T>
static hipError_t apply_np(int np, const T* v, int level, long long ms, long long ls, long long cs, int nq, int batch,
                           double p0, double dp, const unsigned short* wb, T* out, long long os, hipStream_t s) {
  // one workgroup per CU (its LDS holds the weights and the row ring); each
  // walks about the same number of (member, q group) tasks
  const int tasks = batch * ((nq + kRowsOut - 1) / kRowsOut);
  const unsigned grid = (unsigned)(tasks < 256 ? tasks : 256);
  if (np == 128)
    hipLaunchKernelGGL((closure_apply_kernel<T, 128>), dim3(grid), dim3(kApplyThreads), 0, s, v, level, ms, ls, cs,
                       nq, batch, p0, dp, wb, out, os);
  else if (np == 256)
    hipLaunchKernelGGL((closure_apply_kernel<T, 256>), dim3(grid), dim3(kApplyThreads), 0, s, v, level, ms, ls, cs,
                       nq, batch, p0, dp, wb, out, os);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_closure_apply(int precision, int np, const void* v, int level, long long member_stride,
                                long long level_stride, long long comp_stride, int nq, int batch, double p0,
                                double dp, const unsigned short* wb, void* out, long long out_stride, hipStream_t s) {
  if (precision == QHFPE_FP64)
    return apply_np<double>(np, static_cast<const double*>(v), level, member_stride, level_stride, comp_stride, nq,
                            batch, p0, dp, wb, static_cast<double*>(out), out_stride, s);
  return apply_np<float>(np, static_cast<const float*>(v), level, member_stride, level_stride, comp_stride, nq,
                         batch, p0, dp, wb, static_cast<float*>(out), out_stride, s);
}

template <typename T>
static hipError_t stats_np(int np, const T* v, int level, long long ms, long long ls, long long cs, int nq,
                           int batch, double p0, double dp, double* stats, hipStream_t s) {
  const dim3 grid(kStatBlocksA + kStatBlocksC + 1);
  if (np == 128)
    hipLaunchKernelGGL((closure_stats_kernel<T, 128>), grid, dim3(kStatThreads), 0, s, v, level, ms, ls, cs, nq,
                       batch, p0, dp, stats);
  else if (np == 256)
    hipLaunchKernelGGL((closure_stats_kernel<T, 256>), grid, dim3(kStatThreads), 0, s, v, level, ms, ls, cs, nq,
                       batch, p0, dp, stats);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_closure_stats(int precision, int np, const void* v, int level, long long member_stride,
                                long long level_stride, long long comp_stride, int nq, int batch, double p0,
                                double dp, double* stats, hipStream_t s) {
  if (precision == QHFPE_FP64)
    return stats_np<double>(np, static_cast<const double*>(v), level, member_stride, level_stride, comp_stride, nq,
                            batch, p0, dp, stats, s);
  return stats_np<float>(np, static_cast<const float*>(v), level, member_stride, level_stride, comp_stride, nq, batch,
                         p0, dp, stats, s);
}

// One gradient-descent (Adam) iteration on the three layers; see the layout
// of the training state in qhfpe_internal.hpp.  loss != nullptr: also the
// normalised loss of the weights before the update.
hipError_t launch_closure_train_step(const double* stats, const float* prior, double ridge, float* st, int t,
                                     float lr, double* loss, hipStream_t s) {
  using L = ClosureTrainLayout;
  float* W1 = st + L::w1;
  float* W2 = st + L::w2;
  float* W3 = st + L::w3;
  float* G1 = st + L::g1;
  float* G2 = st + L::g2;
  float* G3 = st + L::g3;
  float* W12 = st + L::w12;
  float* G12 = st + L::g12;
  float* K = st + L::k;
  float* GK = st + L::gk;
  double* terms = reinterpret_cast<double*>(st + L::terms);
  constexpr int CI = kClosureIn, M = kClosureHidden, CO = kClosureOut;
  // W12 = W1 * W2 (9 x 9, CI -> M);  K = W12 * W3 (13 x 13, CI -> CO)
  hipLaunchKernelGGL(stack_convolve_kernel, dim3(blocks_for(81 * CI * M, 256)), dim3(256), 0, s, W1, 5, W2, 5, CI, M,
                     M, W12);
  hipLaunchKernelGGL(stack_convolve_kernel, dim3(blocks_for(169 * CI * CO, 256)), dim3(256), 0, s, W12, 9, W3, 5, CI,
                     M, CO, K);
  hipLaunchKernelGGL(closure_grad_kernel, dim3(blocks_for(kClosureKernelElems, 256)), dim3(256), 0, s, stats, K, prior,
                     ridge, GK, terms);
  if (loss) hipLaunchKernelGGL(closure_loss_kernel, dim3(1), dim3(256), 0, s, terms, loss);
  // dW3 = corr_right(W12, g);  dW12 = corr_left(g, W3)
  hipLaunchKernelGGL(stack_correlate_right_kernel, dim3(blocks_for(25 * M * CO, 256)), dim3(256), 0, s, W12, 9, GK,
                     13, CI, M, CO, G3);
  hipLaunchKernelGGL(stack_correlate_left_kernel, dim3(blocks_for(81 * CI * M, 256)), dim3(256), 0, s, GK, 13, W3, 5,
                     CI, M, CO, G12);
  // dW1 = corr_left(dW12, W2);  dW2 = corr_right(W1, dW12)
  hipLaunchKernelGGL(stack_correlate_left_kernel, dim3(blocks_for(25 * CI * M, 256)), dim3(256), 0, s, G12, 9, W2, 5,
                     CI, M, M, G1);
  hipLaunchKernelGGL(stack_correlate_right_kernel, dim3(blocks_for(25 * M * M, 256)), dim3(256), 0, s, W1, 5, G12, 9,
                     CI, M, M, G2);
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(L::nparam, 256)), dim3(256), 0, s, st + L::w1, st + L::g1,
                     st + L::m, st + L::v, L::nparam, lr, b1, b2, c1, c2, 1e-12f);
  return hipGetLastError();
}

// The normalised data loss of a given composite kernel; terms: scratch of
// kClosureKernelElems doubles, g: scratch of kClosureKernelElems floats.
hipError_t launch_closure_loss(const double* stats, const float* K, float* g, double* terms, double* loss,
                               hipStream_t s) {
  hipLaunchKernelGGL(closure_grad_kernel, dim3(blocks_for(kClosureKernelElems, 256)), dim3(256), 0, s, stats, K,
                     nullptr, 0.0, g, terms);
  hipLaunchKernelGGL(closure_loss_kernel, dim3(1), dim3(256), 0, s, terms, loss);
  return hipGetLastError();
}

// The composite kernel of the current weights (and its loss, if asked).
hipError_t launch_closure_compose(const double* stats, float* st, double* loss, hipStream_t s) {
  using L = ClosureTrainLayout;
  constexpr int CI = kClosureIn, M = kClosureHidden, CO = kClosureOut;
  hipLaunchKernelGGL(stack_convolve_kernel, dim3(blocks_for(81 * CI * M, 256)), dim3(256), 0, s, st + L::w1, 5,
                     st + L::w2, 5, CI, M, M, st + L::w12);
  hipLaunchKernelGGL(stack_convolve_kernel, dim3(blocks_for(169 * CI * CO, 256)), dim3(256), 0, s, st + L::w12, 9,
                     st + L::w3, 5, CI, M, CO, st + L::k);
  if (loss) {
    double* terms = reinterpret_cast<double*>(st + L::terms);
    hipLaunchKernelGGL(closure_grad_kernel, dim3(blocks_for(kClosureKernelElems, 256)), dim3(256), 0, s, stats,
                       st + L::k, nullptr, 0.0, st + L::gk, terms);
    hipLaunchKernelGGL(closure_loss_kernel, dim3(1), dim3(256), 0, s, terms, loss);
  }
  return hipGetLastError();
}

}  // namespace qhfpe
