// Fused RK4 stage for the MS-QHFPE hierarchy:  out = y + coef * L v.
//
// L is the right-hand side of Eq. (heom) of Ikeda & Tanimura (2017) with one
// Drude exponential and V(q) = q, closed by Eq. (GMFP) at n = N:
//
//   L v^(n) = -(p/m) D_q v^(n)                         kinetic, 5th-order upwind (Sec. III)
//           + P v^(n)                                   potential term, Eq. (quantum-liouvillian)
//           - n gamma v^(n) + c_delta D_p2 v^(n)
//           + D_p v^(n+1)                               (n < N)
//           + D_p (zeta p v^(N) + c0 D_p v^(N))         (n = N, terminator)
//           + n gamma (zeta p v^(n-1) + c0 D_p v^(n-1)) (n >= 1)
//
// One workgroup owns one level n of one batch member on a tile of TQ whole
// p-columns.  The tile of v^(n) is staged in LDS.  The local terms are
// accumulated in registers first; the potential term then runs in place in
// LDS as a two-pass FFT along p (np = n1 * n2), a pointwise multiplication
// in the conjugate r-space, and the inverse two-pass FFT.  Diagonal
// potentials are r-dependent (U(q + r/2) - U(q - r/2)), so they go through
// the transform; two real diagonal components share one complex transform.
// The constant diabatic couplings are a pointwise commutator in p-space.
//
// State layout (packed reals): [member][level][comp][q][p], p fastest.
#pragma once

#include "device_common.hpp"
#include "qhfpe_internal.hpp"

namespace qhfpe {

template <int NP>
struct PlanOf;
#define QHFPE_PLAN(NP_, N1_, N2_, TQ_)                 \
  template <>                                          \
  struct PlanOf<NP_> {                                 \
    static constexpr int N1 = N1_, N2 = N2_, TQ = TQ_; \
  };
QHFPE_PLAN(8, 4, 2, 16)
QHFPE_PLAN(12, 4, 3, 16)
QHFPE_PLAN(16, 4, 4, 16)
QHFPE_PLAN(24, 6, 4, 16)
QHFPE_PLAN(32, 8, 4, 16)
QHFPE_PLAN(48, 8, 6, 16)
QHFPE_PLAN(64, 8, 8, 16)
QHFPE_PLAN(96, 12, 8, 8)
QHFPE_PLAN(128, 16, 8, 8)
QHFPE_PLAN(192, 16, 12, 4)
QHFPE_PLAN(256, 16, 16, 4)
#undef QHFPE_PLAN

// Upwind coefficients (x60) for p >= 0 on offsets -3..2; the p < 0 stencil
// is the mirror image with opposite sign (Sec. III).
__device__ constexpr double kUpwind[6] = {-2.0, 15.0, -60.0, 20.0, 30.0, -3.0};

template <typename T, int NS>
__device__ __forceinline__ T poly_eval(const double (&c)[QHFPE_MAX_STATES][5], int j, T x) {
  T r = T(c[j][4]);
  r = r * x + T(c[j][3]);
  r = r * x + T(c[j][2]);
  r = r * x + T(c[j][1]);
  r = r * x + T(c[j][0]);
  return r;
}

template <typename T>
__device__ __forceinline__ T clampT(T x, T lo, T hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

template <typename T, int NS, int NP>
__global__ void __launch_bounds__(kBlock) stage_kernel(StageArgs a) {
  using P = PlanOf<NP>;
  constexpr int N1 = P::N1, N2 = P::N2, TQ = P::TQ;
  constexpr int NC = NS * NS;
  constexpr int NPAIR = NS * (NS - 1) / 2;
  // complex transforms per tile: diagonal pairs (0,1) per column, (2 of c,
  // 2 of c+1) per column pair when NS = 3, and each off-diagonal pair.
  constexpr int NFFT = TQ + (NS == 3 ? TQ / 2 : 0) + NPAIR * TQ;
  constexpr int CELLS = TQ * NP;
  constexpr int CPT = (CELLS + kBlock - 1) / kBlock;
  static_assert(NS == 2 || TQ % 2 == 0, "three-state tiles pair columns");

  __shared__ T sv[TQ * NC * NP];
  __shared__ cx<T> stw[NP];

  const int tid = threadIdx.x;
  const int bid = blockIdx.x;
  const int tile = bid % a.ntiles;
  const int rest = bid / a.ntiles;
  const int L = a.depth + 1;
  const int n = rest % L;
  const int b = rest / L;
  const int q0 = tile * TQ;
  const int nq = a.nq;

  const T* __restrict__ v = static_cast<const T*>(a.v) + (long long)b * a.member_stride;
  const T* __restrict__ vn = v + (long long)n * a.level_stride;
  const long long cs = a.comp_stride;

  // ---- P0: twiddles and the v^(n) tile into LDS -------------------------
  for (int j = tid; j < NP; j += kBlock) stw[j] = static_cast<const cx<T>*>(a.twiddle)[j];
  for (int e = tid; e < TQ * NC * NP; e += kBlock) {
    const int c = e / (NC * NP);
    const int comp = (e / NP) % NC;
    const int ia = e % NP;
    const int q = q0 + c;
    sv[e] = (q < nq) ? vn[comp * cs + (long long)q * NP + ia] : T(0);
  }
  __syncthreads();

  // ---- P1: local terms into registers -----------------------------------
  const T dqinv = T(1.0 / (60.0 * a.dq));
  const T dpinv = T(1.0 / (12.0 * a.dp));
  const T dp2inv = T(1.0 / (12.0 * a.dp * a.dp));
  const T dpdpinv = T(1.0 / (144.0 * a.dp * a.dp));
  const T zeta = T(a.zeta), c0 = T(a.c0), cdel = T(a.cdelta);
  const T ng = T(n * a.gamma);
  const T inv_mass = T(a.inv_mass);
  T coup[NS][NS];
#pragma unroll
  for (int j = 0; j < NS; ++j)
#pragma unroll
    for (int k = 0; k < NS; ++k) coup[j][k] = T(a.coup[j][k]);

  T acc[CPT][NC];
#pragma unroll
  for (int t = 0; t < CPT; ++t) {
    const int e = tid + t * kBlock;
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) acc[t][comp] = T(0);
    if (e >= CELLS) continue;
    const int c = e / NP;
    const int ia = e % NP;
    const int q = q0 + c;
    if (q >= nq) continue;
    const T p = T(a.p0 + ia * a.dp);
    const int sgn = (p >= T(0)) ? 1 : -1;
    const int am1 = (ia + NP - 1) % NP, am2 = (ia + NP - 2) % NP;
    const int ap1 = (ia + 1) % NP, ap2 = (ia + 2) % NP;
    const T* svc = sv + c * NC * NP;
    T hv[NC];
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) {
      const T* s = svc + comp * NP;
      const T w0 = s[ia];
      hv[comp] = w0;
      // kinetic: -(p/m) sgn sum_d c_d v(q + sgn d)
      T dq_acc = T(0);
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        const int off = sgn * (d - 3);
        const int cc = c + off;
        const int qq = q + off;
        T val;
        if (cc >= 0 && cc < TQ) {
          val = sv[(cc * NC + comp) * NP + ia];
        } else {
          val = (qq >= 0 && qq < nq) ? vn[comp * cs + (long long)qq * NP + ia] : T(0);
        }
        dq_acc += T(kUpwind[d]) * val;
      }
      T f = -(p * inv_mass) * T(sgn) * dqinv * dq_acc;
      // damping and the delta-correlated (low-temperature) correction
      f += -ng * w0;
      f += cdel * dp2inv * (-s[ap2] + T(16) * s[ap1] - T(30) * w0 + T(16) * s[am1] - s[am2]);
      // level couplings
      const long long col = comp * cs + (long long)q * NP;
      if (n < a.depth) {
        const T* u = v + (long long)(n + 1) * a.level_stride + col;
        T g2p = u[ap2], g1p = u[ap1], g1m = u[am1], g2m = u[am2];
        if (n >= 1) {
          const T* l = v + (long long)(n - 1) * a.level_stride + col;
          const T k = ng * c0;
          g2p += k * l[ap2];
          g1p += k * l[ap1];
          g1m += k * l[am1];
          g2m += k * l[am2];
          f += ng * zeta * p * l[ia];
        }
        f += dpinv * (-g2p + T(8) * g1p - T(8) * g1m + g2m);
      } else {
        // terminator: D_p(zeta p v + N gamma c0 v^(N-1)) + c0 D_p D_p v + N gamma zeta p v^(N-1)
        const T pp2 = T(a.p0 + ap2 * a.dp), pp1 = T(a.p0 + ap1 * a.dp);
        const T pm1 = T(a.p0 + am1 * a.dp), pm2 = T(a.p0 + am2 * a.dp);
        T g2p = zeta * pp2 * s[ap2], g1p = zeta * pp1 * s[ap1];
        T g1m = zeta * pm1 * s[am1], g2m = zeta * pm2 * s[am2];
        if (n >= 1) {
          const T* l = v + (long long)(n - 1) * a.level_stride + col;
          const T k = ng * c0;
          g2p += k * l[ap2];
          g1p += k * l[ap1];
          g1m += k * l[am1];
          g2m += k * l[am2];
          f += ng * zeta * p * l[ia];
        }
        f += dpinv * (-g2p + T(8) * g1p - T(8) * g1m + g2m);
        const int ap3 = (ia + 3) % NP, ap4 = (ia + 4) % NP;
        const int am3 = (ia + NP - 3) % NP, am4 = (ia + NP - 4) % NP;
        f += c0 * dpdpinv *
             (s[am4] - T(16) * s[am3] + T(64) * s[am2] + T(16) * s[am1] - T(130) * w0 +
              T(16) * s[ap1] + T(64) * s[ap2] - T(16) * s[ap3] + s[ap4]);
      }
      acc[t][comp] = f;
    }
    // constant diabatic couplings: -(i/hbar) [Delta, W], pointwise in p
    T cm[NC];
    commutator_mi<NS, T>(coup, hv, cm);
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) acc[t][comp] += cm[comp];
  }
  __syncthreads();

  // ---- P2..P5: potential term, in place in LDS ---------------------------
  // Transform f reads its real part from array re_of(f) and its imaginary
  // part from im_of(f) (each one p-column of one packed component).
  auto fft_desc = [&](int f, int& colA, int& compA, int& colB, int& compB, int& kind, int& sj,
                       int& sk) {
    // kind 0: two real diagonal components (states sj of colA, sk of colB)
    // kind 1: off-diagonal pair (sj, sk) of column colA
    if (f < TQ) {
      colA = colB = f;
      compA = 0;
      compB = 1;
      kind = 0;
      sj = 0;
      sk = 1;
      return;
    }
    f -= TQ;
    if (NS == 3 && f < TQ / 2) {
      colA = 2 * f;
      colB = 2 * f + 1;
      compA = compB = 2;
      kind = 0;
      sj = sk = 2;
      return;
    }
    if (NS == 3) f -= TQ / 2;
    const int c = f / NPAIR;
    const int pr = f % NPAIR;
    const int j = (pr < NS - 1) ? 0 : 1;
    const int k = (pr == 0) ? 1 : (pr == 1 ? (NS == 2 ? 1 : 2) : 2);
    colA = colB = c;
    sj = j;
    sk = k;
    compA = Packing<NS>::re(j, k);
    compB = compA + 1;
    kind = 1;
  };

  // P2: first forward pass, thread item (f, n2): N1-point DFTs over stride n2.
  for (int it = tid; it < NFFT * N2; it += kBlock) {
    const int f = it / N2, n2 = it % N2;
    int colA, compA, colB, compB, kind, sj, sk;
    fft_desc(f, colA, compA, colB, compB, kind, sj, sk);
    T* re = sv + (colA * NC + compA) * NP;
    T* im = sv + (colB * NC + compB) * NP;
    cx<T> x[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) x[n1] = {re[N2 * n1 + n2], im[N2 * n1 + n2]};
    SmallDft<N1, 1, T>::run(x);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      const cx<T> w = stw[(n2 * k1) % NP];
      const cx<T> y = cmul(x[k1], w);
      re[N2 * k1 + n2] = y.re;
      im[N2 * k1 + n2] = y.im;
    }
  }
  __syncthreads();

  // P3: second forward pass, item (f, k1): contiguous N2-point DFTs.
  for (int it = tid; it < NFFT * N1; it += kBlock) {
    const int f = it / N1, k1 = it % N1;
    int colA, compA, colB, compB, kind, sj, sk;
    fft_desc(f, colA, compA, colB, compB, kind, sj, sk);
    T* re = sv + (colA * NC + compA) * NP + N2 * k1;
    T* im = sv + (colB * NC + compB) * NP + N2 * k1;
    cx<T> x[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) x[n2] = {re[n2], im[n2]};
    SmallDft<N2, 1, T>::run(x);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      re[k2] = x[k2].re;
      im[k2] = x[k2].im;
    }
  }
  __syncthreads();

  // P4: r-space multiplication (position k2 + N2 k1 holds index m = k1 + N1 k2),
  // then the first inverse pass over k2 and its twiddle.  Results stay in
  // registers until every thread has read its partner values.
  constexpr int ITEMS4 = NFFT * N1;
  constexpr int IPT4 = (ITEMS4 + kBlock - 1) / kBlock;
  cx<T> gbuf[IPT4][N2];
  const T half_dr = T(0.5 * a.dr);
  const T qlo = T(a.qlo), qhi = T(a.qhi);
  const T inv_hbar = T(a.inv_hbar);
  const T inv_np = T(1.0 / NP);
#pragma unroll
  for (int t = 0; t < IPT4; ++t) {
    const int it = tid + t * kBlock;
    if (it >= ITEMS4) continue;
    const int f = it / N1, k1 = it % N1;
    int colA, compA, colB, compB, kind, sj, sk;
    fft_desc(f, colA, compA, colB, compB, kind, sj, sk);
    const T* re = sv + (colA * NC + compA) * NP;
    const T* im = sv + (colB * NC + compB) * NP;
    const T qa = T(a.q0 + (q0 + colA) * a.dq);
    const T qb = T(a.q0 + (q0 + colB) * a.dq);
    cx<T> y[N2];
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int m = k1 + N1 * k2;
      const int mh = (m <= NP / 2) ? m : m - NP;
      const T hr = T(mh) * half_dr;  // r/2
      const bool nyq = (m == NP / 2);
      const cx<T> z = {re[k2 + N2 * k1], im[k2 + N2 * k1]};
      if (kind == 0) {
        T dA = T(0), dB = T(0);
        if (!nyq) {
          dA = (poly_eval<T, NS>(a.poly, sj, clampT(qa + hr, qlo, qhi)) -
                poly_eval<T, NS>(a.poly, sj, clampT(qa - hr, qlo, qhi))) *
               inv_hbar;
          dB = (poly_eval<T, NS>(a.poly, sk, clampT(qb + hr, qlo, qhi)) -
                poly_eval<T, NS>(a.poly, sk, clampT(qb - hr, qlo, qhi))) *
               inv_hbar;
        }
        const int mp = (NP - m) % NP;
        const int pp = (mp / N1) + N2 * (mp % N1);
        const cx<T> zp = {re[pp], -im[pp]};  // conj(Z[-m])
        const T s = (dA + dB) * T(0.5) * inv_np, d = (dA - dB) * T(0.5) * inv_np;
        // Y = -i [ s Z + d conj(Z[-m]) ]
        const cx<T> u = {s * z.re + d * zp.re, s * z.im + d * zp.im};
        y[k2] = {u.im, -u.re};
      } else {
        const T xp = clampT(qa + hr, qlo, qhi), xm = clampT(qa - hr, qlo, qhi);
        T gap;
        if (!nyq) {
          gap = poly_eval<T, NS>(a.poly, sj, xp) - poly_eval<T, NS>(a.poly, sk, xm);
        } else {
          gap = T(0.5) * (poly_eval<T, NS>(a.poly, sj, xp) + poly_eval<T, NS>(a.poly, sj, xm)) -
                T(0.5) * (poly_eval<T, NS>(a.poly, sk, xp) + poly_eval<T, NS>(a.poly, sk, xm));
        }
        const T g = gap * inv_hbar * inv_np;
        // Y = -i g Z
        y[k2] = {g * z.im, -g * z.re};
      }
    }
    SmallDft<N2, -1, T>::run(y);
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) gbuf[t][n2] = cmulc(y[n2], stw[(n2 * k1) % NP]);
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < IPT4; ++t) {
    const int it = tid + t * kBlock;
    if (it >= ITEMS4) continue;
    const int f = it / N1, k1 = it % N1;
    int colA, compA, colB, compB, kind, sj, sk;
    fft_desc(f, colA, compA, colB, compB, kind, sj, sk);
    T* re = sv + (colA * NC + compA) * NP + N2 * k1;
    T* im = sv + (colB * NC + compB) * NP + N2 * k1;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      re[n2] = gbuf[t][n2].re;
      im[n2] = gbuf[t][n2].im;
    }
  }
  __syncthreads();

  // P5: second inverse pass, item (f, n2): N1-point DFTs over stride n2,
  // natural order out.
  for (int it = tid; it < NFFT * N2; it += kBlock) {
    const int f = it / N2, n2 = it % N2;
    int colA, compA, colB, compB, kind, sj, sk;
    fft_desc(f, colA, compA, colB, compB, kind, sj, sk);
    T* re = sv + (colA * NC + compA) * NP;
    T* im = sv + (colB * NC + compB) * NP;
    cx<T> x[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) x[k1] = {re[n2 + N2 * k1], im[n2 + N2 * k1]};
    SmallDft<N1, -1, T>::run(x);
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      re[n2 + N2 * n1] = x[n1].re;
      im[n2 + N2 * n1] = x[n1].im;
    }
  }
  __syncthreads();

  // ---- P6: combine, write, level-0 trace partial -------------------------
  T* outp = static_cast<T*>(a.out) + (long long)b * a.member_stride +
                         (long long)n * a.level_stride;
  const T* yp =
      a.y ? static_cast<const T*>(a.y) + (long long)b * a.member_stride + (long long)n * a.level_stride
          : nullptr;
  const T coef = T(a.coef);
  const bool want_trace = (a.partials != nullptr) && (n == 0);
  double tr = 0.0;
#pragma unroll
  for (int t = 0; t < CPT; ++t) {
    const int e = tid + t * kBlock;
    if (e >= CELLS) continue;
    const int c = e / NP;
    const int ia = e % NP;
    const int q = q0 + c;
    if (q >= nq) continue;
    T o[NC];
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) {
      const long long idx = comp * cs + (long long)q * NP + ia;
      const T base = yp ? yp[idx] : T(0);
      o[comp] = base + coef * (acc[t][comp] + sv[(c * NC + comp) * NP + ia]);
      outp[idx] = o[comp];
    }
    if (want_trace) {
#pragma unroll
      for (int j = 0; j < NS; ++j) tr += a.mu[j][j] * (double)o[j];
#pragma unroll
      for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int k = j + 1; k < NS; ++k)
          tr += 2.0 * a.mu[j][k] * (double)o[Packing<NS>::re(j, k)];
    }
  }
  if (want_trace) {
    // deterministic workgroup sum: wave butterfly, then fixed-order over waves
    __shared__ double wsum[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = tr;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) s += wsum[w];
      a.partials[((long long)b * kRespSlots + a.slot) * a.ntiles + tile] = s;
    }
  }
}

template <typename T, int NS>
hipError_t launch_stage(int np, const StageArgs& a, int nblocks, hipStream_t s) {
  switch (np) {
#define QHFPE_CASE(NP_)                                                             \
  case NP_:                                                                         \
    hipLaunchKernelGGL((stage_kernel<T, NS, NP_>), dim3(nblocks), dim3(kBlock), 0, s, a); \
    return hipGetLastError();
    QHFPE_CASE(8)
    QHFPE_CASE(12)
    QHFPE_CASE(16)
    QHFPE_CASE(24)
    QHFPE_CASE(32)
    QHFPE_CASE(48)
    QHFPE_CASE(64)
    QHFPE_CASE(96)
    QHFPE_CASE(128)
    QHFPE_CASE(192)
    QHFPE_CASE(256)
#undef QHFPE_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace qhfpe
