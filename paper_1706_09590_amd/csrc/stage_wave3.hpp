// Fused RK4 stage, wave-independent variant for three electronic states:
// out = y + coef * L v with the operator of stage_kernel.hpp (Eq. (heom) of
// Ikeda & Tanimura (2017) with one Drude exponential and V(q) = q, closed by
// Eq. (GMFP); potential term of Eq. (quantum-liouvillian) through the DFT
// along p; Sec. III discretisation), for np = 128 or 256.
//
// The plan of the two-state wave variant (stage_wave.hpp), widened to the
// nine packed components of three states.  One wave owns a task: C
// neighbouring q columns of one level of one batch member (C = 2 at
// np = 128, 1 at np = 256).  Lane l holds the K = np / 64 consecutive p
// nodes K l .. K l + K - 1 of every column.  The waves of a workgroup share
// only the twiddle and symbol tables.
//
//  - local terms (kinetic, level couplings, terminator) one component at a
//    time, exactly as for two states; the constant couplings -(i/hbar)
//    [Delta, W] afterwards, from this lane's own LDS entries of all nine
//    components;
//  - potential term: four complex np-point transforms per column (the
//    diagonal pair W00 + i W11 and the coherences W01, W02, W12) and one for
//    W22 (W22 of the first column + i W22 of the second; with one column
//    per task, + i times a zero column).  The transform count is not a multiple of the
//    wave's width, so each FFT pass runs in rounds of 64 items (the last one
//    partly idle); in the contiguous passes a round holds four whole
//    transforms, so the partner row -m of every row of a round lies in the
//    same round and the r-space multiply runs round by round in place.
//
// LDS per wave: the real columns of the task's transforms (18 at np = 128,
// 10.6 KB in FP32; 10 at np = 256, 11 KB in FP32).  Two columns per task at
// np = 256 would need 19.9 KB per FP32 wave (six waves per CU) and 40 KB per
// FP64 one; one column holds twelve FP32 waves per CU, at the price of a
// half-empty W22 transform and a 7-column window for one output column.
#pragma once

#include "stage_wave.hpp"

namespace qhfpe {

template <int NP_, int WPB_>
struct WavePlan3 {
  static constexpr int NP = NP_;
  static constexpr int N1 = FftSplit<NP>::N1, N2 = FftSplit<NP>::N2;
  static constexpr int K = NP / 64;       // p nodes per lane
  static constexpr int C = wave3_columns(NP);  // q columns per task
  static constexpr int NC = 9;            // packed components (three states)
  static constexpr int NF = 4 * C + (C + 1) / 2;  // complex transforms per task
  static constexpr int P1 = NF * N2;      // items of the stride-N2 passes
  static constexpr int P2 = NF * N1;      // items of the contiguous passes
  static constexpr int R1 = (P1 + 63) / 64, R2 = (P2 + 63) / 64;  // rounds of 64 items
  static constexpr int WPB = WPB_;
  static constexpr int NT = 64 * WPB;
  static constexpr int LDP0 = NP + NP / N2;
  static constexpr int LDP = LDP0 + ((4 - LDP0 % 16) + 16) % 16;
  static_assert((C == 1 || C == 2) && K >= 2 && 64 % N1 == 0 && N2 % 4 == 0, "three-state wave plan");
};

// LDS column of packed component comp of task column i (C columns per
// task): transform f = 4 i + t takes columns 2 f (real part) and 2 f + 1
// (imaginary part): t = 0 the diagonal pair (W00, W11), t = 1..3 the
// coherence (Re, Im) of the pairs (0,1), (0,2), (1,2); transform 4 C takes
// W22 of columns 0 and 1 (with C = 1, column 8 C + 1 holds zeros).
template <int C>
__device__ __forceinline__ constexpr int wave3_slot(int i, int comp) {
  return comp < 2 ? 8 * i + comp : (comp == 2 ? 8 * C + i : 8 * i + comp - 1);
}

// Waves per SIMD the register allocation aims at (the second launch bound):
// three in FP32, two in FP64 (LDS allows no more).
template <typename T, int NP>
constexpr int wave3_waves_per_simd() {
  return sizeof(T) == 4 ? 3 : 2;
}

// NTS: non-temporal output stores (StageArgs::stream_out).  WPB: waves per
// workgroup (StageArgs::wpb).  MIX: members of their own depths
// (StageArgs::mlev).
template <typename T, int NP, bool NTS, int WPB_, bool MIX>
__global__ void __launch_bounds__((WavePlan3<NP, WPB_>::NT), (wave3_waves_per_simd<T, NP>()))
    stage_wave3_kernel(StageArgs a) {
  using W = WavePlan3<NP, WPB_>;
  constexpr int N1 = W::N1, N2 = W::N2, K = W::K, C = W::C, NC = W::NC, WPB = W::WPB;
  constexpr int NF = W::NF, P1 = W::P1, P2 = W::P2, R1 = W::R1, R2 = W::R2;
  constexpr int LDP = W::LDP;
  auto pad = [](int x) { return x + x / N2; };  // padded position of p node x in a column
  __shared__ T sbuf[WPB][2 * NF * LDP];  // per wave: v tile, transformed in place
  __shared__ cx<T> stw[N1 * (N2 + 1)];   // w^(n2 k1), row k1 padded to N2 + 1
  __shared__ T ssym[2 * NP];             // DFT symbols of D_p2 and D_p D_p (scaled by 1/np)

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nq = a.nq;
  const int ntasks = stage_units<MIX>(a);
  // levels fastest, so that the tasks of all levels of one column pair run
  // together and share their level neighbours through L2
  const int task_id = xcd_logical_block(blockIdx.x, a.nblocks_padded) * WPB + wid;
  // a wave past the last task still meets its workgroup at the table
  // barrier below; it takes task 0's indices and ends after the barrier
  const bool active = task_id < ntasks;
  const int task = active ? task_id : 0;
  const UnitPos pos = unit_pos<MIX>(a, task);
  const int n = pos.n, tile = pos.tile, b = pos.b;
  const int q0 = C * tile;
  T* const s = sbuf[wid];

  constexpr unsigned ES = sizeof(T);
  const unsigned level_bytes = (unsigned)(a.level_stride * ES);
  const unsigned cbytes = (unsigned)(a.comp_stride * ES);
  const T* vm = static_cast<const T*>(a.v) + (long long)b * a.member_stride;
  // loads past a descriptor's size return zero: the ghost columns beyond
  // the q edges, v^(n+1) at n = N, v^(n-1) at n = 0 and a missing y
  const bool has_up = n < pos.depth, has_dn = n >= 1;
  const rsrc_t rn = make_rsrc(vm + (long long)n * a.level_stride, level_bytes);
  const rsrc_t ru = make_rsrc(vm + (long long)(has_up ? n + 1 : n) * a.level_stride, has_up ? level_bytes : 0u);
  const rsrc_t rd = make_rsrc(vm + (long long)(has_dn ? n - 1 : n) * a.level_stride, has_dn ? level_bytes : 0u);
  const bool has_y = a.y != nullptr;
  const rsrc_t ry = make_rsrc(has_y ? static_cast<const T*>(a.y) + (long long)b * a.member_stride +
                                          (long long)n * a.level_stride
                                    : vm,
                              has_y ? level_bytes : 0u);
  const double* bath = a.bath + kBathStride * b;
  const T zeta = T(bath[0]), c0 = T(bath[2]), cdel = T(bath[3]);
  const T ng = T(n * bath[1]);
  const T coef = T(a.coef);
  const int a0 = K * lane;  // first p node of this lane
  T p[K], kscale[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    p[j] = T(a.p0 + (a0 + j) * a.dp);
    kscale[j] = -(p[j] * T(a.inv_mass)) * T(1.0 / (60.0 * a.dq));
  }
  // upwind coefficients (x60) on q offsets -3..3 for the sign of p at this
  // lane's first node, and the mirrored stencil for nodes of the other sign
  const bool pos0 = p[0] >= T(0);
  T kc[7], kcm[7];
#pragma unroll
  for (int o = -3; o <= 3; ++o) {
    const double cp = (o <= 2) ? kUpwind[o + 3] : 0.0;
    const double cn = (o >= -2) ? -kUpwind[3 - o] : 0.0;
    kc[o + 3] = T(pos0 ? cp : cn);
    kcm[o + 3] = T(pos0 ? cn : cp);
  }
  const bool mixed = (p[K - 1] >= T(0)) != pos0;
  const bool any_mixed = __any(mixed);

  // byte offsets of the q columns q0-3 .. q0+C+2 at this lane's first node;
  // columns outside the grid point past the end of every level (read as 0)
  constexpr unsigned kGhost = 0x7fffff00u;
  unsigned qo[C + 6];
#pragma unroll
  for (int t = 0; t < C + 6; ++t) {
    const int q = q0 + t - 3;
    qo[t] = (q >= 0 && q < nq) ? ((unsigned)q * NP + a0) * ES : kGhost;
  }
  const T dpinv = T(1.0 / (12.0 * a.dp));
  // the terminator level differentiates zeta p v^(N) in place of v^(N+1)
  // (Eq. (GMFP))
  const T zterm = has_up ? T(0) : zeta;

  // ---- local terms, one component at a time ------------------------------
  // FP32 issues the loads of component c + 1 while component c is computed
  // (second register slots: the window and y after c's kinetic term,
  // v^(n +- 1) after c's level terms); FP64 issues them once c is done.
  constexpr bool kPipe = sizeof(T) == 4;
  constexpr int NSW = kPipe ? 2 : 1;  // window slots
  T base[C][NC][K];     // y + coef * (all terms except the potential)
  T lw[2][2][C][K];     // v^(n+1), v^(n-1) at the task columns
  T ky[2][C][K];        // y at the task columns
  T kw[NSW][C + 6][K];  // kinetic window q0-3 .. q0+C+2
  auto issue_level = [&](int comp, int slot) {
    const unsigned so = comp * cbytes;
#pragma unroll
    for (int i = 0; i < C; ++i) {
      buf_load_n<K>(ru, qo[i + 3], so, lw[slot][0][i]);
      buf_load_n<K>(rd, qo[i + 3], so, lw[slot][1][i]);
    }
  };
  auto issue_window = [&](int comp, int slot) {
    const unsigned so = comp * cbytes;
#pragma unroll
    for (int t = 0; t < C + 6; ++t) buf_load_n<K>(rn, qo[t], so, kw[slot][t]);
  };
  auto issue_y = [&](int comp, int slot) {
    const unsigned so = comp * cbytes;
#pragma unroll
    for (int i = 0; i < C; ++i) buf_load_n<K>(ry, qo[i + 3], so, ky[slot][i]);
  };
  // table loads first, the first component's loads right after them, then
  // the table stores and the workgroup's only barrier (as for two states)
  {
    constexpr int NTW = N1 * (N2 + 1), NSY = 2 * NP;
    constexpr int RTW = (NTW + W::NT - 1) / W::NT, RSY = (NSY + W::NT - 1) / W::NT;
    T twr[RTW][2], syr[RSY];
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
      const T* const t = static_cast<const T*>(a.twiddle2) + 2 * min(tid + r * W::NT, NTW - 1);
      twr[r][0] = t[0];
      twr[r][1] = t[1];
    }
#pragma unroll
    for (int r = 0; r < RSY; ++r) syr[r] = static_cast<const T*>(a.psym)[min(tid + r * W::NT, NSY - 1)];
    __builtin_amdgcn_sched_barrier(0);
    issue_window(0, 0);
    issue_y(0, 0);
    issue_level(0, 0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
      const int j = tid + r * W::NT;
      if (j < NTW) stw[j] = cx<T>{twr[r][0], twr[r][1]};
    }
#pragma unroll
    for (int r = 0; r < RSY; ++r) {
      const int j = tid + r * W::NT;
      if (j < NSY) ssym[j] = syr[r];
    }
    __syncthreads();  // the only workgroup barrier
  }
  if (!active) return;
#pragma unroll
  for (int comp = 0; comp < NC; ++comp) {
    const int ws = kPipe ? (comp & 1) : 0;
    const int ls = comp & 1;
    T kin[C][K];
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) {
        T k = T(0);
#pragma unroll
        for (int o = 0; o < 7; ++o) k += kc[o] * kw[ws][i + o][j];
        if (any_mixed && ((p[j] >= T(0)) != pos0)) {
          k = T(0);
#pragma unroll
          for (int o = 0; o < 7; ++o) k += kcm[o] * kw[ws][i + o][j];
        }
        kin[i][j] = kscale[j] * k;
        asm volatile("" : "+v"(kin[i][j]));
      }
    __builtin_amdgcn_sched_barrier(0);
    if (kPipe && comp + 1 < NC) {
      issue_window(comp + 1, ws ^ 1);
      issue_y(comp + 1, ls ^ 1);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < C; ++i) {
      T g[K], lev[K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const T w0 = kw[ws][i + 3][j];
        //   n < N: v^(n+1) + n gamma c0 v^(n-1);  n = N: zeta p v^(N) + N gamma c0 v^(N-1)
        g[j] = lw[ls][0][i][j] + (zterm * p[j]) * w0 + (ng * c0) * lw[ls][1][i][j];
        lev[j] = -ng * w0 + (ng * zeta * p[j]) * lw[ls][1][i][j];
        s[wave3_slot<C>(i, comp) * LDP + pad(a0 + j)] = w0;
        if (C == 1 && comp == 2) s[(8 * C + 1) * LDP + pad(a0 + j)] = T(0);  // imaginary part of the W22 transform
      }
      // D_p g with the neighbouring lanes' nodes (periodic in p)
      T e[K + 4];
      e[0] = lane_prev(g[K - 2]);
      e[1] = lane_prev(g[K - 1]);
#pragma unroll
      for (int j = 0; j < K; ++j) e[j + 2] = g[j];
      e[K + 2] = lane_next(g[0]);
      e[K + 3] = lane_next(g[1]);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        lev[j] += dpinv * (-e[j + 4] + T(8) * e[j + 3] - T(8) * e[j + 1] + e[j]);
        base[i][comp][j] = ky[ls][i][j] + coef * (kin[i][j] + lev[j]);
        asm volatile("" : "+v"(base[i][comp][j]));
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (comp + 1 < NC) {
      if (kPipe) {
        issue_level(comp + 1, ls ^ 1);
      } else {
        issue_window(comp + 1, 0);
        issue_y(comp + 1, ls ^ 1);
        issue_level(comp + 1, ls ^ 1);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // constant diabatic couplings -(i/hbar) [Delta, W], pointwise in p, from
  // this lane's own LDS entries of the nine components (each lane reads only
  // what it wrote, so no barrier is needed)
  if (a.coup[0][1] != 0.0 || a.coup[0][2] != 0.0 || a.coup[1][2] != 0.0) {
    T cpl[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) cpl[j][k] = T(a.coup[j][k]);
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) {
        T hv[NC], cm[NC];
#pragma unroll
        for (int comp = 0; comp < NC; ++comp) hv[comp] = s[wave3_slot<C>(i, comp) * LDP + pad(a0 + j)];
        commutator_mi<3, T>(cpl, hv, cm);
#pragma unroll
        for (int comp = 0; comp < NC; ++comp) base[i][comp][j] += coef * cm[comp];
      }
  }
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int comp = 0; comp < NC; ++comp)
#pragma unroll
      for (int j = 0; j < K; ++j) asm volatile("" : "+v"(base[i][comp][j]));

  // ---- potential term ----------------------------------------------------
  // transform f: real part in LDS column 2 f, imaginary part in 2 f + 1
  auto re_of = [&](int f) { return s + 2 * f * LDP; };

  // first forward pass: N1-point DFTs over stride N2, twiddle (item: f, n2)
#pragma unroll
  for (int t = 0; t < R1; ++t) {
    const int item = lane + 64 * t;
    if (P1 % 64 == 0 || t + 1 < R1 || item < P1) {
      const int n2 = item % N2;
      T* const re = re_of(item / N2);
      T* const im = re + LDP;
      cx<T> x[N1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) x[n1] = {re[(N2 + 1) * n1 + n2], im[(N2 + 1) * n1 + n2]};
      SmallDft<N1, 1, T>::run(x);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) {
        const cx<T> y = cmul(x[k1], stw[k1 * (N2 + 1) + n2]);
        re[(N2 + 1) * k1 + n2] = y.re;
        im[(N2 + 1) * k1 + n2] = y.im;
      }
    }
  }
  wave_lds_sync();

  // r-space multipliers of row k1 of transform f (host-permuted so that the
  // N2 values of a row are contiguous).  Planes: 0..2 the diagonal tables
  // of states 0..2, 3..5 the coherence tables of the pairs (0,1), (0,2),
  // (1,2) halved (a coherence is treated as a pair of equal multipliers).
  // The packed diagonals take planes 0 and 1 at their column; the W22
  // transform takes plane 2 at column q0 (real part) and q0 + 1 (imaginary;
  // with one column per task its multiplier meets a zero column and does
  // not matter).
  const unsigned tbytes = (unsigned)((long long)nq * NP * ES);
  const rsrc_t rt = make_rsrc(a.mtab, (unsigned)kWaveTables3 * tbytes);
  auto load_mul = [&](int t, T* mA, T* mB) {
    const int item = min(lane + 64 * t, P2 - 1);
    const int f = item / N1, k1 = item % N1;
    const int col = (f < 4 * C) ? f / 4 : 0, kind = (f < 4 * C) ? f % 4 : 4;
    const int pa = kind == 0 ? 0 : (kind == 4 ? 2 : 2 + kind);
    const int pb = kind == 0 ? 1 : pa;
    const int qa = min(q0 + col, nq - 1), qb = min(q0 + (kind == 4 ? 1 : col), nq - 1);
    const unsigned oa = (unsigned)pa * tbytes + ((unsigned)qa * NP + (unsigned)k1 * N2) * ES;
    const unsigned ob = (unsigned)pb * tbytes + ((unsigned)qb * NP + (unsigned)k1 * N2) * ES;
#pragma unroll
    for (int k2 = 0; k2 < N2; k2 += 4) {
      const Quad<T> qa4 = buf_load4(rt, oa + k2 * ES, 0, T(0));
      const Quad<T> qb4 = buf_load4(rt, ob + k2 * ES, 0, T(0));
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        mA[k2 + j] = qa4.v[j];
        mB[k2 + j] = qb4.v[j];
      }
    }
  };
  // round t's multipliers are loaded one round ahead (round 0's before the
  // second forward pass)
  T mulA[2][N2], mulB[2][N2];
  load_mul(0, mulA[0], mulB[0]);

  // second forward pass: contiguous N2-point DFTs of row k1 (item: f, k1)
#pragma unroll
  for (int t = 0; t < R2; ++t) {
    const int item = lane + 64 * t;
    if (P2 % 64 == 0 || t + 1 < R2 || item < P2) {
      const int k1 = item % N1;
      T* const zr = re_of(item / N1) + (N2 + 1) * k1;
      T* const zi = zr + LDP;
      cx<T> x[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) x[n2] = {zr[n2], zi[n2]};
      SmallDft<N2, 1, T>::run(x);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        zr[k2] = x[k2].re;
        zi[k2] = x[k2].im;
      }
      // row 0 also stores X[0] in its padding slot, so that the partner of
      // index m lies at pbase - k2 for every row
      if (k1 == 0) {
        zr[N2] = x[0].re;
        zi[N2] = x[0].im;
      }
    }
  }
  wave_lds_sync();

  // r-space multiplication (position k2 + (N2+1) k1 holds index
  // m = k1 + N1 k2) and the first inverse pass, round by round: a round
  // holds whole transforms, and its lanes read their own and partner rows
  // before any of them writes
  const T c0t = has_up ? T(0) : c0;  // terminator level carries c0 D_p D_p
#pragma unroll
  for (int t = 0; t < R2; ++t) {
    if (t + 1 < R2) load_mul(t + 1, mulA[(t + 1) & 1], mulB[(t + 1) & 1]);
    const int item = lane + 64 * t;
    const bool live = P2 % 64 == 0 || t + 1 < R2 || item < P2;
    const int k1 = item % N1;
    const int f = live ? item / N1 : 0;
    cx<T> yk[N2];
    if (live) {
      const T* const re = re_of(f);
      const T* const im = re + LDP;
      const T* zr = re + (N2 + 1) * k1;
      const T* zi = im + (N2 + 1) * k1;
      const int pbase = (k1 == 0) ? N2 : (N2 - 1) + (N2 + 1) * (N1 - k1);
      const T* pr = re + pbase;
      const T* pi = im + pbase;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const cx<T> z = {zr[k2], zi[k2]};
        const cx<T> zp = {pr[-k2], -pi[-k2]};
        const T e = cdel * ssym[k1 + N1 * k2] + c0t * ssym[NP + k1 + N1 * k2];
        // Y = -i [ s Z[m] + d conj(Z[-m]) ] + e Z
        const T sA = mulA[t & 1][k2] + mulB[t & 1][k2], dA = mulA[t & 1][k2] - mulB[t & 1][k2];
        const cx<T> u = {sA * z.re + dA * zp.re, sA * z.im + dA * zp.im};
        yk[k2] = {u.im + e * z.re, -u.re + e * z.im};
      }
      SmallDft<N2, -1, T>::run(yk);
    }
    wave_lds_sync();
    if (live) {
      T* const zr = re_of(f) + (N2 + 1) * k1;
      T* const zi = zr + LDP;
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) {
        const cx<T> g = cmulc(yk[n2], stw[k1 * (N2 + 1) + n2]);
        zr[n2] = g.re;
        zi[n2] = g.im;
      }
    }
  }
  wave_lds_sync();

  // second inverse pass: N1-point DFTs over stride N2, natural order out
#pragma unroll
  for (int t = 0; t < R1; ++t) {
    const int item = lane + 64 * t;
    if (P1 % 64 == 0 || t + 1 < R1 || item < P1) {
      const int n2 = item % N2;
      T* const re = re_of(item / N2);
      T* const im = re + LDP;
      cx<T> x[N1];
#pragma unroll
      for (int kk = 0; kk < N1; ++kk) x[kk] = {re[n2 + (N2 + 1) * kk], im[n2 + (N2 + 1) * kk]};
      SmallDft<N1, -1, T>::run(x);
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        re[n2 + (N2 + 1) * n1] = x[n1].re;
        im[n2 + (N2 + 1) * n1] = x[n1].im;
      }
    }
  }
  wave_lds_sync();

  // ---- combine, write, level-0 trace partial -----------------------------
  const rsrc_t ro = make_rsrc(static_cast<T*>(a.out) + (long long)b * a.member_stride + (long long)n * a.level_stride,
                              level_bytes);
  const bool want_trace = (a.partials != nullptr) && (n == 0);
  double tr = 0.0;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    if (q0 + i >= nq) continue;
    T o[NC][K];
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) {
#pragma unroll
      for (int j = 0; j < K; ++j) o[comp][j] = base[i][comp][j] + coef * s[wave3_slot<C>(i, comp) * LDP + pad(a0 + j)];
      buf_store_n<K, NTS ? kStoreNT : 0>(o[comp], ro, qo[i + 3], comp * cbytes);
    }
    if (want_trace) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        tr += a.mu[0][0] * (double)o[0][j] + a.mu[1][1] * (double)o[1][j] + a.mu[2][2] * (double)o[2][j];
        tr += 2.0 * (a.mu[0][1] * (double)o[3][j] + a.mu[0][2] * (double)o[5][j] + a.mu[1][2] * (double)o[7][j]);
      }
    }
  }
  if (want_trace) {
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
    if (lane == 0) a.partials[((long long)b * kRespSlots + a.slot) * a.ntiles + tile] = tr;
  }
}

// (MIX: members of their own depths, StageArgs::mlev)
template <typename T, int NP, bool NTS, int WPB>
hipError_t launch_wave3_one(const StageArgs& a, int nblocks, hipStream_t s) {
  if (a.mlev)
    hipLaunchKernelGGL((stage_wave3_kernel<T, NP, NTS, WPB, true>), dim3(nblocks), dim3(WavePlan3<NP, WPB>::NT), 0, s,
                       a);
  else
    hipLaunchKernelGGL((stage_wave3_kernel<T, NP, NTS, WPB, false>), dim3(nblocks), dim3(WavePlan3<NP, WPB>::NT), 0, s,
                       a);
  return hipGetLastError();
}

// workgroup sizes: four waves only in FP32 (large launches); two in FP64
// (a four-wave FP64 workgroup's LDS would leave room for one per CU)
template <typename T, int NP>
hipError_t launch_wave3_np(const StageArgs& a, int nblocks, hipStream_t s) {
  if (a.closure != nullptr || a.qcoup) return hipErrorInvalidValue;
  if (a.wpb == kWaveTasksPerBlockSmall)
    return a.stream_out ? launch_wave3_one<T, NP, true, kWaveTasksPerBlockSmall>(a, nblocks, s)
                        : launch_wave3_one<T, NP, false, kWaveTasksPerBlockSmall>(a, nblocks, s);
  if constexpr (sizeof(T) == 4) {
    if (a.wpb == kWaveTasksPerBlock)
      return a.stream_out ? launch_wave3_one<T, NP, true, kWaveTasksPerBlock>(a, nblocks, s)
                          : launch_wave3_one<T, NP, false, kWaveTasksPerBlock>(a, nblocks, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_stage_wave3(int np, const StageArgs& a, int nblocks, hipStream_t s) {
  if (np == 128) return launch_wave3_np<T, 128>(a, nblocks, s);
  if (np == 256) return launch_wave3_np<T, 256>(a, nblocks, s);
  return hipErrorInvalidValue;
}

}  // namespace qhfpe
