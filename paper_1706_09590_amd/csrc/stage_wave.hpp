// Fused RK4 stage, wave-independent variant for two electronic states and
// np = 128 or 256:  out = y + coef * L v  with the same operator as
// stage_kernel.hpp (Eq. (heom) of Ikeda & Tanimura (2017) with one Drude
// exponential and V(q) = q, closed by Eq. (GMFP); potential term of Eq.
// (quantum-liouvillian) through the DFT along p; Sec. III discretisation).
//
// One wave owns a whole task: C neighbouring q columns (C = 512 / np) of one
// level of one batch member, all four packed components.  Lane l holds the
// K = np / 64 consecutive p nodes K l .. K l + K - 1 of every column.  The
// waves of a workgroup share only the twiddle and symbol tables (loaded once
// behind the single workgroup barrier); every later step orders its LDS
// accesses within the wave, so a wave waiting for memory never stalls
// another.
//
//  - kinetic -(p/m) D_q: 5th-order upwind over a (C + 6)-column q window;
//  - D_p of the level field g: the stencil neighbours p +- 1, +- 2 of a
//    lane's nodes are its own or the neighbouring lanes' (DPP wave
//    rotations; the p grid is periodic and one column fills the wave);
//  - potential term: 2 C complex np-point transforms per task (the two real
//    diagonals of a column packed into one, the off-diagonal pair in
//    another), two-pass FFT np = N1 N2 with 2 C N2 / 64 and 2 C N1 / 64 items
//    per lane in the two passes (every lane busy), r-space multiply in place
//    (all lanes read their own and partner rows before any lane writes),
//    inverse transform;
//  - constant diabatic coupling: pointwise commutator in p, added while the
//    last component is computed; a q-dependent coupling U_01(q) instead
//    enters the r-space multiply (QC instantiation), where it mixes the
//    packed-diagonal and coherence transforms of a column.
#pragma once

#include "device_common.hpp"
#include "qhfpe_internal.hpp"
#include "stage_kernel.hpp"

namespace qhfpe {

template <int NP_, int WPB_ = kWaveTasksPerBlock>
struct WavePlan {
  static constexpr int NP = NP_;
  static constexpr int N1 = FftSplit<NP>::N1, N2 = FftSplit<NP>::N2;
  static constexpr int K = NP / 64;            // p nodes per lane
  static constexpr int C = wave_columns(NP);   // q columns per task
  static constexpr int NC = 4;                 // packed components (two states)
  static constexpr int NF = 2 * C;             // complex transforms per task
  static constexpr int I1 = NF * N2 / 64;      // items per lane, stride-N2 passes
  static constexpr int I2 = NF * N1 / 64;      // items per lane, contiguous passes
  static constexpr int WPB = WPB_;  // waves per workgroup
  static constexpr int NT = 64 * WPB;
  static constexpr int LDP0 = NP + NP / N2;
  static constexpr int LDP = LDP0 + ((4 - LDP0 % 16) + 16) % 16;
  static_assert(K >= 2 && NF * N2 % 64 == 0 && NF * N1 % 64 == 0 && N2 % 4 == 0, "wave plan");
};

// M consecutive elements per lane stored with one or two 16-byte (or one
// 8-byte) accesses; voff aligned to the access size.
template <int M, int CPOL = 0>
__device__ __forceinline__ void buf_store_n(const float* v, rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (M == 2) {
    using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    const qhfpe_f2 x = {v[0], v[1]};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, (int)voff, (int)soff, CPOL);
  } else {
    static_assert(M == 4, "2 or 4 floats");
    buf_store4<CPOL>(Quad<float>{{v[0], v[1], v[2], v[3]}}, r, voff, soff);
  }
}
template <int M, int CPOL = 0>
__device__ __forceinline__ void buf_store_n(const double* v, rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (M == 2) {
    using u4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    const qhfpe_d2 x = {v[0], v[1]};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, x), r, (int)voff, (int)soff, CPOL);
  } else {
    static_assert(M == 4, "2 or 4 doubles");
    buf_store4<CPOL>(Quad<double>{{v[0], v[1], v[2], v[3]}}, r, voff, soff);
  }
}

// QC: q-dependent diabatic coupling U_01(q), applied in the r-space multiply
// (it mixes the packed-diagonal and coherence transforms of a column).
// Occupancy (the second launch bound, waves per SIMD): FP32 without QC is
// held to four waves per SIMD (128 VGPRs); the others run two (FP64: 79 KB
// of LDS per four-wave workgroup allows no more).
// NTS: non-temporal output stores (the launcher picks it when the state
// arrays exceed the memory-side cache, StageArgs::stream_out).  WPB: waves
// per workgroup (StageArgs::wpb).  MIX: members of their own depths
// (StageArgs::mlev).
template <typename T, int NP, bool QC, bool NTS = false, int WPB_ = kWaveTasksPerBlock, bool MIX = false>
__global__ void __launch_bounds__((WavePlan<NP, WPB_>::NT), (sizeof(T) == 4 && !QC ? 4 : 2))
    stage_wave_kernel(StageArgs a) {
  using W = WavePlan<NP, WPB_>;
  constexpr int N1 = W::N1, N2 = W::N2, K = W::K, C = W::C, NC = W::NC, WPB = W::WPB;
  constexpr int I1 = W::I1, I2 = W::I2;
  constexpr int LDP = W::LDP;
  auto pad = [](int x) { return x + x / N2; };  // padded position of p node x in a column
  __shared__ T sbuf[WPB][C * NC * LDP];  // per wave: v tile, transformed in place
  __shared__ cx<T> stw[N1 * (N2 + 1)];   // w^(n2 k1), row k1 padded to N2 + 1
  __shared__ T ssym[2 * NP];             // DFT symbols of D_p2 and D_p D_p (scaled by 1/np)

  const int tid = threadIdx.x;
  // the wave index is uniform across the wave; saying so keeps every
  // quantity derived from it (task, level, member, buffer descriptors) in
  // scalar registers instead of per-lane loops over descriptor values
  const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nq = a.nq;
  const int ntasks = stage_units<MIX>(a);
  // levels fastest, as in stage_kernel: the tasks of all levels of one
  // column group run together and share their level neighbours through L2
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
  // Loads past a descriptor's size return zero.  That supplies the zero
  // ghost columns beyond the q edges (their offsets are set past every
  // level), v^(n+1) at n = N, v^(n-1) at n = 0 and a missing y.
  const bool has_up = n < pos.depth, has_dn = n >= 1;
  // learned terminator: at n = N the level above is the closure's W^(N+1)
  const bool clos = a.closure != nullptr && !has_up;
  const rsrc_t rn = make_rsrc(vm + (long long)n * a.level_stride, level_bytes);
  const rsrc_t ru =
      clos ? make_rsrc(static_cast<const T*>(a.closure) + (long long)b * a.level_stride, level_bytes)
           : make_rsrc(vm + (long long)(has_up ? n + 1 : n) * a.level_stride, has_up ? level_bytes : 0u);
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
  // lane's first node; nodes of the other sign (only where p = 0 falls
  // inside a lane) are redone below
  const bool pos0 = p[0] >= T(0);
  T kc[7], kcm[7];  // this lane's stencil and the mirrored one
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
  // (Eq. (GMFP)), unless a learned closure supplies W^(N+1)
  const T zterm = (has_up || clos) ? T(0) : zeta;

  // ---- local terms, one component at a time ------------------------------
  // v^(n) at the task columns is the middle of the kinetic window, so it is
  // loaded once.  In FP32 at np = 128 the loads of component c + 1 are
  // issued while component c is computed, into second register slots: the
  // window and y after c's kinetic term, v^(n +- 1) after c's level terms.
  // Double has no registers for a second window; it issues all loads of
  // component c + 1 once component c is done.  FP32 at np = 256 does the
  // same as double: without the second slots it holds four waves per SIMD
  // instead of three, which is faster there.
  constexpr bool kPipe = sizeof(T) == 4 && NP == 128;
  constexpr int NSW = kPipe ? 2 : 1;  // window slots
  T base[C][NC][K];  // y + coef * (all terms except the potential)
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
  // constant diabatic coupling -(i/hbar) [Delta, W] (pointwise in p): with
  // d = Delta_01 / hbar it adds -2 d Im W01 to W00, +2 d Im W01 to W11, 0 to
  // Re W01 and d (W00 - W11) to Im W01; it is applied with the last
  // component, reading W00 and W11 back from this lane's own LDS entries
  const bool has_coup = a.coup[0][1] != 0.0;
  const T dcoef = T(a.coef * a.coup[0][1]);
  // The twiddle and symbol tables go to LDS behind the workgroup's only
  // barrier.  Their loads are issued first and the first component's loads
  // right after them, so that the wait for the tables (loads complete in
  // issue order) does not wait for the component and the component's
  // latency overlaps the table stores and the barrier.
  {
    constexpr int NTW = N1 * (N2 + 1), NSY = 2 * NP;
    constexpr int RTW = (NTW + W::NT - 1) / W::NT, RSY = (NSY + W::NT - 1) / W::NT;
    T twr[RTW][2], syr[RSY];  // (plain scalars: an array of cx<T> went to scratch)
    // (lanes past a table's end load its last entry and store nothing, so
    // that the loads need no branch)
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
      const T* const t = static_cast<const T*>(a.twiddle2) + 2 * min(tid + r * W::NT, NTW - 1);
      twr[r][0] = t[0];
      twr[r][1] = t[1];
    }
#pragma unroll
    for (int r = 0; r < RSY; ++r) syr[r] = static_cast<const T*>(a.psym)[min(tid + r * W::NT, NSY - 1)];
    __builtin_amdgcn_sched_barrier(0);
    // (an inactive wave loads task 0's data too: in bounds, and no branch)
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
    // kinetic term at the lane's nodes of every column
    T kin[C][K];
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) {
        T k = T(0);
#pragma unroll
        for (int o = 0; o < 7; ++o) k += kc[o] * kw[ws][i + o][j];
        if (any_mixed && ((p[j] >= T(0)) != pos0)) {
          // where p = 0 falls inside a lane, its nodes of the other sign
          // take the mirrored stencil
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
    // level field and level terms, then the base state
#pragma unroll
    for (int i = 0; i < C; ++i) {
      T g[K], lev[K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const T w0 = kw[ws][i + 3][j];
        // field differentiated once along p:
        //   n < N: v^(n+1) + n gamma c0 v^(n-1);  n = N: zeta p v^(N) + N gamma c0 v^(N-1)
        // (the absent neighbour levels read as zero; n gamma = 0 at n = 0)
        g[j] = lw[ls][0][i][j] + (zterm * p[j]) * w0 + (ng * c0) * lw[ls][1][i][j];
        lev[j] = -ng * w0 + (ng * zeta * p[j]) * lw[ls][1][i][j];
        s[(i * NC + comp) * LDP + pad(a0 + j)] = w0;
      }
      // D_p g: nodes a0-2, a0-1 come from the previous lane, a0+K, a0+K+1
      // from the next one (periodic in p: one column spans the whole wave)
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
        if (comp == NC - 1 && has_coup) {
          const T w3 = kw[ws][i + 3][j];  // Im W01
          const T h00 = s[(i * NC + 0) * LDP + pad(a0 + j)], h11 = s[(i * NC + 1) * LDP + pad(a0 + j)];
          base[i][0][j] -= T(2) * dcoef * w3;
          base[i][1][j] += T(2) * dcoef * w3;
          base[i][3][j] += dcoef * (h00 - h11);
        }
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
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int comp = 0; comp < NC; ++comp)
#pragma unroll
      for (int j = 0; j < K; ++j) asm volatile("" : "+v"(base[i][comp][j]));

  // ---- potential term ----------------------------------------------------
  // transform f (0 .. 2C-1): column f % C; f / C = 0 for the packed
  // diagonals (0, 1), 1 for the off-diagonal pair.  Its real part is the
  // LDS column of component 2 (f / C), its imaginary part the next one.
  auto re_of = [&](int f) { return s + ((f % C) * NC + 2 * (f / C)) * LDP; };

  // first forward pass: N1-point DFTs over stride N2, twiddle
#pragma unroll
  for (int t = 0; t < I1; ++t) {
    const int item = lane + 64 * t;
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
  wave_lds_sync();

  // r-space multipliers of this lane's items (host-permuted so that the N2
  // values of row k1 are contiguous): the packed diagonals take the tables
  // of states 0 and 1, the coupling transform the coupling table (stored
  // halved, twice)
  T mulA[I2][N2], mulB[I2][N2];
  {
    const unsigned tbytes = (unsigned)((long long)nq * NP * ES);
    const rsrc_t rt = make_rsrc(a.mtab, (unsigned)kWaveTables * tbytes);
#pragma unroll
    for (int t = 0; t < I2; ++t) {
      const int item = lane + 64 * t;
      const int f = item / N1, k1 = item % N1;
      const int kind = f / C;
      const int qc = min(q0 + f % C, nq - 1);
      const unsigned row = ((unsigned)qc * NP + (unsigned)k1 * N2) * ES;
      const unsigned oa = (kind ? 2u : 0u) * tbytes + row, ob = (kind ? 2u : 1u) * tbytes + row;
#pragma unroll
      for (int k2 = 0; k2 < N2; k2 += 4) {
        const Quad<T> qa = buf_load4(rt, oa + k2 * ES, 0, T(0));
        const Quad<T> qb = buf_load4(rt, ob + k2 * ES, 0, T(0));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          mulA[t][k2 + j] = qa.v[j];
          mulB[t][k2 + j] = qb.v[j];
        }
      }
    }
  }
  // q-dependent coupling: U_01(q + r/2), U_01(q - r/2) of this lane's rows.
  // In FP32 they are loaded here with the other multipliers; in FP64 they
  // are loaded four at a time inside the r-space loop, since holding all of
  // them through the forward passes would exceed the register budget.
  constexpr bool kQcEarly = QC && sizeof(T) == 4;
  const unsigned qc_tbytes = (unsigned)((long long)nq * NP * ES);
  const rsrc_t qc_rt = make_rsrc(a.mtab, (unsigned)kWaveTables * qc_tbytes);
  auto qc_row = [&](int t) {
    const int item = lane + 64 * t;
    const int f = item / N1, k1 = item % N1;
    const int qc = min(q0 + f % C, nq - 1);
    return ((unsigned)qc * NP + (unsigned)k1 * N2) * ES;
  };
  T cP[kQcEarly ? I2 : 1][kQcEarly ? N2 : 1], cM[kQcEarly ? I2 : 1][kQcEarly ? N2 : 1];
  if constexpr (kQcEarly) {
#pragma unroll
    for (int t = 0; t < I2; ++t) {
      const unsigned row = qc_row(t);
#pragma unroll
      for (int k2 = 0; k2 < N2; k2 += 4) {
        const Quad<T> qp = buf_load4(qc_rt, 3u * qc_tbytes + row + k2 * ES, 0, T(0));
        const Quad<T> qm = buf_load4(qc_rt, 4u * qc_tbytes + row + k2 * ES, 0, T(0));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cP[t][k2 + j] = qp.v[j];
          cM[t][k2 + j] = qm.v[j];
        }
      }
    }
  }
  // second forward pass: contiguous N2-point DFTs of row k1
#pragma unroll
  for (int t = 0; t < I2; ++t) {
    const int item = lane + 64 * t;
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
  wave_lds_sync();

  // r-space multiplication (position k2 + (N2+1) k1 holds index
  // m = k1 + N1 k2) and the first inverse pass; every lane reads its own and
  // its partner rows before any lane writes
  const T c0t = (has_up || clos) ? T(0) : c0;  // terminator level carries c0 D_p D_p
  cx<T> yk[I2][N2];
#pragma unroll
  for (int t = 0; t < I2; ++t) {
    const int item = lane + 64 * t;
    const int k1 = item % N1;
    const T* const re = re_of(item / N1);
    const T* const im = re + LDP;
    const T* zr = re + (N2 + 1) * k1;
    const T* zi = im + (N2 + 1) * k1;
    const int pbase = (k1 == 0) ? N2 : (N2 - 1) + (N2 + 1) * (N1 - k1);
    const T* pr = re + pbase;
    const T* pi = im + pbase;
    // the other transform of the same column (q-dependent coupling only)
    const int fi = item / N1, kind = fi / C;
    const T* const ore = re_of(fi % C + C * (1 - kind));
    const T* const ozr = ore + (N2 + 1) * k1;
    const T* const ozi = ore + LDP + (N2 + 1) * k1;
    const T* const opr = ore + pbase;
    const T* const opi = ore + LDP + pbase;
    const T hk = kind ? T(0.5) : T(1);
    Quad<T> qp4{}, qm4{};  // FP64: the coupling values of k2 .. k2 + 3
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      if constexpr (QC && !kQcEarly) {
        if (k2 % 4 == 0) {
          __builtin_amdgcn_sched_barrier(0);
          qp4 = buf_load4(qc_rt, 3u * qc_tbytes + qc_row(t) + k2 * ES, 0, T(0));
          qm4 = buf_load4(qc_rt, 4u * qc_tbytes + qc_row(t) + k2 * ES, 0, T(0));
        }
      }
      const cx<T> z = {zr[k2], zi[k2]};
      const cx<T> zp = {pr[-k2], -pi[-k2]};
      const T e = cdel * ssym[k1 + N1 * k2] + c0t * ssym[NP + k1 + N1 * k2];
      // Y = -i [ s Z[m] + d conj(Z[-m]) ] + e Z; the coupling transform has
      // mulA = mulB = g/2, so s = g and d = 0
      const T sA = mulA[t][k2] + mulB[t][k2], dA = mulA[t][k2] - mulB[t][k2];
      const cx<T> u = {sA * z.re + dA * zp.re, sA * z.im + dA * zp.im};
      yk[t][k2] = {u.im + e * z.re, -u.re + e * z.im};
      if constexpr (QC) {
        // Z, Z' = the other transform of this column at m and conj at -m:
        //   packed diagonals += (c+ + i c-) Z - (c- + i c+) Z'          (Z = coherence)
        //   coherence        += (-c+ + i c-)/2 Z + (c+ + i c-)/2 Z'     (Z = packed diagonals)
        const cx<T> zo = {ozr[k2], ozi[k2]};
        const cx<T> zop = {opr[-k2], -opi[-k2]};
        T cp, cm;
        if constexpr (kQcEarly) {
          cp = cP[t][k2];
          cm = cM[t][k2];
        } else {
          cp = qp4.v[k2 % 4];
          cm = qm4.v[k2 % 4];
        }
        const T xp = hk * cp, xm = hk * cm;
        const cx<T> al = {kind ? -xp : xp, xm};
        const cx<T> be = {kind ? xp : -xm, kind ? xm : -xp};
        yk[t][k2].re += al.re * zo.re - al.im * zo.im + be.re * zop.re - be.im * zop.im;
        yk[t][k2].im += al.re * zo.im + al.im * zo.re + be.re * zop.im + be.im * zop.re;
      }
    }
    SmallDft<N2, -1, T>::run(yk[t]);
  }
  wave_lds_sync();
#pragma unroll
  for (int t = 0; t < I2; ++t) {
    const int item = lane + 64 * t;
    const int k1 = item % N1;
    T* const zr = re_of(item / N1) + (N2 + 1) * k1;
    T* const zi = zr + LDP;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      const cx<T> g = cmulc(yk[t][n2], stw[k1 * (N2 + 1) + n2]);
      zr[n2] = g.re;
      zi[n2] = g.im;
    }
  }
  wave_lds_sync();

  // second inverse pass: N1-point DFTs over stride N2, natural order out
#pragma unroll
  for (int t = 0; t < I1; ++t) {
    const int item = lane + 64 * t;
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
      for (int j = 0; j < K; ++j) o[comp][j] = base[i][comp][j] + coef * s[(i * NC + comp) * LDP + pad(a0 + j)];
      // non-temporal stores (NTS) when the state arrays exceed the
      // memory-side cache: the output is read back only by the next stage
      // launch, from HBM anyway, and the stores then drain during the launch
      // instead of leaving dirty lines for the end-of-launch write-back
      buf_store_n<K, NTS ? kStoreNT : 0>(o[comp], ro, qo[i + 3], comp * cbytes);
    }
    if (want_trace) {
#pragma unroll
      for (int j = 0; j < K; ++j)
        tr += a.mu[0][0] * (double)o[0][j] + a.mu[1][1] * (double)o[1][j] + 2.0 * a.mu[0][1] * (double)o[2][j];
    }
  }
  if (want_trace) {
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
    if (lane == 0) a.partials[((long long)b * kRespSlots + a.slot) * a.ntiles + tile] = tr;
  }
}

// (MIX: members of their own depths, StageArgs::mlev)
template <typename T, int NP, bool QC, bool NTS, int WPB>
hipError_t launch_wave_one(const StageArgs& a, int nblocks, hipStream_t s) {
  if (a.mlev)
    hipLaunchKernelGGL((stage_wave_kernel<T, NP, QC, NTS, WPB, true>), dim3(nblocks), dim3(WavePlan<NP, WPB>::NT), 0, s,
                       a);
  else
    hipLaunchKernelGGL((stage_wave_kernel<T, NP, QC, NTS, WPB, false>), dim3(nblocks), dim3(WavePlan<NP, WPB>::NT), 0,
                       s, a);
  return hipGetLastError();
}

// instantiations: plain stores in both workgroup sizes and non-temporal
// stores (large states, so large launches) with four waves per workgroup for
// a constant coupling; four waves per workgroup for a q-dependent one (two
// would make the compiler trade registers for a higher occupancy and spill)
template <typename T, int NP, bool QC>
hipError_t launch_wave_np(const StageArgs& a, int nblocks, hipStream_t s) {
  if constexpr (!QC) {
    if (a.wpb == kWaveTasksPerBlockSmall)
      return launch_wave_one<T, NP, false, false, kWaveTasksPerBlockSmall>(a, nblocks, s);
    if (a.wpb != kWaveTasksPerBlock) return hipErrorInvalidValue;
    if (a.stream_out) return launch_wave_one<T, NP, false, true, kWaveTasksPerBlock>(a, nblocks, s);
    return launch_wave_one<T, NP, false, false, kWaveTasksPerBlock>(a, nblocks, s);
  } else {
    if (a.wpb != kWaveTasksPerBlock) return hipErrorInvalidValue;
    return launch_wave_one<T, NP, true, false, kWaveTasksPerBlock>(a, nblocks, s);
  }
}

template <typename T>
hipError_t launch_stage_wave(int np, const StageArgs& a, int nblocks, hipStream_t s) {
  switch (np * 2 + (a.qcoup ? 1 : 0)) {
    case 256: return launch_wave_np<T, 128, false>(a, nblocks, s);
    case 257: return launch_wave_np<T, 128, true>(a, nblocks, s);
    case 512: return launch_wave_np<T, 256, false>(a, nblocks, s);
    case 513: return launch_wave_np<T, 256, true>(a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qhfpe
