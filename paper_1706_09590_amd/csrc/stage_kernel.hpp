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
// The constant diabatic couplings are a pointwise commutator in p-space; a
// q-dependent coupling (the QC instantiation, 2 cells per thread) enters
// the r-space multiply instead, where it mixes the transforms of a column.
//
// State layout (packed reals): [member][level][comp][q][p], p fastest.
#pragma once

#include "device_common.hpp"
#include "qhfpe_internal.hpp"

namespace qhfpe {

// FFT split np = N1 * N2 per supported np.
template <int NP>
struct FftSplit;
#define QHFPE_SPLIT(NP_, N1_, N2_) \
  template <>                      \
  struct FftSplit<NP_> {           \
    static constexpr int N1 = N1_, N2 = N2_; \
  };
QHFPE_SPLIT(8, 4, 2)
QHFPE_SPLIT(12, 4, 3)
QHFPE_SPLIT(16, 4, 4)
QHFPE_SPLIT(24, 6, 4)
QHFPE_SPLIT(32, 8, 4)
QHFPE_SPLIT(48, 8, 6)
QHFPE_SPLIT(64, 8, 8)
QHFPE_SPLIT(96, 12, 8)
QHFPE_SPLIT(128, 16, 8)
QHFPE_SPLIT(192, 16, 12)
QHFPE_SPLIT(256, 16, 16)
#undef QHFPE_SPLIT

// Launch shape of the stage kernel: NT = np * G threads, TQ = G * CPT columns.
template <typename T, int NS, int NP, int CPT_>
struct PlanOf {
  static constexpr int N1 = FftSplit<NP>::N1, N2 = FftSplit<NP>::N2;
  static constexpr int G = plan_groups(NP);
  static constexpr int NT = NP * G;
  static constexpr int CPT = CPT_;
  static constexpr int TQ = G * CPT;
};

// One complex transform of a tile: real part from (colA, compA), imaginary
// part from (colB, compB); kind 0 packs two real diagonal components of
// states sj and sk, kind 1 is the off-diagonal pair (sj, sk).
struct FftItem {
  int colA, compA, colB, compB, kind, sj, sk;
};

// Upwind coefficients (x60) for p >= 0 on offsets -3..2; the p < 0 stencil
// is the mirror image with opposite sign (Sec. III).
__device__ constexpr double kUpwind[6] = {-2.0, 15.0, -60.0, 20.0, 30.0, -3.0};

// Hardware block ids are dealt round-robin over the 8 XCDs; this maps them
// so that each XCD receives one contiguous range of logical blocks (whole
// q tiles with all their levels), so halo and level reads hit that XCD's L2.
__device__ __forceinline__ int xcd_logical_block(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int per = (nblocks + kXcd - 1) / kXcd;
  return (bid % kXcd) * per + bid / kXcd;
}

// q-dependent couplings (QC instantiation).  The r-space matrix of one tile
// column at index m: the diagonals separated from their packed transforms
// (H_00 + i H_11 of the column; for three states H_22 from the transform
// that packs the W22 of the column pair c & ~1, c | 1), the coherences
// H_jk (j < k) from their own transforms, and H_kj(m) = conj H_jk(-m).
// pm, pp: LDS positions of m and -m within a column.
template <typename T, int NS>
__device__ __forceinline__ void rspace_matrix(const T* sv, int ldp, int c, int pm, int pp, cx<T> (&H)[NS][NS]) {
  constexpr int NC = NS * NS;
  const T* d0 = sv + (c * NC + 0) * ldp;
  const T* d1 = d0 + ldp;
  {
    const cx<T> z = {d0[pm], d1[pm]}, zc = {d0[pp], -d1[pp]};  // Z(m), conj Z(-m)
    H[0][0] = {T(0.5) * (z.re + zc.re), T(0.5) * (z.im + zc.im)};
    H[1][1] = {T(0.5) * (z.im - zc.im), T(-0.5) * (z.re - zc.re)};  // (Z - conj Z(-m)) / 2i
  }
  if constexpr (NS == 3) {
    const T* a2 = sv + ((c & ~1) * NC + 2) * ldp;
    const T* b2 = sv + ((c | 1) * NC + 2) * ldp;
    const cx<T> z = {a2[pm], b2[pm]}, zc = {a2[pp], -b2[pp]};
    H[2][2] = (c & 1) ? cx<T>{T(0.5) * (z.im - zc.im), T(-0.5) * (z.re - zc.re)}
                      : cx<T>{T(0.5) * (z.re + zc.re), T(0.5) * (z.im + zc.im)};
  }
#pragma unroll
  for (int j = 0; j < NS; ++j)
#pragma unroll
    for (int k = j + 1; k < NS; ++k) {
      const T* r = sv + (c * NC + Packing<NS>::re(j, k)) * ldp;
      const T* i = r + ldp;
      H[j][k] = {r[pm], i[pm]};
      H[k][j] = {r[pp], -i[pp]};
    }
}

// The coupling part of the potential term in r space at one column and m:
//   C_jk = -i [ sum_{l != j} up_jl H_lk - sum_{l != k} H_jl um_lk ]
// with up_jl = U_jl(q + r/2) / (hbar np), um_jl = U_jl(q - r/2) / (hbar np)
// (off-diagonal surfaces only; the diagonal ones are in the multipliers).
template <typename T, int NS>
__device__ __forceinline__ cx<T> coupling_rspace(const cx<T> (&H)[NS][NS], const T (&up)[NS][NS],
                                                 const T (&um)[NS][NS], int j, int k) {
  cx<T> s = {T(0), T(0)};
#pragma unroll
  for (int jj = 0; jj < NS; ++jj)
#pragma unroll
    for (int kk = 0; kk < NS; ++kk) {
      if (jj != j || kk != k) continue;
#pragma unroll
      for (int l = 0; l < NS; ++l) {
        if (l != jj) {
          s.re += up[jj][l] * H[l][kk].re;
          s.im += up[jj][l] * H[l][kk].im;
        }
        if (l != kk) {
          s.re -= H[jj][l].re * um[l][kk];
          s.im -= H[jj][l].im * um[l][kk];
        }
      }
    }
  return {s.im, -s.re};
}

// Position of stage unit t of a launch (a task of the wave variants, a
// workgroup of this one): levels fastest, then q tiles, then members.  MIX:
// members have depths of their own (StageArgs::mlev): member b owns
// ntiles * (its levels) consecutive units, and every row of ntiles units
// belongs to one member.  (A compile-time switch: the lookup's dependent
// scalar loads would otherwise lengthen every wave's start.)
struct UnitPos {
  int b, tile, n, depth;
};
template <bool MIX>
__device__ __forceinline__ int stage_units(const StageArgs& a) {
  if constexpr (MIX) return a.ntiles * (a.mlev[a.mfirst + a.batch] - a.mlev[a.mfirst]);
  return a.ntiles * (a.depth + 1) * a.batch;
}
template <bool MIX>
__device__ __forceinline__ UnitPos unit_pos(const StageArgs& a, int t) {
  UnitPos u;
  if constexpr (!MIX) {
    const int L = a.depth + 1;
    u.n = t % L;
    u.tile = (t / L) % a.ntiles;
    u.b = t / (L * a.ntiles);
    u.depth = a.depth;
    return u;
  }
  const int tg = t + a.ntiles * a.mlev[a.mfirst];
  const int bg = a.lev_member[tg / a.ntiles];
  const int r0 = a.mlev[bg], L = a.mlev[bg + 1] - r0;
  const int local = tg - a.ntiles * r0;
  u.n = local % L;
  u.tile = local / L;
  u.b = bg - a.mfirst;
  u.depth = L - 1;
  return u;
}

template <typename T, int NS, int NP, int CPT_, bool QC = false, bool MIX = false>
__global__ void __launch_bounds__((PlanOf<T, NS, NP, CPT_>::NT), 2) stage_kernel(StageArgs a) {
  using P = PlanOf<T, NS, NP, CPT_>;
  constexpr int N1 = P::N1, N2 = P::N2, TQ = P::TQ, NT = P::NT, CPT = P::CPT;
  constexpr int NC = NS * NS;
  constexpr int NPAIR = NS * (NS - 1) / 2;
  // complex transforms per tile: diagonal pairs (0,1) per column, (2 of c,
  // 2 of c+1) per column pair when NS = 3, and each off-diagonal pair.
  constexpr int NFFT = TQ + (NS == 3 ? TQ / 2 : 0) + NPAIR * TQ;
  static_assert(NS == 2 || TQ % 2 == 0, "three-state tiles pair columns");

  // LDS columns are padded by one element per N2 block (index a + a / N2),
  // so the FFT passes that walk a column with stride N2 are free of bank
  // conflicts; the column stride is then rounded to 4 (mod 16) elements so
  // that the transforms of neighbouring columns, which share a wave, start
  // on different banks.
  constexpr int LDP0 = NP + NP / N2;
  constexpr int LDP = (NP >= 64) ? LDP0 + ((4 - LDP0 % 16) + 16) % 16 : LDP0;
  __shared__ T sv[TQ * NC * LDP];   // v^(n) tile, then the potential term in place
  __shared__ T sg[TQ * NC * LDP];   // field differentiated once along p, then the potential term
  __shared__ cx<T> stw[N1 * (N2 + 1)];  // w^(n2 k1), row k1 padded to N2 + 1
  __shared__ T ssym[2 * NP];            // DFT symbols of D_p2 and D_p D_p (scaled by 1/np)

  const int nblocks = stage_units<MIX>(a);
  const int lb = xcd_logical_block(blockIdx.x, a.nblocks_padded);
  if (lb >= nblocks) return;
  const int tid = threadIdx.x;
  // levels run fastest: the blocks of every level of one q tile are
  // resident together, so the reads of v^(n) by levels n - 1 and n + 1
  // hit the copy that level n's own block brought into L2
  const UnitPos pos = unit_pos<MIX>(a, lb);
  const int n = pos.n, tile = pos.tile, b = pos.b;
  const int q0 = tile * TQ;
  const int nq = a.nq;
  const int ia = tid % NP;           // this thread's p node
  const int iap = ia + ia / N2;      // its padded LDS index
  const int cb = (tid / NP) * CPT;   // first of its CPT tile columns
  const unsigned cs = (unsigned)a.comp_stride;

  // buffer resources over whole levels of this member: the per-lane byte
  // offset addresses (q, p), the uniform soffset selects the component
  constexpr unsigned ES = sizeof(T);
  const unsigned level_bytes = (unsigned)(a.level_stride * ES);
  const T* vm = static_cast<const T*>(a.v) + (long long)b * a.member_stride;
  const bool has_up = n < pos.depth, has_dn = n >= 1;
  const rsrc_t rn = make_rsrc(vm + (long long)n * a.level_stride, level_bytes);
  const rsrc_t ru = make_rsrc(vm + (long long)(has_up ? n + 1 : n) * a.level_stride, level_bytes);
  const rsrc_t rd = make_rsrc(vm + (long long)(has_dn ? n - 1 : n) * a.level_stride, level_bytes);
  const bool has_y = a.y != nullptr;
  const rsrc_t ry = make_rsrc(has_y ? static_cast<const T*>(a.y) + (long long)b * a.member_stride +
                                          (long long)n * a.level_stride
                                    : vm,
                              has_y ? level_bytes : 0u);
  const unsigned cbytes = cs * ES;   // soffset step per packed component

  // the twiddle and symbol tables are loaded first and stored to LDS just
  // before the first barrier, so that their latency overlaps phase P1 (the
  // loads complete in issue order: by then P1 has waited for later ones).
  // Lanes past a table's end load its last entry and store nothing.
  constexpr int NTW = N1 * (N2 + 1), NSY = 2 * NP;
  constexpr int RTW = (NTW + NT - 1) / NT, RSY = (NSY + NT - 1) / NT;
  T twr[RTW][2], syr[RSY];
#pragma unroll
  for (int r = 0; r < RTW; ++r) {
    const T* const t = static_cast<const T*>(a.twiddle2) + 2 * min(tid + r * NT, NTW - 1);
    twr[r][0] = t[0];
    twr[r][1] = t[1];
  }
#pragma unroll
  for (int r = 0; r < RSY; ++r) syr[r] = static_cast<const T*>(a.psym)[min(tid + r * NT, NSY - 1)];

  const T p = T(a.p0 + ia * a.dp);
  const double* bath = a.bath + kBathStride * b;
  const T zeta = T(bath[0]), c0 = T(bath[2]), cdel = T(bath[3]);
  const T ng = T(n * bath[1]);
  // kinetic term -(p/m) D_q with the upwind stencil chosen by the sign of p:
  // coefficients on q offsets -3..3 (one end is zero for either sign)
  T kc[7];
  {
    const T scale = -(p * T(a.inv_mass)) * T(1.0 / (60.0 * a.dq));
    const bool pos = p >= T(0);
#pragma unroll
    for (int o = -3; o <= 3; ++o) {
      const double cp = (o <= 2) ? kUpwind[o + 3] : 0.0;
      const double cn = (o >= -2) ? -kUpwind[3 - o] : 0.0;
      kc[o + 3] = scale * T(pos ? cp : cn);
    }
  }

  // ---- P1: all global loads of this thread, then local terms -------------
  // byte offsets of this thread's p node in the q columns cb-3 .. cb+CPT+2,
  // clamped to the grid; tiles that touch the q edges mask the ghost
  // columns to zero (a uniform branch)
  T acc[CPT][NC];
  T hv[CPT][NC];  // v^(n) at this thread's cells (for the pointwise coupling)
  unsigned qo[CPT + 6];
  bool qin[CPT + 6];
  const bool edge = (q0 - 3 < 0) || (q0 + TQ + 3 > nq);
#pragma unroll
  for (int j = 0; j < CPT + 6; ++j) {
    const int q = q0 + cb + j - 3;
    qin[j] = (q >= 0) && (q < nq);
    qo[j] = ((unsigned)(q < 0 ? 0 : (q >= nq ? nq - 1 : q)) * NP + ia) * ES;
  }
  // components are processed in groups of LGRP; the scheduling barrier keeps
  // the next group's loads from being hoisted, which bounds register use.
  // FP64 tiles are held to two workgroups per CU by LDS, which leaves room
  // for all loads at once, and so are three-state FP32 tiles (three per CU;
  // all loads at once measured 2% faster there); two-state FP32 runs four
  // workgroups and loads in halves.
  constexpr int LGRP = (sizeof(T) == 8 || NS == 3) ? NC : 2;
#pragma unroll
  for (int comp = 0; comp < NC; ++comp) {
    if (comp % LGRP == 0 && comp > 0) __builtin_amdgcn_sched_barrier(0);
    const unsigned so = comp * cbytes;
    T w[CPT + 6];
#pragma unroll
    for (int j = 0; j < CPT + 6; ++j) w[j] = buf_load<T>(rn, qo[j], so);
    if (edge) {
#pragma unroll
      for (int j = 0; j < CPT + 6; ++j) w[j] = qin[j] ? w[j] : T(0);
    }
    T up[CPT], dn[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      up[i] = buf_load<T>(ru, qo[i + 3], so);
      dn[i] = buf_load<T>(rd, qo[i + 3], so);
    }
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      T f = T(0);
#pragma unroll
      for (int o = 0; o < 7; ++o) f += kc[o] * w[i + o];
      const T w0 = w[i + 3];
      f -= ng * w0;
      // field differentiated once along p:
      //   n < N: v^(n+1) + n gamma c0 v^(n-1);  n = N: zeta p v^(N) + N gamma c0 v^(N-1)
      T g = has_up ? up[i] : zeta * p * w0;
      if (has_dn) {
        g += ng * c0 * dn[i];
        f += ng * zeta * p * dn[i];
      }
      acc[i][comp] = f;
      hv[i][comp] = w0;
      sv[((cb + i) * NC + comp) * LDP + iap] = w0;
      sg[((cb + i) * NC + comp) * LDP + iap] = (!edge || qin[i + 3]) ? g : T(0);
    }
  }
  // constant diabatic couplings: -(i/hbar) [Delta, W], pointwise in p
  {
    T coup[NS][NS];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int k = 0; k < NS; ++k) coup[j][k] = T(a.coup[j][k]);
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      T cm[NC];
      commutator_mi<NS, T>(coup, hv[i], cm);
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) acc[i][comp] += cm[comp];
    }
  }
  // materialise the local terms here: otherwise their arithmetic is sunk to
  // the final combine and every loaded q-window stays live across the barriers
#pragma unroll
  for (int i = 0; i < CPT; ++i)
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) asm volatile("" : "+v"(acc[i][comp]));
  // the RK base state y is fetched now, so that its latency overlaps the
  // barrier and the stencil of P2
  T base[CPT][NC];
#pragma unroll
  for (int i = 0; i < CPT; ++i)
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) base[i][comp] = buf_load<T>(ry, qo[i + 3], comp * cbytes);
#pragma unroll
  for (int r = 0; r < RTW; ++r) {
    const int j = tid + r * NT;
    if (j < NTW) stw[j] = cx<T>{twr[r][0], twr[r][1]};
  }
#pragma unroll
  for (int r = 0; r < RSY; ++r) {
    const int j = tid + r * NT;
    if (j < NSY) ssym[j] = syr[r];
  }
  __syncthreads();

  // ---- P2: D_p of the level-coupling field -------------------------------
  // (the periodic p-stencils acting on v^(n) itself, c_delta D_p2 and the
  // terminator's c0 D_p D_p, are applied in the DFT domain in P5).
  // base = y + coef * (local terms) stays in registers until the combine.
  // P2 reads only sg and the first FFT pass (P3) only sv, so the two share
  // one phase.
  {
    const T dpinv = T(1.0 / (12.0 * a.dp));
    const T coef = T(a.coef);
    auto pd = [](int x) { return x + x / N2; };
    const int am1 = pd((ia + NP - 1) % NP), am2 = pd((ia + NP - 2) % NP);
    const int ap1 = pd((ia + 1) % NP), ap2 = pd((ia + 2) % NP);
#pragma unroll
    for (int i = 0; i < CPT; ++i)
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) {
        const T* gg = sg + ((cb + i) * NC + comp) * LDP;
        const T f = acc[i][comp] + dpinv * (-gg[ap2] + T(8) * gg[ap1] - T(8) * gg[am1] + gg[am2]);
        base[i][comp] += coef * f;
      }
  }
  // materialise base now, so the stencil operands are not kept live through
  // the transforms
#pragma unroll
  for (int i = 0; i < CPT; ++i)
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) asm volatile("" : "+v"(base[i][comp]));

  // ---- P3..P6: potential term (in place in sv, then sg) -------------------
  // Transform f takes its real part from one packed component column and its
  // imaginary part from another.
  // (returned by value: out-parameters here were demoted to scratch memory)
  auto fft_desc = [](int f) {
    FftItem d;
    if (f < TQ) {  // diagonal pair (0, 1) of column f
      d.colA = d.colB = f;
      d.compA = 0;
      d.compB = 1;
      d.kind = 0;
      d.sj = 0;
      d.sk = 1;
      return d;
    }
    f -= TQ;
    if (NS == 3 && f < TQ / 2) {  // diagonal 2 of columns 2f and 2f + 1
      d.colA = 2 * f;
      d.colB = 2 * f + 1;
      d.compA = d.compB = 2;
      d.kind = 0;
      d.sj = d.sk = 2;
      return d;
    }
    if (NS == 3) f -= TQ / 2;
    const int pr = f % NPAIR;  // off-diagonal pair (j, k) of column f / NPAIR
    d.colA = d.colB = f / NPAIR;
    d.sj = (pr < NS - 1) ? 0 : 1;
    d.sk = (pr == 0) ? 1 : 2;
    d.compA = NS + 2 * pr;
    d.compB = d.compA + 1;
    d.kind = 1;
    return d;
  };

  // P3: first forward pass, item (f, n2): N1-point DFTs over stride N2.
  constexpr int ITEMS3 = NFFT * N2;
#pragma unroll
  for (int t = 0; t < (ITEMS3 + NT - 1) / NT; ++t) {
    const int it = tid + t * NT;
    if (it >= ITEMS3) continue;
    const int f = it / N2, n2 = it % N2;
    const FftItem d = fft_desc(f);
    const int colA = d.colA, compA = d.compA, colB = d.colB, compB = d.compB, kind = d.kind;
    T* re = sv + (colA * NC + compA) * LDP;
    T* im = sv + (colB * NC + compB) * LDP;
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
  __syncthreads();

  // P4: second forward pass, item (f, k1): contiguous N2-point DFTs.  The
  // r-space multipliers that this thread needs in P5 (same item) are
  // fetched here so their latency overlaps the DFT work.
  constexpr int ITEMS5 = NFFT * N1;
  constexpr int IPT5 = (ITEMS5 + NT - 1) / NT;
  T mulA[IPT5][N2], mulB[IPT5][N2];
  {
    const unsigned tbytes = (unsigned)((long long)nq * NP * ES);  // one multiplier table
    const rsrc_t rdt = make_rsrc(a.dtab, NS * tbytes);
    const rsrc_t rgt = make_rsrc(a.gtab, NPAIR * tbytes);
#pragma unroll
    for (int t = 0; t < IPT5; ++t) {
      const int it = tid + t * NT;
      const int f = (it < ITEMS5 ? it : 0) / N1, k1 = it % N1;
      const FftItem d = fft_desc(f);
      const int colA = d.colA, colB = d.colB, kind = d.kind, sj = d.sj, sk = d.sk;
      const int qa = min(q0 + colA, nq - 1), qb = min(q0 + colB, nq - 1);
      const unsigned oa = ((unsigned)qa * NP + k1) * ES, ob = ((unsigned)qb * NP + k1) * ES;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        if (kind == 0) {
          mulA[t][k2] = buf_load<T>(rdt, oa + N1 * k2 * ES, sj * tbytes);
          mulB[t][k2] = buf_load<T>(rdt, ob + N1 * k2 * ES, sk * tbytes);
        } else {
          mulA[t][k2] = buf_load<T>(rgt, oa + N1 * k2 * ES, (sj + sk - 1) * tbytes);
          mulB[t][k2] = T(0);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < IPT5; ++t) {
    const int it = tid + t * NT;
    if (it >= ITEMS5) continue;
    const int f = it / N1, k1 = it % N1;
    const FftItem d = fft_desc(f);
    const int colA = d.colA, compA = d.compA, colB = d.colB, compB = d.compB, kind = d.kind;
    T* re = sv + (colA * NC + compA) * LDP + (N2 + 1) * k1;
    T* im = sv + (colB * NC + compB) * LDP + (N2 + 1) * k1;
    cx<T> x[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) x[n2] = {re[n2], im[n2]};
    SmallDft<N2, 1, T>::run(x);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      re[k2] = x[k2].re;
      im[k2] = x[k2].im;
    }
    // block 0 also stores X[0] in its padding slot, so that the partner of
    // index m lies at base - k2 for every block (see P5)
    if (k1 == 0) {
      re[N2] = x[0].re;
      im[N2] = x[0].im;
    }
  }
  __syncthreads();

  // P5: r-space multiplication (position k2 + (N2+1) k1 holds index
  // m = k1 + N1 k2), then the first inverse pass over k2 and its twiddle;
  // results stay in registers until every thread has read its partner values.
  const T c0t = has_up ? T(0) : c0;  // terminator level carries c0 D_p D_p
#pragma unroll
  for (int t = 0; t < IPT5; ++t) {
    const int it = tid + t * NT;
    if (it >= ITEMS5) continue;
    const int f = it / N1, k1 = it % N1;
    const FftItem d = fft_desc(f);
    const int colA = d.colA, compA = d.compA, colB = d.colB, compB = d.compB, kind = d.kind;
    const T* re = sv + (colA * NC + compA) * LDP;
    const T* im = sv + (colB * NC + compB) * LDP;
    const T* zr = re + (N2 + 1) * k1;
    const T* zi = im + (N2 + 1) * k1;
    // partner -m of m = k1 + N1 k2 sits at position pbase - k2 (block
    // N1 - k1 read backwards; block 0 pairs within itself via its padding copy)
    const int pbase = (k1 == 0) ? N2 : (N2 - 1) + (N2 + 1) * (N1 - k1);
    const T* pr = re + pbase;
    const T* pi = im + pbase;
    const T* sy = ssym + k1;
    cx<T> y[N2];
    // QC: the coupling surfaces of the transform's column(s) at this row
    const unsigned tb = (unsigned)((long long)nq * NP * ES);
    const rsrc_t rct = make_rsrc(a.ctab, QC ? 2u * NPAIR * tb : 0u);
    const int qA = min(q0 + colA, nq - 1), qB = min(q0 + colB, nq - 1);
    auto surfaces = [&](int q, int k2, T (&up)[NS][NS], T (&um)[NS][NS]) {
      const unsigned off = ((unsigned)q * NP + (unsigned)(k1 + N1 * k2)) * ES;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        up[j][j] = um[j][j] = T(0);
#pragma unroll
        for (int k = j + 1; k < NS; ++k) {
          const int pr = Packing<NS>::pair(j, k);
          up[j][k] = up[k][j] = buf_load<T>(rct, off, (2 * pr) * tb);
          um[j][k] = um[k][j] = buf_load<T>(rct, off, (2 * pr + 1) * tb);
        }
      }
    };
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const cx<T> z = {zr[k2], zi[k2]};
      // real, even symbol of the p-stencils that act on v^(n) in every component
      const T e = cdel * sy[N1 * k2] + c0t * sy[NP + N1 * k2];
      if (kind == 0) {
        // two real sequences in one transform: Y = -i [ s Z[m] + d conj(Z[-m]) ]
        const cx<T> zp = {pr[-k2], -pi[-k2]};
        const T sA = mulA[t][k2] + mulB[t][k2], dA = mulA[t][k2] - mulB[t][k2];
        const cx<T> u = {sA * z.re + dA * zp.re, sA * z.im + dA * zp.im};
        y[k2] = {u.im + e * z.re, -u.re + e * z.im};
      } else {
        // Y = -i g Z
        const T gg = mulA[t][k2];
        y[k2] = {gg * z.im + e * z.re, -gg * z.re + e * z.im};
      }
      if constexpr (QC) {
        const int pm = (N2 + 1) * k1 + k2, pp = pbase - k2;
        cx<T> H[NS][NS];
        T up[NS][NS], um[NS][NS];
        rspace_matrix<T, NS>(sv, LDP, colA, pm, pp, H);
        surfaces(qA, k2, up, um);
        if (kind == 1) {
          y[k2] = y[k2] + coupling_rspace<T, NS>(H, up, um, d.sj, d.sk);
        } else if (d.sj == 0) {
          // packed diagonals of one column: C_00 + i C_11
          const cx<T> c00 = coupling_rspace<T, NS>(H, up, um, 0, 0), c11 = coupling_rspace<T, NS>(H, up, um, 1, 1);
          y[k2] = y[k2] + cx<T>{c00.re - c11.im, c00.im + c11.re};
        } else {
          // W22 of two columns: C_22 of colA + i C_22 of colB
          const cx<T> ca = coupling_rspace<T, NS>(H, up, um, NS - 1, NS - 1);
          rspace_matrix<T, NS>(sv, LDP, colB, pm, pp, H);
          surfaces(qB, k2, up, um);
          const cx<T> cb2 = coupling_rspace<T, NS>(H, up, um, NS - 1, NS - 1);
          y[k2] = y[k2] + cx<T>{ca.re - cb2.im, ca.im + cb2.re};
        }
      }
    }
    SmallDft<N2, -1, T>::run(y);
    // the result goes to the same positions of sg (sv still holds partner
    // values other threads are reading)
    T* ore = sg + (colA * NC + compA) * LDP + (N2 + 1) * k1;
    T* oim = sg + (colB * NC + compB) * LDP + (N2 + 1) * k1;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      const cx<T> g = cmulc(y[n2], stw[k1 * (N2 + 1) + n2]);
      ore[n2] = g.re;
      oim[n2] = g.im;
    }
  }
  __syncthreads();

  // P6: second inverse pass, item (f, n2): N1-point DFTs over stride N2,
  // natural order out (in place in sg).
#pragma unroll
  for (int t = 0; t < (ITEMS3 + NT - 1) / NT; ++t) {
    const int it = tid + t * NT;
    if (it >= ITEMS3) continue;
    const int f = it / N2, n2 = it % N2;
    const FftItem d = fft_desc(f);
    const int colA = d.colA, compA = d.compA, colB = d.colB, compB = d.compB, kind = d.kind;
    T* re = sg + (colA * NC + compA) * LDP;
    T* im = sg + (colB * NC + compB) * LDP;
    cx<T> x[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) x[k1] = {re[n2 + (N2 + 1) * k1], im[n2 + (N2 + 1) * k1]};
    SmallDft<N1, -1, T>::run(x);
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      re[n2 + (N2 + 1) * n1] = x[n1].re;
      im[n2 + (N2 + 1) * n1] = x[n1].im;
    }
  }
  __syncthreads();

  // ---- P7: combine, write, level-0 trace partial -------------------------
  const rsrc_t ro = make_rsrc(static_cast<T*>(a.out) + (long long)b * a.member_stride + (long long)n * a.level_stride,
                              level_bytes);
  const T coef = T(a.coef);
  const bool want_trace = (a.partials != nullptr) && (n == 0);
  double tr = 0.0;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int q = q0 + cb + i;
    if (q >= nq) continue;
    T o[NC];
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) {
      o[comp] = base[i][comp] + coef * sg[((cb + i) * NC + comp) * LDP + iap];
      buf_store(o[comp], ro, qo[i + 3], comp * cbytes);
    }
    if (want_trace) {
#pragma unroll
      for (int j = 0; j < NS; ++j) tr += a.mu[j][j] * (double)o[j];
#pragma unroll
      for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int k = j + 1; k < NS; ++k) tr += 2.0 * a.mu[j][k] * (double)o[Packing<NS>::re(j, k)];
    }
  }
  if (want_trace) {
    // deterministic workgroup sum: wave butterfly, then fixed order over waves
    constexpr int NW = (NT + 63) / 64;
    __shared__ double wsum[NW];
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = tr;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += wsum[w];
      a.partials[((long long)b * kRespSlots + a.slot) * a.ntiles + tile] = s;
    }
  }
}

template <typename T, int NS, int NP, int CPT, bool QC = false>
hipError_t launch_stage_variant(const StageArgs& a, int nblocks, hipStream_t s) {
  if constexpr (cpt_supported_c((int)sizeof(T), NS, CPT)) {
    if (a.mlev)
      hipLaunchKernelGGL((stage_kernel<T, NS, NP, CPT, QC, true>), dim3(nblocks), dim3(PlanOf<T, NS, NP, CPT>::NT), 0,
                         s, a);
    else
      hipLaunchKernelGGL((stage_kernel<T, NS, NP, CPT, QC, false>), dim3(nblocks), dim3(PlanOf<T, NS, NP, CPT>::NT), 0,
                         s, a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

// a q-dependent coupling has one variant, kQcCpt cells per thread
template <typename T, int NS, int NP>
hipError_t launch_stage_np(int cpt, const StageArgs& a, int nblocks, hipStream_t s) {
  if (a.qcoup) return cpt == kQcCpt ? launch_stage_variant<T, NS, NP, kQcCpt, true>(a, nblocks, s) : hipErrorInvalidValue;
  switch (cpt) {
    case 2:
      return launch_stage_variant<T, NS, NP, 2>(a, nblocks, s);
    case 4:
      return launch_stage_variant<T, NS, NP, 4>(a, nblocks, s);
    case 8:
      return launch_stage_variant<T, NS, NP, 8>(a, nblocks, s);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, int NS>
hipError_t launch_stage(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s) {
  switch (np) {
#define QHFPE_CASE(NP_) \
  case NP_:             \
    return launch_stage_np<T, NS, NP_>(cpt, a, nblocks, s);
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
