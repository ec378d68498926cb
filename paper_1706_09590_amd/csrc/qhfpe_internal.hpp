// Internal declarations shared by the host API and the kernels of the
// MS-QHFPE library.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "qhfpe.h"

namespace qhfpe {

constexpr int kBlock = 256;        // threads per workgroup of every grid kernel
constexpr int kRespSlots = 256;    // response samples buffered between finalisations
constexpr int kBathStride = 8;     // doubles per member in the bath table

// Two-pass FFT plan along p (np = n1 * n2, n1 even) for every supported np.
struct Plan {
  int np, n1, n2;
};
constexpr Plan kPlans[] = {
    {8, 4, 2},   {12, 4, 3},  {16, 4, 4},   {24, 6, 4},    {32, 8, 4},    {48, 8, 6},
    {64, 8, 8},  {96, 12, 8}, {128, 16, 8}, {192, 16, 12}, {256, 16, 16},
};
inline const Plan* find_plan(int np) {
  for (const Plan& p : kPlans)
    if (p.np == np) return &p;
  return nullptr;
}

// Stage workgroup shape: G = max(1, 256/np) groups of np threads; each
// thread owns one p node of CPT consecutive q columns; a tile is TQ = G*CPT
// columns (even, so three-state tiles can pair columns).  CPT is a tuning
// variant: 2, 4 or 8 for FP32 two-state; 2 or 4 for FP64 two-state and FP32
// three-state; 2 for FP64 three-state (larger LDS tiles would not fit).
constexpr int plan_groups(int np) { return np >= 256 ? 1 : 256 / np; }
constexpr int kMinCpt = 2;
// The workgroup variant with a q-dependent coupling (the coupling surfaces
// in the r-space multiply) exists for 2 cells per thread only.
constexpr int kQcCpt = 2;
constexpr bool cpt_supported_c(int elem_bytes, int ns, int cpt) {
  return (ns == 2) ? (cpt == 2 || cpt == 4 || (cpt == 8 && elem_bytes == 4))
                   : (elem_bytes == 8 ? cpt == 2 : (cpt == 2 || cpt == 4));
}
inline bool cpt_supported(int elem_bytes, int ns, int cpt) { return cpt_supported_c(elem_bytes, ns, cpt); }
// Three states: 2 cells per thread in both precisions (with 4, the LDS of a
// 256-thread workgroup leaves room for one workgroup per CU at np = 256).
inline int cpt_default(int /*elem_bytes*/, int ns) { return (ns == 3) ? 2 : 4; }

// Tile code of the wave-independent stage variant (stage_wave.hpp): one
// wave per 512/np q columns, two states and np = 128 or 256.
constexpr int kTileWave = 1;
constexpr int kMaxGroups = 4;  // member groups (streams) of qhfpe_step
constexpr int kWaveTables = 5;  // multiplier planes of the wave variant
// Waves per workgroup of the wave variant: four share the twiddle and symbol
// tables in LDS; launches of at most kWaveSmallTasks tasks (one round on the
// GPU) use two, whose finer workgroups spread the waves more evenly over the
// CUs and so shorten the launch's tail.
constexpr int kWaveTasksPerBlock = 4;
constexpr int kWaveTasksPerBlockSmall = 2;
constexpr int kWaveSmallTasks = 2048;
inline bool wave_supported(int ns, int np) { return ns == 2 && (np == 128 || np == 256); }
// q columns per task of the wave variant (a lane holds np / 64 p nodes)
constexpr int wave_columns(int np) { return 512 / np; }
// The three-state wave variant (stage_wave3.hpp): np = 128 or 256, constant
// couplings only, six multiplier planes; two q columns per task at np = 128,
// one at np = 256 (LDS: 11 KB per FP32 wave instead of 20).
constexpr int wave3_columns(int np) { return np == 256 ? 1 : 2; }
constexpr int kWaveTables3 = 6;
inline bool wave3_supported(int /*elem_bytes*/, int np) { return np == 128 || np == 256; }
inline bool wave_variant_supported(int elem_bytes, int ns, int np) {
  return ns == 2 ? wave_supported(ns, np) : wave3_supported(elem_bytes, np);
}
inline int wave_columns_of(int ns, int np) { return ns == 3 ? wave3_columns(np) : wave_columns(np); }
inline int wave_table_planes(int ns) { return ns == 3 ? kWaveTables3 : kWaveTables; }
// Waves per workgroup of a three-state wave launch of `tasks` tasks: four
// only for large FP32 launches (an FP64 four-wave group's LDS would leave
// room for one group per CU).
inline int wave3_wpb(int elem_bytes, int /*np*/, long long tasks) {
  return (elem_bytes == 4 && tasks > kWaveSmallTasks) ? kWaveTasksPerBlock : kWaveTasksPerBlockSmall;
}
inline bool tile_supported(int elem_bytes, int ns, int np, int code) {
  return code == kTileWave ? wave_variant_supported(elem_bytes, ns, np) : cpt_supported(elem_bytes, ns, code);
}
// the wave variant wherever it exists (three states: 1.3-2.1x faster than
// the workgroup variant on 128x128 and 256x256 batches of 3-16 members)
inline int tile_default(int elem_bytes, int ns, int np) {
  return wave_variant_supported(elem_bytes, ns, np) ? kTileWave : cpt_default(elem_bytes, ns);
}

// Arguments of the fused RK-stage kernel (passed by value).
struct StageArgs {
  const void* v;         // stage input, packed [B][N+1][nc][nq][np]
  const void* y;         // RK4 base state (nullptr: treated as zero)
  void* out;             // y + coef * L v
  double* partials;      // [B][kRespSlots][ntiles] level-0 trace partials, or nullptr
  const void* twiddle2;  // [n1][n2+1] complex exp(+2 pi i (n2 k1 mod np)/np), state precision
  const void* dtab;      // [ns][nq][np]: (U_j(q+r/2) - U_j(q-r/2)) / (2 hbar np), 0 at Nyquist
  const void* gtab;      // [npair][nq][np]: (U_j(q+r/2) - U_k(q-r/2)) / (hbar np), j < k
  const void* ctab;      // [npair][2][nq][np]: U_jl(q + r/2), U_jl(q - r/2) / (hbar np), pair j < l
                         // (q-dependent couplings in the workgroup variant)
  const void* mtab;      // wave variant: [kWaveTables][nq][n1][n2] = dtab 0, dtab 1, gtab / 2, U_01(q + r/2),
                         // U_01(q - r/2) (both / (hbar np)), entry (k1, k2) at m = k1 + n1 k2;
                         // three states: [kWaveTables3][nq][n1][n2] = dtab 0..2, gtab 0..2 / 2
  const double* bath;    // [B][kBathStride]: r0/m (= zeta), gamma, c0, c_delta, beta per member
  const void* psym;      // [2][np]: DFT symbols of D_p2 and D_p D_p, divided by np
  const void* closure;   // wave variant: learned W^(N+1) [B][4][nq][np] (one level per member), or nullptr
  // per-member depths (nullptr: every member has `depth`): member b has
  // levels mlev[b] .. mlev[b + 1] - 1 of a row numbering over all members,
  // and lev_member[row] is the member of a row.  mfirst: the member (in
  // that numbering) of this launch's member 0.
  const int* mlev;
  const int* lev_member;
  int mfirst;
  int slot;
  int qcoup;  // 1: q-dependent coupling through the r-space multiply (wave variant, two states)
  int nq;
  int depth;
  int ntiles;
  int batch;
  int nblocks_padded;       // grid size: ntiles * (depth+1) * batch rounded up to a multiple of 8
  int stream_out;           // wave variant: 1 = non-temporal output stores (the state exceeds the
                            // memory-side cache)
  int wpb;                  // wave variant: waves (tasks) per workgroup, kWaveTasksPerBlock or
                            // kWaveTasksPerBlockSmall
  long long member_stride;  // elements per member
  long long level_stride;   // elements per level
  long long comp_stride;    // elements per packed component (nq * np)
  double coef;
  double dq, dp, p0;
  double inv_mass;
  double coup[QHFPE_MAX_STATES][QHFPE_MAX_STATES];     // off-diagonal couplings / hbar
  double mu[QHFPE_MAX_STATES][QHFPE_MAX_STATES];
};

// Learned terminator (closure.hip): a linear 13x13 convolution over (q, p)
// from 8 input channels (the packed components of level N and the same times
// p) to the 4 packed components of level N + 1, trained as three 5x5 layers
// with kClosureHidden channels.
constexpr int kClosureHalf = 6;
constexpr int kClosureIn = 8;
constexpr int kClosureOut = 4;
constexpr int kClosureHidden = 32;
constexpr int kClosureKernelElems = 13 * 13 * kClosureIn * kClosureOut;   // K[13][13][8][4]
constexpr int kClosureStatsA = 25 * 25 * kClosureIn * kClosureIn;         // A[25][25][8][8]
constexpr int kClosureStatsC = 13 * 13 * kClosureIn * kClosureOut;        // C[13][13][8][4]
constexpr int kClosureStatsSize = kClosureStatsA + kClosureStatsC + 1;    // + yy
constexpr int kClosureWeightElems = 16 * 7 * 16 * 16;                     // BF16 MFMA B layout
// Training state (floats): the three layers, their gradients, Adam moments,
// the 9x9 product of the first two layers and its gradient, the composite
// kernel and its gradient, and per-entry loss terms (doubles).
struct ClosureTrainLayout {
  static constexpr int w1 = 0, n1 = 25 * kClosureIn * kClosureHidden;
  static constexpr int w2 = w1 + n1, n2 = 25 * kClosureHidden * kClosureHidden;
  static constexpr int w3 = w2 + n2, n3 = 25 * kClosureHidden * kClosureOut;
  static constexpr int nparam = n1 + n2 + n3;
  static constexpr int g1 = nparam, g2 = g1 + n1, g3 = g2 + n2;
  static constexpr int m = 2 * nparam, v = 3 * nparam;
  static constexpr int w12 = 4 * nparam, n12 = 81 * kClosureIn * kClosureHidden;
  static constexpr int g12 = w12 + n12;
  static constexpr int k = g12 + n12;
  static constexpr int gk = k + kClosureKernelElems;
  static constexpr int terms = gk + kClosureKernelElems;  // kClosureKernelElems doubles
  static constexpr int loss = terms + 2 * kClosureKernelElems;  // one double
  static constexpr int total = loss + 2;
};
static_assert(ClosureTrainLayout::terms % 2 == 0 && ClosureTrainLayout::loss % 2 == 0, "doubles stay aligned");

hipError_t launch_closure_weights(const float* K, unsigned short* wb, hipStream_t s);
hipError_t launch_closure_apply(int precision, int np, const void* v, int level, long long member_stride,
                                long long level_stride, long long comp_stride, int nq, int batch, double p0,
                                double dp, const unsigned short* wb, void* out, long long out_stride, hipStream_t s);
hipError_t launch_closure_stats(int precision, int np, const void* v, int level, long long member_stride,
                                long long level_stride, long long comp_stride, int nq, int batch, double p0,
                                double dp, double* stats, hipStream_t s);
hipError_t launch_closure_train_step(const double* stats, const float* prior, double ridge, float* state, int t,
                                     float lr, double* loss, hipStream_t s);
hipError_t launch_closure_compose(const double* stats, float* state, double* loss, hipStream_t s);
hipError_t launch_closure_loss(const double* stats, const float* K, float* g, double* terms, double* loss,
                               hipStream_t s);

// Host launchers (one translation unit per precision and state count).
hipError_t launch_stage_f64_ns2(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s);
hipError_t launch_stage_f64_ns3(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s);
hipError_t launch_stage_f32_ns2(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s);
hipError_t launch_stage_f32_ns3(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s);
hipError_t launch_stage_wave_f64(int np, const StageArgs& a, int nblocks, hipStream_t s);
hipError_t launch_stage_wave_f32(int np, const StageArgs& a, int nblocks, hipStream_t s);
hipError_t launch_stage_wave3_f64(int np, const StageArgs& a, int nblocks, hipStream_t s);
hipError_t launch_stage_wave3_f32(int np, const StageArgs& a, int nblocks, hipStream_t s);

// Pointwise and reduction kernels (aux_kernels.hip).
struct DipoleMu {
  double m[QHFPE_MAX_STATES][QHFPE_MAX_STATES];
};

struct GridDesc {
  int ns, nq, np, levels, batch, precision;
  long long member_stride, level_stride, comp_stride;
};

hipError_t launch_pack(const GridDesc& g, const double* canon, int phase, void* packed,
                       int member_offset, int nmembers, double* red, int* nred_blocks,
                       hipStream_t s);
hipError_t launch_unpack(const GridDesc& g, const void* packed, int phase, double* canon,
                         int member_offset, int nmembers, hipStream_t s);
hipError_t launch_dipole(const GridDesc& g, void* packed, const double mu[3][3], hipStream_t s);
hipError_t launch_thermal(const GridDesc& g, void* packed, double q0, double dq, double p0,
                          double dp, const double* bath, double omega, double mass, double hbar,
                          const double* noise, hipStream_t s);
hipError_t launch_trace_partials(const GridDesc& g, const void* packed, const double mu[3][3],
                                 int tq, int ntiles, double* partials, int slot, hipStream_t s);
hipError_t launch_finalize(int batch, int ntiles, int nslots, const double* partials,
                           double scale, int phase, double* resp, long long resp_stride,
                           long long resp_offset, int* flag, hipStream_t s);
hipError_t launch_clear_flag(int* flag, hipStream_t s);
// device-to-device copy of `bytes` (dst and src 16-byte aligned) by a
// streaming kernel: no memcpy or memset node when captured into a graph
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_norm_partials(const GridDesc& g, const void* packed, double* red,
                                int* nblocks_per_member, hipStream_t s);
hipError_t launch_spectrum_abs(const double* series, long long n, double dt, const double* omega,
                               int n_omega, double* out, hipStream_t s);
// The fixed device scratch of qhfpe_spectrum_corr_noalloc: kScratchDoubles
// doubles per device; scratch_pointer() returns the current device's address.
constexpr size_t kScratchDoubles = size_t(1) << 17;  // 1 MiB
constexpr int kMaxDevices = 64;
hipError_t scratch_pointer(double** out);
hipError_t launch_spectrum_corr(const double* r3, int n1, int n3, double dt1, double dt3,
                                const double* w1, int nw1, const double* w3, int nw3,
                                double* work, double* out, hipStream_t s);

}  // namespace qhfpe
