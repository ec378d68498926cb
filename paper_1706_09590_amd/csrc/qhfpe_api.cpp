// Host side of the MS-QHFPE C-ABI: parameter validation, workspace layout,
// launch sequencing of the RK4 stages, response finalisation and errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qhfpe.h"
#include "qhfpe_internal.hpp"

using namespace qhfpe;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(QHFPE_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t elem = 0;
  long long member_elems = 0, level_elems = 0, comp_elems = 0;
  size_t state_bytes = 0;
  size_t off_y = 0, off_va = 0, off_vb = 0, off_partials = 0, off_red = 0, off_tw = 0, off_flag = 0, off_mlev = 0;
  size_t off_dtab = 0, off_gtab = 0, off_ctab = 0, off_mtab = 0, off_bath = 0, off_psym = 0;
  int n1 = 0, n2 = 0;
  size_t total = 0;
  size_t red_count = 0;
  int max_tiles = 0;  // tiles per level at the narrowest tile variant
};

int validate(const qhfpe_params* p) {
  if (!p) return fail(QHFPE_EINVAL, "params is NULL");
  if (p->n_states != 2 && p->n_states != 3)
    return fail(QHFPE_EUNSUPPORTED, "n_states must be 2 or 3 (got %d)", p->n_states);
  if (p->nq < 4) return fail(QHFPE_EINVAL, "nq must be >= 4 (got %d)", p->nq);
  if (!find_plan(p->np))
    return fail(QHFPE_EUNSUPPORTED, "np=%d not supported (8,12,16,24,32,48,64,96,128,192,256)", p->np);
  if (p->depth < 0 || p->depth > 64) return fail(QHFPE_EINVAL, "depth must be in [0, 64] (got %d)", p->depth);
  // members index the second grid dimension of the pointwise kernels
  if (p->batch < 1 || p->batch > 65535) return fail(QHFPE_EINVAL, "batch must be in [1, 65535] (got %d)", p->batch);
  if (p->precision != QHFPE_FP64 && p->precision != QHFPE_FP32_FP64RED)
    return fail(QHFPE_EINVAL, "unknown precision %d", p->precision);
  if (p->reserved != 0) return fail(QHFPE_EINVAL, "reserved must be 0");
  if (!(p->q_max > p->q_min) || !(p->p_max > p->p_min)) return fail(QHFPE_EINVAL, "empty q or p range");
  if (!(p->mass > 0) || !(p->hbar > 0)) return fail(QHFPE_EINVAL, "mass and hbar must be > 0");
  if (!(p->zeta >= 0) || !(p->gamma > 0) || !(p->beta > 0))
    return fail(QHFPE_EINVAL, "need zeta >= 0, gamma > 0, beta > 0");
  if (p->low_temp_correction && !(p->beta * p->hbar * p->gamma < 2.0 * M_PI))
    return fail(QHFPE_EUNSUPPORTED, "low-temperature correction needs beta hbar gamma < 2 pi");
  if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(QHFPE_EINVAL, "dt must be finite and > 0");
  const int ns = p->n_states;
  for (int j = 0; j < ns; ++j)
    for (int l = 0; l < ns; ++l) {
      for (int k = 0; k < 5; ++k) {
        if (!std::isfinite(p->poly[j][l][k])) return fail(QHFPE_EINVAL, "poly has a non-finite entry");
        if (p->poly[j][l][k] != p->poly[l][j][k]) return fail(QHFPE_EINVAL, "poly must be symmetric");
      }
      if (!std::isfinite(p->mu[j][l]) || p->mu[j][l] != p->mu[l][j])
        return fail(QHFPE_EINVAL, "mu must be finite and symmetric");
    }
  const long double elems = (long double)p->batch * (p->depth + 1) * ns * ns * p->nq * p->np;
  // (the cap also keeps a stage grid's count of q tiles x levels x members,
  // about elems / (512 ns^2) plus levels x members, far below 2^31)
  if (elems > 4.0e11L) return fail(QHFPE_EINVAL, "state too large");
  // one hierarchy level of one member is addressed with 32-bit byte offsets
  const long double level_bytes = (long double)ns * ns * p->nq * p->np * 8.0L;
  if (level_bytes >= 2147483648.0L) return fail(QHFPE_EUNSUPPORTED, "one level exceeds 2 GiB");
  return QHFPE_OK;
}

Layout make_layout(const qhfpe_params* p) {
  Layout L;
  const Plan* pl = find_plan(p->np);
  const int nc = p->n_states * p->n_states;
  L.elem = (p->precision == QHFPE_FP64) ? 8 : 4;
  L.comp_elems = (long long)p->nq * p->np;
  L.level_elems = L.comp_elems * nc;
  L.member_elems = L.level_elems * (p->depth + 1);
  L.state_bytes = align_up((size_t)L.member_elems * p->batch * L.elem);
  const int esz = (p->precision == QHFPE_FP64) ? 8 : 4;
  const bool wave_ok = wave_variant_supported(esz, p->n_states, p->np);
  const int min_tq = wave_ok ? std::min(plan_groups(p->np) * kMinCpt, wave_columns_of(p->n_states, p->np))
                             : plan_groups(p->np) * kMinCpt;
  L.max_tiles = (p->nq + min_tq - 1) / min_tq;
  const long long cells = (long long)(p->depth + 1) * p->nq * p->np;
  const long long pack_blocks = (cells + kBlock - 1) / kBlock;
  L.red_count = (size_t)p->batch * (size_t)std::max<long long>(2 * pack_blocks, 1024);
  size_t off = 0;
  L.off_y = off;
  off += L.state_bytes;
  L.off_va = off;
  off += L.state_bytes;
  L.off_vb = off;
  off += L.state_bytes;
  L.off_partials = off;
  off += align_up((size_t)p->batch * kRespSlots * L.max_tiles * sizeof(double));
  L.off_red = off;
  off += align_up(L.red_count * sizeof(double));
  L.n1 = pl->n1;
  L.n2 = pl->n2;
  L.off_tw = off;
  off += align_up((size_t)pl->n1 * (pl->n2 + 1) * 2 * L.elem);
  const int ns = p->n_states;
  L.off_dtab = off;
  off += align_up((size_t)ns * L.comp_elems * L.elem);
  L.off_gtab = off;
  off += align_up((size_t)(ns * (ns - 1) / 2) * L.comp_elems * L.elem);
  L.off_ctab = off;
  off += align_up((size_t)(ns * (ns - 1)) * L.comp_elems * L.elem);
  L.off_mtab = off;
  if (wave_ok) off += align_up((size_t)wave_table_planes(ns) * L.comp_elems * L.elem);
  L.off_bath = off;
  off += align_up((size_t)p->batch * kBathStride * sizeof(double));
  L.off_psym = off;
  off += align_up((size_t)2 * p->np * L.elem);
  L.off_flag = off;
  off += kAlign;
  // per-member depths: level-row prefix [B + 1] and the member of each row
  L.off_mlev = off;
  off += align_up(((size_t)p->batch + 1 + (size_t)p->batch * (p->depth + 1)) * sizeof(int));
  L.total = off;
  return L;
}

// r0/m, gamma, c0, c_delta of the Drude bath (single exponential plus the
// delta-correlated term that absorbs the Matsubara frequencies).
void bath_constants(const qhfpe_params& p, double zeta, double gamma, double beta, double out[kBathStride]) {
  for (int k = 0; k < kBathStride; ++k) out[k] = 0.0;
  out[0] = zeta;  // r0 / m with r0 = m zeta
  out[1] = gamma;
  out[4] = beta;
  if (p.low_temp_correction) {
    const double x = 0.5 * beta * p.hbar * gamma;
    out[2] = 0.5 * p.mass * zeta * p.hbar * gamma * std::cos(x) / std::sin(x);
    out[3] = p.mass * zeta / beta - out[2];
  } else {
    out[2] = p.mass * zeta / beta;
    out[3] = 0.0;
  }
}

double poly_value(const double* c, double x) {
  return (((c[4] * x + c[3]) * x + c[2]) * x + c[1]) * x + c[0];
}

// r-space multipliers of the potential term at (q_i, r_m), with the argument
// q +- r/2 clamped to the q-grid and the Nyquist column averaged over +-r.
// Surfaces U_jl(x), j <= l: the params' polynomials or a host function; or
// the caller's tables of U_jl(q_i +- r_m/2) themselves ([ns][ns][nq][np],
// used as given).
struct Surfaces {
  const qhfpe_params* p = nullptr;
  qhfpe_potential_fn fn = nullptr;
  void* ctx = nullptr;
  const double* up_tab = nullptr;
  const double* um_tab = nullptr;
  double operator()(int j, int l, double x) const {
    if (fn) return fn(j, l, x, ctx);
    return poly_value(p->poly[j][l], x);
  }
};

// r-space multipliers at (q_i, r_m) for every table the kernels use:
//   dtab[j] = (U_jj(q + r/2) - U_jj(q - r/2)) / (2 hbar np)
//   gtab[pair j<k] = (U_jj(q + r/2) - U_kk(q - r/2)) / (hbar np)
//   ctab[2 pair], ctab[2 pair + 1] = U_jk(q + r/2) / (hbar np), U_jk(q - r/2) / (hbar np)
// Arguments are clamped to the q grid; at the Nyquist column both arguments
// take the average of the two values.  Returns false if a value is not
// finite; *coup_const tells whether every off-diagonal U_jl had one value
// (then coup[j][l] holds it divided by hbar).
bool multiplier_tables(const qhfpe_params& p, const Surfaces& U, double dq, double dp, std::vector<double>& dtab,
                       std::vector<double>& gtab, std::vector<double>& ctab, bool* coup_const,
                       double coup[QHFPE_MAX_STATES][QHFPE_MAX_STATES]) {
  const int ns = p.n_states, nq = p.nq, np = p.np;
  const double dr = 2.0 * M_PI * p.hbar / (np * dp);
  const double qlo = p.q_min, qhi = p.q_min + (nq - 1) * dq;
  auto clampq = [&](double x) { return x < qlo ? qlo : (x > qhi ? qhi : x); };
  const size_t plane = (size_t)nq * np;
  dtab.assign((size_t)ns * plane, 0.0);
  gtab.assign((size_t)(ns * (ns - 1) / 2) * plane, 0.0);
  ctab.assign((size_t)(ns * (ns - 1)) * plane, 0.0);
  double first[QHFPE_MAX_STATES][QHFPE_MAX_STATES] = {};
  bool seen = false, same = true, finite = true;
  for (int i = 0; i < nq; ++i) {
    const double q = p.q_min + i * dq;
    for (int m = 0; m < np; ++m) {
      const int mh = (m <= np / 2) ? m : m - np;
      const double xp = clampq(q + 0.5 * mh * dr), xm = clampq(q - 0.5 * mh * dr);
      const bool nyq = (m == np / 2);
      double up[QHFPE_MAX_STATES][QHFPE_MAX_STATES], um[QHFPE_MAX_STATES][QHFPE_MAX_STATES];
      for (int j = 0; j < ns; ++j)
        for (int l = j; l < ns; ++l) {
          if (U.up_tab) {
            const size_t t = (((size_t)j * ns + l) * nq + i) * np + m;
            up[j][l] = U.up_tab[t];
            um[j][l] = U.um_tab[t];
          } else {
            up[j][l] = U(j, l, xp);
            um[j][l] = U(j, l, xm);
          }
          finite = finite && std::isfinite(up[j][l]) && std::isfinite(um[j][l]);
          if (nyq && !U.up_tab) up[j][l] = um[j][l] = 0.5 * (up[j][l] + um[j][l]);
          if (l > j) {
            if (!seen) first[j][l] = up[j][l];
            same = same && up[j][l] == first[j][l] && um[j][l] == first[j][l];
          }
        }
      seen = true;
      const size_t at = (size_t)i * np + m;
      for (int j = 0; j < ns; ++j) dtab[j * plane + at] = (up[j][j] - um[j][j]) / (2.0 * p.hbar * np);
      int pr = 0;
      for (int j = 0; j < ns; ++j)
        for (int k = j + 1; k < ns; ++k, ++pr) gtab[pr * plane + at] = (up[j][j] - um[k][k]) / (p.hbar * np);
      pr = 0;
      for (int j = 0; j < ns; ++j)
        for (int k = j + 1; k < ns; ++k, ++pr) {
          ctab[2 * pr * plane + at] = up[j][k] / (p.hbar * np);
          ctab[(2 * pr + 1) * plane + at] = um[j][k] / (p.hbar * np);
        }
    }
  }
  *coup_const = same;
  for (int j = 0; j < ns; ++j)
    for (int l = 0; l < ns; ++l)
      coup[j][l] = (j == l || !same) ? 0.0 : first[std::min(j, l)][std::max(j, l)] / p.hbar;
  return finite;
}

// The multiplier tables of the wave variant in one array, each q row
// permuted so that the n2 values m = k1 + n1 k2 (k2 = 0..n2-1) of row k1
// are contiguous.  Two states: dtab 0, dtab 1, the coherence table halved
// (the kernel treats it as a pair of equal diagonal multipliers),
// U_01(q + r/2) and U_01(q - r/2) (used only for a q-dependent coupling).
// Three states: dtab 0..2, then the coherence tables of the pairs (0,1),
// (0,2), (1,2) halved.
void wave_tables(const qhfpe_params& p, int n1, int n2, const std::vector<double>& dtab,
                 const std::vector<double>& gtab, const std::vector<double>& ctab, std::vector<double>& mtab) {
  const int nq = p.nq, np = p.np, ns = p.n_states;
  const int planes = wave_table_planes(ns);
  const size_t plane = (size_t)nq * np;
  mtab.assign(planes * plane, 0.0);
  for (int t = 0; t < planes; ++t)
    for (int i = 0; i < nq; ++i)
      for (int k1 = 0; k1 < n1; ++k1)
        for (int k2 = 0; k2 < n2; ++k2) {
          const size_t src = (size_t)i * np + k1 + n1 * k2;
          double v;
          if (t < ns)
            v = dtab[t * plane + src];
          else if (ns == 3 || t == 2)
            v = 0.5 * gtab[(t - ns) * plane + src];
          else
            v = ctab[(t - 3) * plane + src];
          mtab[t * plane + (size_t)i * np + (size_t)k1 * n2 + k2] = v;
        }
}

// Symbols of the periodic fourth-order p-stencils in the DFT convention
// rho~[m] = sum_a W[a] exp(+2 pi i a m / np): a stencil sum_k c_k W[a + k]
// multiplies rho~[m] by sum_k c_k exp(-i k theta), theta = 2 pi m / np.
//   D_p2:      (-30 + 32 cos theta - 2 cos 2 theta) / (12 dp^2)
//   D_p D_p:  -(16 sin theta - 2 sin 2 theta)^2 / (144 dp^2)
// Both are stored divided by np (the inverse-transform normalisation).
void stencil_symbols(int np, double dp, std::vector<double>& sym) {
  sym.assign(2 * (size_t)np, 0.0);
  for (int m = 0; m < np; ++m) {
    const double th = 2.0 * M_PI * (double)m / (double)np;
    const double s1 = 16.0 * std::sin(th) - 2.0 * std::sin(2.0 * th);
    sym[m] = (-30.0 + 32.0 * std::cos(th) - 2.0 * std::cos(2.0 * th)) / (12.0 * dp * dp) / np;
    sym[np + m] = -(s1 * s1) / (144.0 * dp * dp) / np;
  }
}

// n1 x (n2 + 1) padded table of exp(+2 pi i (n2 k1 mod np) / np)
void twiddle_table(int np, int n1, int n2, std::vector<double>& tw) {
  tw.assign((size_t)n1 * (n2 + 1) * 2, 0.0);
  for (int k1 = 0; k1 < n1; ++k1)
    for (int j = 0; j < n2; ++j) {
      const double ang = 2.0 * M_PI * (double)((j * k1) % np) / (double)np;
      tw[2 * ((size_t)k1 * (n2 + 1) + j)] = std::cos(ang);
      tw[2 * ((size_t)k1 * (n2 + 1) + j) + 1] = std::sin(ang);
    }
}

template <typename T>
std::vector<T> convert(const std::vector<double>& x) {
  return std::vector<T>(x.begin(), x.end());
}

}  // namespace

struct qhfpe_handle {
  qhfpe_params p;
  Layout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int phase = 0;
  int ns = 0, nc = 0, levels = 0;
  int cpt = 4;  // stage tile variant (cells per thread along q)
  // off-diagonal couplings: constant (coup, applied pointwise) or
  // q-dependent (qcoup: the r-space multiply of the wave variant)
  double coup[QHFPE_MAX_STATES][QHFPE_MAX_STATES] = {};
  int qcoup = 0;
  // Member groups of qhfpe_step: each group's launches go to a stream of its
  // own, so that one group's next stage fills the GPU while another's launch
  // drains.  Created on first use, destroyed with the handle.
  int groups_req = 0;  // 0 = default rule
  int groups_made = 0;
  hipStream_t gstream[kMaxGroups] = {};
  hipEvent_t gfork = nullptr;
  hipEvent_t gjoin[kMaxGroups] = {};
  // orders qhfpe_copy_members between the streams of two handles
  hipEvent_t xevent = nullptr;
  // false until a state is loaded (set_state, init_thermal, copy_members):
  // a partial copy may then set the phase of the (all-zero) state
  bool loaded = false;
  // learned terminator (qhfpe_set_closure): BF16 weights in the MFMA layout
  // and the closure's W^(N+1) [B][level], in the caller's buffer
  unsigned short* closure_wb = nullptr;
  void* closure_out = nullptr;
  // per-member hierarchy depths (qhfpe_set_member_depth): mdepth[b] <= depth;
  // hmlev[b] = sum of the level counts of members before b; mixed when any
  // member has fewer levels than the handle
  std::vector<int> mdepth, hmlev;
  bool mixed = false;

  // (teardown: a failure to release has nothing left to report to)
  ~qhfpe_handle() {
    for (int g = 0; g < groups_made; ++g) {
      if (gstream[g]) (void)hipStreamDestroy(gstream[g]);
      if (gjoin[g]) (void)hipEventDestroy(gjoin[g]);
    }
    if (gfork) (void)hipEventDestroy(gfork);
    if (xevent) (void)hipEventDestroy(xevent);
  }

  // Default for small batches, where one launch per stage leaves most SIMDs
  // with two or three waves that all load, then all transform, in step: one
  // group per member up to three members, two groups for 4..16 members; one
  // group above that (no gain measured from 32 members on).
  int groups() const {
    int want = groups_req;
    if (want == 0) want = p.batch <= 3 ? p.batch : (p.batch <= 16 ? 2 : 1);
    return std::min(want, p.batch);
  }

  hipError_t make_groups(int n) {
    if (!gfork) {
      hipError_t e = hipEventCreateWithFlags(&gfork, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    for (; groups_made < n; ++groups_made) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) {
        if (st) (void)hipStreamDestroy(st);  // the creation error is the one reported
        return e;
      }
      gstream[groups_made] = st;
      gjoin[groups_made] = ev;
    }
    return hipSuccess;
  }

  bool wave() const { return cpt == kTileWave; }
  // variants that take a q-dependent coupling: the two-state wave variant
  // and the workgroup variant with kQcCpt cells per thread
  bool qc_variant(int code) const { return code == kTileWave ? ns == 2 : code == kQcCpt; }
  int tq_of(int np, int code) const {
    return code == kTileWave ? wave_columns_of(ns, np) : plan_groups(np) * code;
  }
  int tq() const { return tq_of(p.np, cpt); }
  // the trace partials hold L.max_tiles tiles per member and slot: a variant
  // with narrower tiles would index past them
  bool tile_fits(int code) const { return (p.nq + tq_of(p.np, code) - 1) / tq_of(p.np, code) <= L.max_tiles; }
  int ntiles() const { return (p.nq + tq() - 1) / tq(); }
  double dq = 0, dp = 0;

  void* y() const { return ws + L.off_y; }
  void* va() const { return ws + L.off_va; }
  void* vb() const { return ws + L.off_vb; }
  double* partials() const { return reinterpret_cast<double*>(ws + L.off_partials); }
  double* red() const { return reinterpret_cast<double*>(ws + L.off_red); }
  void* twiddle() const { return ws + L.off_tw; }
  void* dtab() const { return ws + L.off_dtab; }
  void* gtab() const { return ws + L.off_gtab; }
  void* ctab() const { return ws + L.off_ctab; }
  void* mtab() const { return ws + L.off_mtab; }
  double* bath() const { return reinterpret_cast<double*>(ws + L.off_bath); }
  void* psym() const { return ws + L.off_psym; }
  int* flag() const { return reinterpret_cast<int*>(ws + L.off_flag); }
  int* mlev() const { return reinterpret_cast<int*>(ws + L.off_mlev); }
  int* lev_member() const { return mlev() + p.batch + 1; }
  // stage units (wave-variant tasks or workgroups) of members first ..
  // first + count - 1
  long long units(int first, int count) const {
    return (long long)ntiles() * (mixed ? hmlev[first + count] - hmlev[first] : (long long)levels * count);
  }

  GridDesc grid() const {
    GridDesc g;
    g.ns = ns;
    g.nq = p.nq;
    g.np = p.np;
    g.levels = levels;
    g.batch = p.batch;
    g.precision = p.precision;
    g.member_stride = L.member_elems;
    g.level_stride = L.level_elems;
    g.comp_stride = L.comp_elems;
    return g;
  }

  StageArgs stage_args(const void* v, const void* yb, void* out, double coef) const {
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.v = v;
    a.y = yb;
    a.out = out;
    a.partials = nullptr;
    a.twiddle2 = twiddle();
    a.dtab = dtab();
    a.gtab = gtab();
    a.ctab = ctab();
    a.mtab = wave_variant_supported((int)L.elem, ns, p.np) ? mtab() : nullptr;
    a.qcoup = qcoup;
    a.bath = bath();
    a.psym = psym();
    a.closure = closure_out;
    a.slot = 0;
    a.nq = p.nq;
    a.depth = p.depth;
    a.ntiles = ntiles();
    a.batch = p.batch;
    a.mlev = mixed ? mlev() : nullptr;
    a.lev_member = mixed ? lev_member() : nullptr;
    a.mfirst = 0;
    a.nblocks_padded = padded_blocks(0, p.batch);
    a.wpb = wave_wpb(0, p.batch);
    // the three state arrays of the step against the MI355X's 256 MB
    // memory-side cache: above it, the stage outputs are stored
    // non-temporally (measured: 1024-member 128x128 depth-6 FP32 launch
    // 1248 -> 1201 us; at 113 MB, two 256x256 depth-8 FP64 members, the
    // same stores cost 17%)
    // (the levels the stages touch: with per-member depths, fewer than the
    // handle holds)
    constexpr double kMemorySideCacheBytes = 256.0 * 1024 * 1024;
    const double touched = (double)(mixed ? hmlev[p.batch] : (long long)levels * p.batch) * L.level_elems;
    a.stream_out = 3.0 * touched * L.elem > kMemorySideCacheBytes ? 1 : 0;
    a.member_stride = L.member_elems;
    a.level_stride = L.level_elems;
    a.comp_stride = L.comp_elems;
    a.coef = coef;
    a.dq = dq;
    a.dp = dp;
    a.p0 = p.p_min;
    a.inv_mass = 1.0 / p.mass;
    for (int j = 0; j < ns; ++j)
      for (int l = 0; l < ns; ++l) {
        a.coup[j][l] = coup[j][l];
        a.mu[j][l] = p.mu[j][l];
      }
    return a;
  }

  // waves per workgroup of a wave-variant launch over members first ..
  // first + count - 1
  int wave_wpb(int first, int count) const {
    const long long tasks = units(first, count);
    if (ns == 3) return wave3_wpb((int)L.elem, p.np, tasks);
    return (!qcoup && tasks <= kWaveSmallTasks) ? kWaveTasksPerBlockSmall : kWaveTasksPerBlock;
  }

  // grid of a stage launch over members first .. first + count - 1,
  // rounded up to a multiple of 8
  int padded_blocks(int first, int count) const {
    const long long u = units(first, count);  // workgroups, or waves of the wave variant
    const int wpb = wave_wpb(first, count);
    const long long blocks = wave() ? (u + wpb - 1) / wpb : u;
    return (int)((blocks + 7) / 8 * 8);
  }

  // the same stage restricted to members first .. first + count - 1
  StageArgs member_slice(StageArgs a, int first, int count) const {
    const size_t off = (size_t)first * L.member_elems * L.elem;
    a.v = static_cast<const char*>(a.v) + off;
    if (a.y) a.y = static_cast<const char*>(a.y) + off;
    a.out = static_cast<char*>(a.out) + off;
    if (a.closure) a.closure = static_cast<const char*>(a.closure) + (size_t)first * L.level_elems * L.elem;
    a.bath += (long long)kBathStride * first;
    if (a.partials) a.partials += (long long)first * kRespSlots * a.ntiles;
    a.batch = count;
    if (a.mlev) a.mfirst = first;
    a.nblocks_padded = padded_blocks(first, count);
    a.wpb = wave_wpb(first, count);
    return a;
  }

  hipError_t launch(const StageArgs& a) const { return launch_on(a, stream); }

  hipError_t launch_on(const StageArgs& a, hipStream_t s) const {
    const int nblocks = a.nblocks_padded;
    if (a.closure) {
      // the learned W^(N+1) of this stage's input, for these members
      hipError_t e = launch_closure_apply(p.precision, p.np, a.v, p.depth, L.member_elems, L.level_elems,
                                          L.comp_elems, p.nq, a.batch, p.p_min, dp, closure_wb,
                                          const_cast<void*>(a.closure), L.level_elems, s);
      if (e != hipSuccess) return e;
    }
    if (wave() && ns == 3)
      return p.precision == QHFPE_FP64 ? launch_stage_wave3_f64(p.np, a, nblocks, s)
                                       : launch_stage_wave3_f32(p.np, a, nblocks, s);
    if (wave())
      return p.precision == QHFPE_FP64 ? launch_stage_wave_f64(p.np, a, nblocks, s)
                                       : launch_stage_wave_f32(p.np, a, nblocks, s);
    if (p.precision == QHFPE_FP64)
      return ns == 2 ? launch_stage_f64_ns2(p.np, cpt, a, nblocks, s)
                     : launch_stage_f64_ns3(p.np, cpt, a, nblocks, s);
    return ns == 2 ? launch_stage_f32_ns2(p.np, cpt, a, nblocks, s)
                   : launch_stage_f32_ns3(p.np, cpt, a, nblocks, s);
  }
};

static_assert(QHFPE_CLOSURE_KERNEL_FLOATS == kClosureKernelElems, "closure kernel size");
static_assert(QHFPE_CLOSURE_STATS_DOUBLES == kClosureStatsSize, "closure statistics size");
static_assert(QHFPE_CLOSURE_TRAIN_FLOATS == ClosureTrainLayout::total, "closure training state size");

struct qhfpe_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  size_t nodes = 0;
};

namespace {

int check_handle(const qhfpe_t* h) {
  if (!h) return fail(QHFPE_EINVAL, "handle is NULL");
  return QHFPE_OK;
}

// partial sums of the level-0 trace of y into slot, then (optionally) finalise
int trace_into(qhfpe_t* h, int slot) {
  HIP_TRY(launch_trace_partials(h->grid(), h->y(), h->p.mu, h->tq(), h->ntiles(), h->partials(), slot, h->stream));
  return QHFPE_OK;
}

int finalize(qhfpe_t* h, int nslots, double* resp, long long resp_stride, long long offset) {
  HIP_TRY(launch_finalize(h->p.batch, h->ntiles(), nslots, h->partials(), h->dq * h->dp, h->phase, resp,
                          resp_stride, offset, h->flag(), h->stream));
  return QHFPE_OK;
}

// finalize for members first .. first + count - 1 on stream s
int finalize_members(qhfpe_t* h, int first, int count, int nslots, double* resp, long long resp_stride,
                     long long offset, hipStream_t s) {
  HIP_TRY(launch_finalize(count, h->ntiles(), nslots, h->partials() + (long long)first * kRespSlots * h->ntiles(),
                          h->dq * h->dp, h->phase, resp ? resp + (long long)first * resp_stride : nullptr,
                          resp_stride, offset, h->flag(), s));
  return QHFPE_OK;
}

int read_flag(qhfpe_t* h, int* value) {
  HIP_TRY(hipMemcpyAsync(value, h->flag(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return QHFPE_OK;
}

// true while the handle's stream records into a graph
bool capturing(const qhfpe_t* h) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(h->stream, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusActive;
}

// ||buf||_2 per member into out[b] (host)
int norms(qhfpe_t* h, const void* buf, std::vector<double>& out) {
  int nb = 0;
  HIP_TRY(launch_norm_partials(h->grid(), buf, h->red(), &nb, h->stream));
  std::vector<double> host((size_t)nb * h->p.batch);
  HIP_TRY(hipMemcpyAsync(host.data(), h->red(), host.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  out.assign(h->p.batch, 0.0);
  for (int b = 0; b < h->p.batch; ++b) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += host[(size_t)b * nb + i];
    out[b] = std::sqrt(s);
  }
  return QHFPE_OK;
}

// Multiplier tables from the surfaces U, uploaded to the handle (computed in
// FP64 and rounded once to the state precision).  When the surfaces are
// rejected the handle's tables and coupling mode are unchanged; after a
// failed upload (QHFPE_EHIP) the tables may be partly replaced.
int install_surfaces(qhfpe_t* h, const Surfaces& U) {
  std::vector<double> dt, gt, ct, mt;
  bool coup_const = true;
  double coup[QHFPE_MAX_STATES][QHFPE_MAX_STATES];
  if (!multiplier_tables(h->p, U, h->dq, h->dp, dt, gt, ct, &coup_const, coup))
    return fail(QHFPE_EINVAL, "the potential has a non-finite value on the grid");
  if (wave_variant_supported((int)h->L.elem, h->ns, h->p.np)) wave_tables(h->p, h->L.n1, h->L.n2, dt, gt, ct, mt);
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const std::vector<double>& src) {
    if (e != hipSuccess || src.empty()) return;
    if (h->p.precision == QHFPE_FP64) {
      e = hipMemcpyAsync(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
    } else {
      std::vector<float> f = convert<float>(src);
      e = hipMemcpyAsync(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // the host vectors are temporaries
  };
  up(h->dtab(), dt);
  up(h->gtab(), gt);
  up(h->ctab(), ct);
  up(h->mtab(), mt);
  if (e != hipSuccess) return fail(QHFPE_EHIP, "uploading the potential tables: %s", hipGetErrorString(e));
  for (int j = 0; j < QHFPE_MAX_STATES; ++j)
    for (int l = 0; l < QHFPE_MAX_STATES; ++l) h->coup[j][l] = (j < h->ns && l < h->ns) ? coup[j][l] : 0.0;
  h->qcoup = coup_const ? 0 : 1;
  if (h->qcoup && !h->qc_variant(h->cpt)) h->cpt = wave_supported(h->ns, h->p.np) ? kTileWave : kQcCpt;
  return QHFPE_OK;
}

}  // namespace

extern "C" {

const char* qhfpe_last_error(void) { return g_err.c_str(); }

int qhfpe_workspace_bytes(const qhfpe_params* params, size_t* bytes) {
  if (!bytes) return fail(QHFPE_EINVAL, "bytes is NULL");
  int rc = validate(params);
  if (rc) return rc;
  *bytes = make_layout(params).total;
  return QHFPE_OK;
}

int qhfpe_create(const qhfpe_params* params, void* d_workspace, size_t bytes, void* stream, qhfpe_t** out) {
  if (!out) return fail(QHFPE_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(params);
  if (rc) return rc;
  if (!d_workspace) return fail(QHFPE_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) return fail(QHFPE_EINVAL, "workspace must be 256-byte aligned");
  Layout L = make_layout(params);
  if (bytes < L.total) return fail(QHFPE_ESTATE, "workspace too small: %zu < %zu bytes", bytes, L.total);
  qhfpe_t* h = new (std::nothrow) qhfpe_handle();
  if (!h) return fail(QHFPE_EINVAL, "out of host memory");
  h->p = *params;
  h->L = L;
  h->ws = static_cast<char*>(d_workspace);
  h->stream = static_cast<hipStream_t>(stream);
  h->ns = params->n_states;
  h->nc = h->ns * h->ns;
  h->levels = params->depth + 1;
  h->mdepth.assign(params->batch, params->depth);
  h->hmlev.resize(params->batch + 1);
  for (int b = 0; b <= params->batch; ++b) h->hmlev[b] = b * h->levels;
  h->cpt = tile_default((int)L.elem, params->n_states, params->np);
  h->dq = (params->q_max - params->q_min) / params->nq;
  h->dp = (params->p_max - params->p_min) / params->np;
  // setup tables, computed in FP64 and rounded once to the state precision
  std::vector<double> tw, sym;
  twiddle_table(params->np, L.n1, L.n2, tw);
  stencil_symbols(params->np, h->dp, sym);
  std::vector<double> bath((size_t)params->batch * kBathStride);
  double bc[kBathStride];
  bath_constants(*params, params->zeta, params->gamma, params->beta, bc);
  for (int b = 0; b < params->batch; ++b)
    for (int k = 0; k < kBathStride; ++k) bath[kBathStride * b + k] = bc[k];
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const std::vector<double>& src) {
    if (e != hipSuccess || src.empty()) return;
    if (params->precision == QHFPE_FP64) {
      e = hipMemcpyAsync(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
    } else {
      std::vector<float> f = convert<float>(src);
      e = hipMemcpyAsync(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // f is a temporary
    }
  };
  up(h->twiddle(), tw);
  up(h->psym(), sym);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->bath(), bath.data(), bath.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->y(), 0, 3 * L.state_bytes, h->stream);
  if (e == hipSuccess) e = launch_clear_flag(h->flag(), h->stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->xevent, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return fail(QHFPE_EHIP, "create: %s", hipGetErrorString(e));
  }
  Surfaces poly;
  poly.p = &h->p;
  if (int rc = install_surfaces(h, poly)) {
    delete h;
    return rc;
  }
  *out = h;
  return QHFPE_OK;
}

int qhfpe_set_potential(qhfpe_t* h, qhfpe_potential_fn fn, void* ctx) {
  if (int rc = check_handle(h)) return rc;
  if (!fn) return fail(QHFPE_EINVAL, "fn is NULL");
  Surfaces U;
  U.p = &h->p;
  U.fn = fn;
  U.ctx = ctx;
  return install_surfaces(h, U);
}

int qhfpe_set_potential_tables(qhfpe_t* h, const double* u_plus, const double* u_minus) {
  if (int rc = check_handle(h)) return rc;
  if (!u_plus || !u_minus) return fail(QHFPE_EINVAL, "u_plus and u_minus must not be NULL");
  Surfaces U;
  U.p = &h->p;
  U.up_tab = u_plus;
  U.um_tab = u_minus;
  return install_surfaces(h, U);
}

double qhfpe_morse_gauss_potential(int32_t j, int32_t l, double x, void* ctx) {
  const qhfpe_morse_gauss* c = static_cast<const qhfpe_morse_gauss*>(ctx);
  if (!c || j < 0 || l < 0 || j > 1 || l > 1) return std::nan("");
  if (j == 0 && l == 0) {
    const double e = 1.0 - std::exp(-c->a0 * (x - c->q0));
    return c->D0 * e * e;
  }
  if (j == 1 && l == 1) {
    const double e = 1.0 - std::exp(-c->a1 * (x - c->q1));
    return c->D1 * e * e + c->dE;
  }
  const double d = x - c->qs;
  return c->dV * std::exp(-d * d / (2.0 * c->sigma * c->sigma));
}

int qhfpe_destroy(qhfpe_t* h) {
  if (!h) return QHFPE_OK;
  delete h;
  return QHFPE_OK;
}

int qhfpe_set_member_bath(qhfpe_t* h, int32_t member, double zeta, double gamma, double beta) {
  if (int rc = check_handle(h)) return rc;
  if (member < -1 || member >= h->p.batch) return fail(QHFPE_EINVAL, "member out of range");
  if (!(zeta >= 0) || !(gamma > 0) || !(beta > 0) || !std::isfinite(zeta) || !std::isfinite(gamma) ||
      !std::isfinite(beta))
    return fail(QHFPE_EINVAL, "need finite zeta >= 0, gamma > 0, beta > 0");
  if (h->p.low_temp_correction && !(beta * h->p.hbar * gamma < 2.0 * M_PI))
    return fail(QHFPE_EUNSUPPORTED, "low-temperature correction needs beta hbar gamma < 2 pi");
  double bc[kBathStride];
  bath_constants(h->p, zeta, gamma, beta, bc);
  const int first = member < 0 ? 0 : member;
  const int count = member < 0 ? h->p.batch : 1;
  std::vector<double> buf((size_t)count * kBathStride);
  for (int b = 0; b < count; ++b)
    for (int k = 0; k < kBathStride; ++k) buf[kBathStride * b + k] = bc[k];
  HIP_TRY(hipMemcpyAsync(h->bath() + kBathStride * first, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice,
                         h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return QHFPE_OK;
}

int qhfpe_set_member_depth(qhfpe_t* h, int32_t member, int32_t depth) {
  if (int rc = check_handle(h)) return rc;
  if (member < 0 || member >= h->p.batch) return fail(QHFPE_EINVAL, "member %d out of range", member);
  if (depth < 0 || depth > h->p.depth) return fail(QHFPE_EINVAL, "depth %d outside 0..%d", depth, h->p.depth);
  if (h->closure_out && depth != h->p.depth)
    return fail(QHFPE_EUNSUPPORTED, "a learned closure needs every member at the handle's depth");
  if (capturing(h)) return fail(QHFPE_ESTATE, "qhfpe_set_member_depth synchronises: not allowed while capturing");
  std::vector<int> md = h->mdepth;
  md[member] = depth;
  std::vector<int> lev(h->p.batch + 1 + (size_t)h->p.batch * h->levels, 0);
  bool mixed = false;
  int row = 0;
  for (int b = 0; b < h->p.batch; ++b) {
    lev[b] = row;
    for (int n = 0; n <= md[b]; ++n) lev[h->p.batch + 1 + row++] = b;
    mixed = mixed || md[b] != h->p.depth;
  }
  lev[h->p.batch] = row;
  HIP_TRY(hipMemcpyAsync(h->mlev(), lev.data(), lev.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->mdepth = md;
  h->hmlev.assign(lev.begin(), lev.begin() + h->p.batch + 1);
  h->mixed = mixed;
  return QHFPE_OK;
}

int qhfpe_set_tile(qhfpe_t* h, int32_t cells_per_thread) {
  if (int rc = check_handle(h)) return rc;
  const int c = cells_per_thread == 0 ? tile_default((int)h->L.elem, h->ns, h->p.np) : cells_per_thread;
  if (!tile_supported((int)h->L.elem, h->ns, h->p.np, c) || !h->tile_fits(c))
    return fail(QHFPE_EUNSUPPORTED, "tile variant %d not available for this precision and state count", c);
  if (h->qcoup && !h->qc_variant(c))
    return fail(QHFPE_EUNSUPPORTED, "a q-dependent coupling needs the two-state wave variant (tile 1) or tile %d",
                kQcCpt);
  if (h->closure_out && c != kTileWave)
    return fail(QHFPE_EUNSUPPORTED, "a learned closure needs the wave variant (tile 1)");
  h->cpt = c;
  return QHFPE_OK;
}

int qhfpe_autotune(qhfpe_t* h, int32_t reps, int32_t* h_chosen) {
  if (int rc = check_handle(h)) return rc;
  if (reps < 1) return fail(QHFPE_EINVAL, "reps must be >= 1");
  // time stage launches that read the state and write the scratch buffer
  // (the state is not modified), for every available tile variant
  const int candidates[] = {kTileWave, 2, 4, 8};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(QHFPE_EHIP, "hipEventCreate failed");
  }
  int best = h->cpt;
  float best_ms = 1e30f;
  int rc = QHFPE_OK;
  for (int c : candidates) {
    if (!tile_supported((int)h->L.elem, h->ns, h->p.np, c) || !h->tile_fits(c)) continue;
    if (h->closure_out && c != kTileWave) continue;
    if (h->qcoup && !h->qc_variant(c)) continue;
    h->cpt = c;
    StageArgs a = h->stage_args(h->y(), h->y(), h->va(), 0.25 * h->p.dt);
    hipError_t e = h->launch(a);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = h->launch(a);
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = fail(QHFPE_EHIP, "autotune: %s", hipGetErrorString(e));
      break;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);  // the events are scratch; a release failure changes no result
  (void)hipEventDestroy(e1);
  h->cpt = best;
  if (rc == QHFPE_OK && h_chosen) *h_chosen = best;
  return rc;
}

int qhfpe_set_streams(qhfpe_t* h, int32_t groups) {
  if (int rc = check_handle(h)) return rc;
  if (groups < 0 || groups > kMaxGroups) return fail(QHFPE_EINVAL, "groups must be in [0, %d]", kMaxGroups);
  h->groups_req = groups;
  // the streams of the groups exist before any step (and so before a capture)
  if (h->groups() > 1) HIP_TRY(h->make_groups(h->groups()));
  return QHFPE_OK;
}

int qhfpe_get_streams(const qhfpe_t* h, int32_t* groups) {
  if (int rc = check_handle(h)) return rc;
  if (!groups) return fail(QHFPE_EINVAL, "groups is NULL");
  *groups = h->groups();
  return QHFPE_OK;
}

int qhfpe_get_phase(const qhfpe_t* h, int32_t* phase) {
  if (int rc = check_handle(h)) return rc;
  if (!phase) return fail(QHFPE_EINVAL, "phase is NULL");
  *phase = h->phase;
  return QHFPE_OK;
}

int qhfpe_set_state(qhfpe_t* h, const double* d_canon, int32_t phase, int32_t member) {
  if (int rc = check_handle(h)) return rc;
  if (!d_canon) return fail(QHFPE_EINVAL, "d_canon is NULL");
  if (phase < 0 || phase > 3) return fail(QHFPE_EINVAL, "phase must be 0..3");
  if (member < -1 || member >= h->p.batch) return fail(QHFPE_EINVAL, "member out of range");
  if (member >= 0 && phase != h->phase)
    return fail(QHFPE_ESTATE, "single-member load with phase %d into a handle of phase %d", phase, h->phase);
  const int first = member < 0 ? 0 : member;
  const int count = member < 0 ? h->p.batch : 1;
  int nblk = 0;
  // convert into the scratch buffer first; commit only a Hermitian state
  HIP_TRY(launch_pack(h->grid(), d_canon, phase, h->va(), first, count, h->red(), &nblk, h->stream));
  std::vector<double> red((size_t)nblk * count * 2);
  HIP_TRY(hipMemcpyAsync(red.data(), h->red(), red.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  double dev = 0.0, mag = 0.0;
  for (size_t i = 0; i < red.size(); i += 2) {
    dev = std::max(dev, red[i]);
    mag = std::max(mag, red[i + 1]);
  }
  if (!std::isfinite(dev) || !std::isfinite(mag)) return fail(QHFPE_ENONFINITE, "state has NaN/Inf entries");
  if (dev > 1e-12 * std::max(mag, 1e-300))
    return fail(QHFPE_EUNSUPPORTED, "state is not i^%d times a Hermitian matrix (deviation %.3e of max %.3e)",
                phase, dev, mag);
  const size_t mb = (size_t)h->L.member_elems * h->L.elem;
  HIP_TRY(hipMemcpyAsync(static_cast<char*>(h->y()) + first * mb, static_cast<char*>(h->va()) + first * mb,
                         count * mb, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->phase = phase;
  h->loaded = true;
  return QHFPE_OK;
}

int qhfpe_get_state(qhfpe_t* h, double* d_canon, int32_t member) {
  if (int rc = check_handle(h)) return rc;
  if (!d_canon) return fail(QHFPE_EINVAL, "d_canon is NULL");
  if (member < -1 || member >= h->p.batch) return fail(QHFPE_EINVAL, "member out of range");
  const int first = member < 0 ? 0 : member;
  const int count = member < 0 ? h->p.batch : 1;
  HIP_TRY(launch_unpack(h->grid(), h->y(), h->phase, d_canon, first, count, h->stream));
  return QHFPE_OK;
}

int qhfpe_init_thermal(qhfpe_t* h, double omega, const double* d_noise) {
  if (int rc = check_handle(h)) return rc;
  if (!(omega > 0) || !std::isfinite(omega)) return fail(QHFPE_EINVAL, "omega must be finite and > 0");
  HIP_TRY(launch_thermal(h->grid(), h->y(), h->p.q_min, h->dq, h->p.p_min, h->dp, h->bath(), omega, h->p.mass,
                         h->p.hbar, d_noise, h->stream));
  h->phase = 0;
  h->loaded = true;
  return QHFPE_OK;
}

int qhfpe_apply_dipole(qhfpe_t* h, int32_t mode) {
  if (int rc = check_handle(h)) return rc;
  if (mode != QHFPE_COMMUTATOR) return fail(QHFPE_EUNSUPPORTED, "only QHFPE_COMMUTATOR is supported");
  HIP_TRY(launch_dipole(h->grid(), h->y(), h->p.mu, h->stream));
  h->phase = (h->phase + 1) & 3;
  return QHFPE_OK;
}

}  // extern "C"

namespace {

int check_step_args(const qhfpe_t* h, int64_t nsteps, int32_t stride, const double* d_resp) {
  if (int rc = check_handle(h)) return rc;
  if (nsteps < 0) return fail(QHFPE_EINVAL, "nsteps must be >= 0");
  if (stride < 1) return fail(QHFPE_EINVAL, "stride must be >= 1");
  if (d_resp && nsteps % stride) return fail(QHFPE_EINVAL, "nsteps must be a multiple of stride");
  return QHFPE_OK;
}

// Enqueue nsteps RK4 steps with their trace samples on the handle's stream.
// Non-finite samples set the handle's flag; nothing is read back.
int step_enqueue(qhfpe_t* h, int64_t nsteps, int32_t stride, double* d_resp) {
  const double dt = h->p.dt;
  const long long nsamples = d_resp ? nsteps / stride + 1 : 0;
  int slot = 0;
  long long base = 0;
  if (d_resp) {
    if (int rc = trace_into(h, 0)) return rc;
    slot = 1;
  }
  // RK4 for the autonomous linear L is the degree-4 Taylor polynomial of
  // exp(dt L).  It is applied as the product of its two real quadratic
  // factors 1 + a dt L + b dt^2 L^2 = 1 + a dt L (1 + (b / a) dt L), each
  // from the pair of complex roots of 1 + z + z^2/2 + z^3/6 + z^4/24:
  //   v_a = y + c1 dt L y,  v_b = y + a1 dt L v_a,
  //   v_a = v_b + c2 dt L v_b,  y = v_b + a2 dt L v_a.
  // Two of the four stages read a single array, so a step moves 10 state
  // passes instead of the 11 of the nested (Horner) form.
  constexpr double kA1 = 0.9147466869945951459773425, kC1 = 0.2891102187731809321579357;
  constexpr double kA2 = 0.08525331300540485402265752, kC2 = 1.848047823830076680679732;
  StageArgs s1 = h->stage_args(h->y(), h->y(), h->va(), kC1 * dt);
  StageArgs s2 = h->stage_args(h->va(), h->y(), h->vb(), kA1 * dt);
  StageArgs s3 = h->stage_args(h->vb(), h->vb(), h->va(), kC2 * dt);
  StageArgs s4 = h->stage_args(h->va(), h->vb(), h->y(), kA2 * dt);
  // member groups: group g holds members first[g] .. first[g + 1] - 1 and
  // runs on its own stream between a fork and a join on the handle's stream
  int G = nsteps > 0 ? h->groups() : 1;
  // no stream is created while the handle's stream records a graph; the
  // results do not depend on the grouping
  if (G > h->groups_made && capturing(h)) G = 1;
  int first[kMaxGroups + 1];
  for (int g = 0; g <= G; ++g) first[g] = (int)((long long)g * h->p.batch / G);
  hipStream_t gs[kMaxGroups];
  StageArgs g1[kMaxGroups], g2[kMaxGroups], g3[kMaxGroups];
  if (G > 1) {
    HIP_TRY(h->make_groups(G));
    HIP_TRY(hipEventRecord(h->gfork, h->stream));
    for (int g = 0; g < G; ++g) {
      gs[g] = h->gstream[g];
      HIP_TRY(hipStreamWaitEvent(gs[g], h->gfork, 0));
    }
  } else {
    gs[0] = h->stream;
  }
  for (int g = 0; g < G; ++g) {
    const int cnt = first[g + 1] - first[g];
    g1[g] = G > 1 ? h->member_slice(s1, first[g], cnt) : s1;
    g2[g] = G > 1 ? h->member_slice(s2, first[g], cnt) : s2;
    g3[g] = G > 1 ? h->member_slice(s3, first[g], cnt) : s3;
  }
  auto run = [&]() -> int {
    for (int64_t s = 1; s <= nsteps; ++s) {
      const bool sample = d_resp && (s % stride == 0);
      s4.partials = sample ? h->partials() : nullptr;
      s4.slot = slot;
      for (int g = 0; g < G; ++g) {
        HIP_TRY(h->launch_on(g1[g], gs[g]));
        HIP_TRY(h->launch_on(g2[g], gs[g]));
        HIP_TRY(h->launch_on(g3[g], gs[g]));
        HIP_TRY(h->launch_on(G > 1 ? h->member_slice(s4, first[g], first[g + 1] - first[g]) : s4, gs[g]));
      }
      if (sample && ++slot == kRespSlots) {
        for (int g = 0; g < G; ++g)
          if (int rc = finalize_members(h, first[g], first[g + 1] - first[g], slot, d_resp, nsamples * 2, base,
                                        gs[g]))
            return rc;
        base += slot;
        slot = 0;
      }
    }
    if (d_resp && slot > 0) {
      for (int g = 0; g < G; ++g)
        if (int rc =
                finalize_members(h, first[g], first[g + 1] - first[g], slot, d_resp, nsamples * 2, base, gs[g]))
          return rc;
    }
    return QHFPE_OK;
  };
  int rc_run = run();
  if (G > 1) {
    // join even after an error, so that the handle's stream orders later work
    for (int g = 0; g < G; ++g) {
      if (hipEventRecord(h->gjoin[g], gs[g]) != hipSuccess ||
          hipStreamWaitEvent(h->stream, h->gjoin[g], 0) != hipSuccess)
        if (rc_run == QHFPE_OK) rc_run = fail(QHFPE_EHIP, "step: joining member groups failed");
    }
  }
  if (rc_run) return rc_run;
  if (!d_resp) {
    if (int rc = trace_into(h, 0)) return rc;
    if (int rc = finalize(h, 1, nullptr, 0, 0)) return rc;
  }
  return QHFPE_OK;
}

// Read and clear the handle's non-finite flag (synchronises its stream).
int take_flag(qhfpe_t* h) {
  int flag = 0;
  if (int rc = read_flag(h, &flag)) return rc;
  if (flag) {
    HIP_TRY(launch_clear_flag(h->flag(), h->stream));
    return fail(QHFPE_ENONFINITE, "non-finite trace during propagation (dt too large?)");
  }
  return QHFPE_OK;
}

}  // namespace

extern "C" {

int qhfpe_step(qhfpe_t* h, int64_t nsteps, int32_t stride, double* d_resp) {
  if (int rc = check_step_args(h, nsteps, stride, d_resp)) return rc;
  if (capturing(h)) return fail(QHFPE_ESTATE, "qhfpe_step synchronises: use qhfpe_step_async while capturing");
  HIP_TRY(launch_clear_flag(h->flag(), h->stream));
  if (int rc = step_enqueue(h, nsteps, stride, d_resp)) return rc;
  return take_flag(h);
}

int qhfpe_step_async(qhfpe_t* h, int64_t nsteps, int32_t stride, double* d_resp) {
  if (int rc = check_step_args(h, nsteps, stride, d_resp)) return rc;
  return step_enqueue(h, nsteps, stride, d_resp);
}

int qhfpe_status(qhfpe_t* h) {
  if (int rc = check_handle(h)) return rc;
  if (capturing(h)) return fail(QHFPE_ESTATE, "qhfpe_status synchronises: not allowed while capturing");
  return take_flag(h);
}

int qhfpe_stream_copy(void* d_dst, const void* d_src, size_t bytes, void* stream) {
  if (bytes == 0) return QHFPE_OK;
  if (!d_dst || !d_src) return fail(QHFPE_EINVAL, "NULL pointer");
  if ((reinterpret_cast<uintptr_t>(d_dst) | reinterpret_cast<uintptr_t>(d_src)) % 16)
    return fail(QHFPE_EINVAL, "pointers must be 16-byte aligned");
  const uintptr_t a = reinterpret_cast<uintptr_t>(d_dst), b = reinterpret_cast<uintptr_t>(d_src);
  if (a < b + bytes && b < a + bytes && a != b) return fail(QHFPE_EINVAL, "overlapping ranges");
  HIP_TRY(launch_stream_copy(d_dst, d_src, bytes, static_cast<hipStream_t>(stream)));
  return QHFPE_OK;
}


int qhfpe_response(qhfpe_t* h, double* d_out) {
  if (int rc = check_handle(h)) return rc;
  if (!d_out) return fail(QHFPE_EINVAL, "d_out is NULL");
  if (int rc = trace_into(h, 0)) return rc;
  return finalize(h, 1, d_out, 2, 0);
}

// With per-member depths a stage leaves the levels above a member's depth
// unwritten: clear the output buffer first where it is read as a whole.
static int clear_for_whole_read(qhfpe_t* h, void* buf) {
  if (!h->mixed) return QHFPE_OK;
  if (capturing(h)) return fail(QHFPE_ESTATE, "not while recording with per-member depths");
  HIP_TRY(hipMemsetAsync(buf, 0, (size_t)h->L.member_elems * h->p.batch * h->L.elem, h->stream));
  return QHFPE_OK;
}

int qhfpe_apply_rhs(qhfpe_t* h) {
  if (int rc = check_handle(h)) return rc;
  if (int rc = clear_for_whole_read(h, h->va())) return rc;
  StageArgs a = h->stage_args(h->y(), nullptr, h->va(), 1.0);
  HIP_TRY(h->launch(a));
  HIP_TRY(hipMemcpyAsync(h->y(), h->va(), (size_t)h->L.member_elems * h->p.batch * h->L.elem,
                         hipMemcpyDeviceToDevice, h->stream));
  return QHFPE_OK;
}

int qhfpe_residual(qhfpe_t* h, double* h_out) {
  if (int rc = check_handle(h)) return rc;
  if (!h_out) return fail(QHFPE_EINVAL, "h_out is NULL");
  if (int rc = clear_for_whole_read(h, h->va())) return rc;
  StageArgs a = h->stage_args(h->y(), nullptr, h->va(), 1.0);
  HIP_TRY(h->launch(a));
  std::vector<double> nl, nw;
  if (int rc = norms(h, h->va(), nl)) return rc;
  if (int rc = norms(h, h->y(), nw)) return rc;
  for (int b = 0; b < h->p.batch; ++b) {
    h_out[2 * b] = nl[b];
    h_out[2 * b + 1] = nw[b];
  }
  return QHFPE_OK;
}

int qhfpe_relax(qhfpe_t* h, double tol, int64_t max_steps, int32_t check_every, int64_t* h_steps_done,
                double* h_residual) {
  if (int rc = check_handle(h)) return rc;
  if (!(tol > 0) || max_steps < 0 || check_every < 1) return fail(QHFPE_EINVAL, "bad relax arguments");
  std::vector<double> r(2 * (size_t)h->p.batch);
  int64_t done = 0;
  double worst = INFINITY;
  while (true) {
    if (int rc = qhfpe_residual(h, r.data())) return rc;
    worst = 0.0;
    for (int b = 0; b < h->p.batch; ++b) {
      const double q = r[2 * b] / std::max(r[2 * b + 1], 1e-300);
      if (!std::isfinite(q)) return fail(QHFPE_ENONFINITE, "non-finite residual during relaxation");
      worst = std::max(worst, q);
    }
    if (worst < tol || done >= max_steps) break;
    const int64_t n = std::min<int64_t>(check_every, max_steps - done);
    if (int rc = qhfpe_step(h, n, 1, nullptr)) return rc;
    done += n;
  }
  if (h_steps_done) *h_steps_done = done;
  if (h_residual) *h_residual = worst;
  return QHFPE_OK;
}

int qhfpe_copy_members(const qhfpe_t* src, int32_t src_member, qhfpe_t* dst, int32_t dst_member, int32_t count) {
  if (!src || !dst) return fail(QHFPE_EINVAL, "handle is NULL");
  if (src->ns != dst->ns || src->p.nq != dst->p.nq || src->p.np != dst->p.np || src->p.depth != dst->p.depth ||
      src->p.precision != dst->p.precision)
    return fail(QHFPE_ESTATE, "handles differ in n_states, grid, depth or precision");
  if (count < 0 || src_member < 0 || dst_member < 0 || src_member + count > src->p.batch ||
      dst_member + count > dst->p.batch)
    return fail(QHFPE_EINVAL, "member range out of bounds");
  if (src == dst && src_member < dst_member + count && dst_member < src_member + count && src_member != dst_member)
    return fail(QHFPE_EINVAL, "overlapping member ranges within one handle");
  if (count == 0 || (src == dst && src_member == dst_member)) return QHFPE_OK;
  // a member's levels above its own depth are never updated: copied members
  // must keep their depths
  for (int k = 0; k < count; ++k)
    if (src->mdepth[src_member + k] != dst->mdepth[dst_member + k])
      return fail(QHFPE_ESTATE, "member %d (depth %d) copied onto member %d of depth %d", src_member + k,
                  src->mdepth[src_member + k], dst_member + k, dst->mdepth[dst_member + k]);
  // the phase i^k is one per handle: a partial copy into a loaded handle of
  // another phase would leave its other members read with the wrong phase
  const bool whole = dst_member == 0 && count == dst->p.batch;
  if (dst->loaded && src->phase != dst->phase && !whole)
    return fail(QHFPE_ESTATE, "copying %d of %d members with phase %d into a handle of phase %d", count,
                dst->p.batch, src->phase, dst->phase);
  const size_t mb = (size_t)src->L.member_elems * src->L.elem;
  // on different streams: the copy waits for src's pending work, and src's
  // later work waits for the copy (events only, so the call can be captured)
  const bool two = src->stream != dst->stream;
  if (two) {
    HIP_TRY(hipEventRecord(src->xevent, src->stream));
    HIP_TRY(hipStreamWaitEvent(dst->stream, src->xevent, 0));
  }
  HIP_TRY(launch_stream_copy(static_cast<char*>(dst->y()) + dst_member * mb,
                             static_cast<const char*>(src->y()) + src_member * mb, count * mb, dst->stream));
  if (two) {
    HIP_TRY(hipEventRecord(dst->xevent, dst->stream));
    HIP_TRY(hipStreamWaitEvent(src->stream, dst->xevent, 0));
  }
  dst->phase = src->phase;
  dst->loaded = true;
  return QHFPE_OK;
}

int qhfpe_closure_loss(const double* d_stats, const float* d_kernel, float* d_state, double* h_loss, void* stream) {
  if (!d_stats || !d_kernel || !d_state || !h_loss) return fail(QHFPE_EINVAL, "NULL pointer");
  using TL = ClosureTrainLayout;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* d_loss = reinterpret_cast<double*>(d_state + TL::loss);
  HIP_TRY(launch_closure_loss(d_stats, d_kernel, d_state + TL::gk, reinterpret_cast<double*>(d_state + TL::terms),
                              d_loss, s));
  HIP_TRY(hipMemcpyAsync(h_loss, d_loss, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return QHFPE_OK;
}

int qhfpe_closure_buffer_bytes(const qhfpe_params* params, size_t* bytes) {
  if (!bytes) return fail(QHFPE_EINVAL, "bytes is NULL");
  if (int rc = validate(params)) return rc;
  const Layout L = make_layout(params);
  *bytes = align_up((size_t)kClosureWeightElems * sizeof(unsigned short)) +
           align_up((size_t)L.level_elems * params->batch * L.elem);
  return QHFPE_OK;
}

int qhfpe_set_closure(qhfpe_t* h, const float* d_kernel, void* d_buffer, size_t bytes) {
  if (int rc = check_handle(h)) return rc;
  if (!d_kernel) {
    h->closure_wb = nullptr;
    h->closure_out = nullptr;
    return QHFPE_OK;
  }
  if (!wave_supported(h->ns, h->p.np))
    return fail(QHFPE_EUNSUPPORTED, "a learned closure needs two states and np = 128 or 256");
  if (h->mixed) return fail(QHFPE_EUNSUPPORTED, "a learned closure needs every member at the handle's depth");
  if (!d_buffer || reinterpret_cast<uintptr_t>(d_buffer) % kAlign)
    return fail(QHFPE_EINVAL, "d_buffer must be a 256-byte aligned device buffer");
  size_t need = 0;
  if (int rc = qhfpe_closure_buffer_bytes(&h->p, &need)) return rc;
  if (bytes < need) return fail(QHFPE_ESTATE, "closure buffer too small: %zu < %zu bytes", bytes, need);
  unsigned short* wb = static_cast<unsigned short*>(d_buffer);
  HIP_TRY(launch_closure_weights(d_kernel, wb, h->stream));
  h->closure_wb = wb;
  h->closure_out = static_cast<char*>(d_buffer) + align_up((size_t)kClosureWeightElems * sizeof(unsigned short));
  h->cpt = kTileWave;
  return QHFPE_OK;
}

int qhfpe_closure_stats(qhfpe_t* h, int32_t level, double* d_stats) {
  if (int rc = check_handle(h)) return rc;
  if (!d_stats) return fail(QHFPE_EINVAL, "d_stats is NULL");
  if (!wave_supported(h->ns, h->p.np))
    return fail(QHFPE_EUNSUPPORTED, "closure statistics need two states and np = 128 or 256");
  if (level < 0 || level >= h->p.depth) return fail(QHFPE_EINVAL, "need 0 <= level < depth (level + 1 is the target)");
  for (int b = 0; b < h->p.batch; ++b)
    if (h->mdepth[b] <= level)
      return fail(QHFPE_EUNSUPPORTED, "member %d (depth %d) has no level %d", b, h->mdepth[b], level + 1);
  HIP_TRY(launch_closure_stats(h->p.precision, h->p.np, h->y(), level, h->L.member_elems, h->L.level_elems,
                               h->L.comp_elems, h->p.nq, h->p.batch, h->p.p_min, h->dp, d_stats, h->stream));
  return QHFPE_OK;
}

int qhfpe_closure_gmfp_kernel(const qhfpe_t* h, float* h_kernel) {
  if (int rc = check_handle(h)) return rc;
  if (!h_kernel) return fail(QHFPE_EINVAL, "h_kernel is NULL");
  if (h->ns != 2) return fail(QHFPE_EUNSUPPORTED, "the closure is defined for two states");
  double bc[kBathStride];
  bath_constants(h->p, h->p.zeta, h->p.gamma, h->p.beta, bc);
  const double zeta = bc[0], c0 = bc[2];
  constexpr int S = 2 * kClosureHalf + 1;
  for (int e = 0; e < kClosureKernelElems; ++e) h_kernel[e] = 0.0f;
  auto at = [&](int dq, int dp, int ci, int co) -> float& {
    return h_kernel[((dq * S + dp) * kClosureIn + ci) * kClosureOut + co];
  };
  // W^(N+1) = zeta p W^(N) + c0 D_p W^(N), D_p the periodic fourth-order stencil
  const double w[5] = {1.0, -8.0, 0.0, 8.0, -1.0};  // taps p - 2 .. p + 2, times 1 / (12 dp)
  for (int c = 0; c < 4; ++c) {
    at(kClosureHalf, kClosureHalf, 4 + c, c) = (float)zeta;
    for (int s = -2; s <= 2; ++s)
      if (s != 0) at(kClosureHalf, kClosureHalf + s, c, c) = (float)(c0 * w[s + 2] / (12.0 * h->dp));
  }
  return QHFPE_OK;
}

int qhfpe_closure_train(const double* d_stats, const float* d_prior, double ridge, float* d_state, uint64_t seed,
                        int32_t iters, double lr, double lr_final, float* d_kernel, double* h_loss, void* stream) {
  if (!d_stats || !d_state || !d_kernel) return fail(QHFPE_EINVAL, "NULL pointer");
  if (iters < 0 || !(lr > 0) || !(lr_final > 0)) return fail(QHFPE_EINVAL, "need iters >= 0, lr > 0, lr_final > 0");
  if (!(ridge >= 0) || !std::isfinite(ridge)) return fail(QHFPE_EINVAL, "ridge must be finite and >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  using TL = ClosureTrainLayout;
  // seeded initial layers (uniform, variance 1 / fan-in: the composite of the
  // three layers starts at the scale of its inputs); zero Adam moments
  std::vector<float> init((size_t)TL::total, 0.0f);
  uint64_t x = seed;
  auto next = [&]() {  // splitmix64
    x += 0x9e3779b97f4a7c15ULL;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  };
  auto fill = [&](int off, int n, int fan_in) {
    const double a = std::sqrt(3.0 / fan_in);
    for (int i = 0; i < n; ++i) init[off + i] = (float)(a * (2.0 * ((next() >> 11) * (1.0 / 9007199254740992.0)) - 1.0));
  };
  fill(TL::w1, TL::n1, 25 * kClosureIn);
  fill(TL::w2, TL::n2, 25 * kClosureHidden);
  fill(TL::w3, TL::n3, 25 * kClosureHidden);
  if (d_prior) {
    // start at the prior: the first two layers pass the 8 input channels
    // through their centre taps (identity into hidden channels 0..7), the
    // third holds the prior's central 5 x 5 taps; the random weights stay,
    // scaled down, to break the symmetry of the hidden channels
    std::vector<float> k0(kClosureKernelElems);
    HIP_TRY(hipMemcpyAsync(k0.data(), d_prior, k0.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < TL::nparam; ++i) init[i] *= 1e-3f;
    constexpr int H = kClosureHidden, S = 2 * kClosureHalf + 1;
    for (int c = 0; c < kClosureIn; ++c) {
      init[TL::w1 + (12 * kClosureIn + c) * H + c] = 1.0f;  // tap (2, 2) is the centre of 5 x 5
      init[TL::w2 + (12 * H + c) * H + c] = 1.0f;
    }
    for (int tq = 0; tq < 5; ++tq)
      for (int tp = 0; tp < 5; ++tp)
        for (int c = 0; c < kClosureIn; ++c)
          for (int o = 0; o < kClosureOut; ++o)
            init[TL::w3 + ((tq * 5 + tp) * H + c) * kClosureOut + o] =
                k0[(((tq + kClosureHalf - 2) * S + (tp + kClosureHalf - 2)) * kClosureIn + c) * kClosureOut + o];
  }
  HIP_TRY(hipMemcpyAsync(d_state, init.data(), init.size() * sizeof(float), hipMemcpyHostToDevice, s));
  for (int t = 1; t <= iters; ++t) {
    // learning rate decays geometrically from lr to lr_final
    const double f = iters > 1 ? (double)(t - 1) / (iters - 1) : 0.0;
    const float lr_t = (float)(lr * std::pow(lr_final / lr, f));
    HIP_TRY(launch_closure_train_step(d_stats, d_prior, ridge, d_state, t, lr_t, nullptr, s));
  }
  // the composite kernel of the final layers and its normalised loss
  double* d_loss = reinterpret_cast<double*>(d_state + TL::loss);
  HIP_TRY(launch_closure_compose(d_stats, d_state, d_loss, s));
  HIP_TRY(hipMemcpyAsync(d_kernel, d_state + TL::k, kClosureKernelElems * sizeof(float), hipMemcpyDeviceToDevice, s));
  double loss = 0.0;
  HIP_TRY(hipMemcpyAsync(&loss, d_loss, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h_loss) *h_loss = loss;
  return QHFPE_OK;
}

int qhfpe_graph_begin(void* stream) {
  if (!stream) return fail(QHFPE_EINVAL, "graph capture needs a stream of its own (not the NULL stream)");
  HIP_TRY(hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal));
  return QHFPE_OK;
}

int qhfpe_graph_end(void* stream, qhfpe_graph_t** out) {
  if (!out) return fail(QHFPE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!stream) return fail(QHFPE_EINVAL, "stream is NULL");
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamEndCapture(static_cast<hipStream_t>(stream), &g));
  hipGraphExec_t x = nullptr;
  hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(QHFPE_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  size_t nodes = 0;
  e = hipGraphGetNodes(g, nullptr, &nodes);
  qhfpe_graph_t* r = e == hipSuccess ? new (std::nothrow) qhfpe_graph() : nullptr;
  if (!r) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    return e != hipSuccess ? fail(QHFPE_EHIP, "hipGraphGetNodes: %s", hipGetErrorString(e))
                           : fail(QHFPE_EINVAL, "out of host memory");
  }
  r->graph = g;
  r->exec = x;
  r->nodes = nodes;
  *out = r;
  return QHFPE_OK;
}

int qhfpe_graph_nodes(const qhfpe_graph_t* g, size_t* nodes) {
  if (!g || !nodes) return fail(QHFPE_EINVAL, "NULL pointer");
  *nodes = g->nodes;
  return QHFPE_OK;
}

int qhfpe_graph_launch(qhfpe_graph_t* g, void* stream) {
  if (!g) return fail(QHFPE_EINVAL, "graph is NULL");
  HIP_TRY(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return QHFPE_OK;
}

int qhfpe_graph_destroy(qhfpe_graph_t* g) {
  if (!g) return QHFPE_OK;
  const hipError_t a = hipGraphExecDestroy(g->exec), b = hipGraphDestroy(g->graph);
  delete g;
  if (a != hipSuccess || b != hipSuccess)
    return fail(QHFPE_EHIP, "destroying the graph: %s", hipGetErrorString(a != hipSuccess ? a : b));
  return QHFPE_OK;
}

int qhfpe_spectrum_abs(const double* d_series, int64_t n, double dt, const double* d_omega, int32_t n_omega,
                       double* d_out, void* stream) {
  if (!d_series || !d_omega || !d_out) return fail(QHFPE_EINVAL, "NULL pointer");
  // the trapezoid rule needs an interval: at least two samples
  if (n < 2 || n_omega < 1 || !(dt > 0)) return fail(QHFPE_EINVAL, "need n >= 2 samples, n_omega >= 1, dt > 0");
  HIP_TRY(launch_spectrum_abs(d_series, n, dt, d_omega, n_omega, d_out, static_cast<hipStream_t>(stream)));
  return QHFPE_OK;
}

int qhfpe_spectrum_corr(const double* d_r3, int32_t n1, int32_t n3, double dt1, double dt3, const double* d_w1,
                        int32_t n_w1, const double* d_w3, int32_t n_w3, double* d_work, double* d_out,
                        void* stream) {
  if (!d_r3 || !d_w1 || !d_w3 || !d_work || !d_out) return fail(QHFPE_EINVAL, "NULL pointer");
  if (n1 < 2 || n3 < 2 || n_w1 < 1 || n_w3 < 1 || !(dt1 > 0) || !(dt3 > 0))
    return fail(QHFPE_EINVAL, "need n1, n3 >= 2 samples, n_w1, n_w3 >= 1, dt1, dt3 > 0");
  if (n1 > 65535 || n_w3 > 65535) return fail(QHFPE_EINVAL, "n1 and n_w3 must be <= 65535");
  HIP_TRY(launch_spectrum_corr(d_r3, n1, n3, dt1, dt3, d_w1, n_w1, d_w3, n_w3, d_work, d_out,
                               static_cast<hipStream_t>(stream)));
  return QHFPE_OK;
}

int qhfpe_spectrum_corr_noalloc(const double* d_r3, int32_t n1, int32_t n3, double dt1, double dt3,
                                const double* d_w1, int32_t n_w1, const double* d_w3, int32_t n_w3, double* d_out,
                                void* stream) {
  if (!d_r3 || !d_w1 || !d_w3 || !d_out) return fail(QHFPE_EINVAL, "NULL pointer");
  if (n1 < 2 || n3 < 2 || n_w1 < 1 || n_w3 < 1 || !(dt1 > 0) || !(dt3 > 0))
    return fail(QHFPE_EINVAL, "need n1, n3 >= 2 samples, n_w1, n_w3 >= 1, dt1, dt3 > 0");
  if (n1 > 65535 || n_w3 > 65535) return fail(QHFPE_EINVAL, "n1 and n_w3 must be <= 65535");
  if ((size_t)n1 * (size_t)n_w3 * 2 > kScratchDoubles)
    return fail(QHFPE_EINVAL, "n1 * n_w3 = %lld exceeds the fixed scratch (%zu complex values)",
                (long long)n1 * n_w3, kScratchDoubles / 2);
  double* work = nullptr;
  HIP_TRY(scratch_pointer(&work));
  HIP_TRY(launch_spectrum_corr(d_r3, n1, n3, dt1, dt3, d_w1, n_w1, d_w3, n_w3, work, d_out,
                               static_cast<hipStream_t>(stream)));
  return QHFPE_OK;
}

}  // extern "C"
