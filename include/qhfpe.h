/*
 * qhfpe.h - C-ABI of the MI355X (gfx950) propagator for the multi-state
 * quantum hierarchical Fokker-Planck equation (MS-QHFPE) of
 * Ikeda & Tanimura, J. Chem. Phys. (2017), arXiv:1706.09590.
 *
 * The library integrates the hierarchy W^(n)_jk(p, q), n = 0..N, of
 * Sec. II, Eq. (heom) (one Drude exponential, V(q) = q, so Phi = -d/dp and
 * Lambda^(1) = -p/m), closed at n = N by Eq. (GMFP), with classical RK4.
 * The kinetic term uses the fifth-order upwind scheme and the potential
 * term of Eq. (quantum-liouvillian) is evaluated through a DFT along p, as
 * in Sec. III.  Impulsive dipole excitations and the trace Tr{mu W^(0)}
 * give the response functions of Sec. III, Eqs. (R1) and (R3), and the
 * spectra of Eqs. (I1), (I3) and (transient-absorption).
 *
 * Conventions shared by every entry point:
 *  - Return value: QHFPE_OK (0) or a negative QHFPE_E* code; the message of
 *    the last failure on the calling thread is qhfpe_last_error().
 *  - Every pointer named d_* is device memory on the GPU that is current
 *    when the handle is created; h_* is host memory.  The caller owns all
 *    memory, including the workspace; the library allocates no device
 *    memory and keeps non-owning pointers only (it does create the streams
 *    and events of qhfpe_step's member groups, see qhfpe_set_streams).
 *  - Work is enqueued on the handle's stream (qhfpe_step's member groups
 *    run on their own streams between an event fork and join on it).
 *    qhfpe_create, qhfpe_set_state, qhfpe_set_member_bath,
 *    qhfpe_set_member_depth, qhfpe_set_potential,
 *    qhfpe_set_potential_tables, qhfpe_autotune, qhfpe_step, qhfpe_status,
 *    qhfpe_residual and qhfpe_relax synchronise that stream before they
 *    return (they upload tables or read a result or a status flag back);
 *    the other calls are asynchronous.  Only asynchronous calls may be
 *    recorded into a graph (qhfpe_graph_begin); they enqueue kernels and
 *    event waits only (no memset or memcpy nodes).
 *  - A handle is used by one host thread at a time; different handles may
 *    be used from different threads.
 *  - Canonical state layout ("canon"): interleaved complex128 (re, im)
 *    doubles, index [member][n][j][k][i][a] with n = 0..N, states j, k,
 *    q nodes i (slowest of the grid) and p nodes a (fastest).
 *  - Grids are half-open: q_i = q_min + i (q_max - q_min)/nq,
 *    p_a = p_min + a (p_max - p_min)/np; p is periodic.
 *  - Units are those of the parameters; the response functions' factors
 *    (i/hbar)^k of Eqs. (R1), (R3) are NOT applied inside the library.
 */
#ifndef QHFPE_H
#define QHFPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  QHFPE_OK = 0,
  QHFPE_EINVAL = -1,       /* null pointer, size or value out of range */
  QHFPE_EUNSUPPORTED = -2, /* valid but not supported (np, n_states, coupling form, non-Hermitian state) */
  QHFPE_EHIP = -3,         /* HIP runtime error; message holds hipGetErrorString */
  QHFPE_ENONFINITE = -4,   /* NaN/Inf found in a response sample or norm */
  QHFPE_ESTATE = -5        /* call-order error (e.g. workspace too small, mismatched handles) */
};

enum { QHFPE_FP64 = 0, QHFPE_FP32_FP64RED = 1 };
enum { QHFPE_COMMUTATOR = 0 };
enum { QHFPE_MAX_STATES = 3 };

/* Model and discretisation.  Sec. II, Eqs. (system-Hamiltonian),
 * (Drude-J); Sec. III (mesh).  Entries of poly/mu beyond n_states are
 * ignored. */
typedef struct qhfpe_params {
  int32_t n_states;            /* electronic states, 2 or 3 */
  int32_t nq;                  /* q nodes, >= 4 */
  int32_t np;                  /* p nodes: 8,12,16,24,32,48,64,96,128,192 or 256 */
  int32_t depth;               /* hierarchy depth N >= 0 (levels 0..N) */
  int32_t batch;               /* 1 <= B <= 65535 independent members sharing this model */
  int32_t precision;           /* QHFPE_FP64, or QHFPE_FP32_FP64RED (FP32 state, FP64 traces) */
  int32_t low_temp_correction; /* 1: c0 = (m zeta hbar gamma/2) cot(beta hbar gamma/2), c_delta = m zeta/beta - c0;
                                  0: c0 = m zeta/beta, c_delta = 0 */
  int32_t reserved;            /* must be 0 */
  double q_min, q_max, p_min, p_max;
  double mass, hbar;
  double zeta, gamma, beta;    /* Drude bath: J(w) = (m zeta/pi) w gamma^2/(gamma^2 + w^2) */
  double dt;                   /* RK4 step.  Substeps are the caller's choice of dt and of
                                  qhfpe_step's sampling stride: s substeps per output interval T
                                  are dt = T / s with stride s (the response is still sampled
                                  every T). */
  /* U_jl(x) = sum_k poly[j][l][k] x^k.  Diagonal entries: any quartic.
   * Off-diagonal entries: constants (applied pointwise) or q-dependent
   * (k >= 1 non-zero; applied in the r-space multiply, see
   * qhfpe_set_potential).  poly must be symmetric in (j, l). */
  double poly[QHFPE_MAX_STATES][QHFPE_MAX_STATES][5];
  double mu[QHFPE_MAX_STATES][QHFPE_MAX_STATES]; /* real symmetric Condon dipole */
} qhfpe_params;

typedef struct qhfpe_handle qhfpe_t;

/* Bytes of device workspace a handle with these parameters needs.
 * Pure host call (validates the parameters; touches no GPU). */
int qhfpe_workspace_bytes(const qhfpe_params* params, size_t* bytes);

/* Create a handle.  d_workspace: device memory of >= qhfpe_workspace_bytes,
 * 256-byte aligned, owned by the caller and kept alive until
 * qhfpe_destroy.  stream: a hipStream_t (NULL = default stream).  The
 * state starts at zero with phase 0.  Parameter arrays are copied. */
int qhfpe_create(const qhfpe_params* params, void* d_workspace, size_t bytes,
                 void* stream, qhfpe_t** out);
int qhfpe_destroy(qhfpe_t* h);

/* Load a canonical state.  The state is W = i^phase H with H Hermitian in
 * (j, k) at every node (Sec. II: every hierarchy member of a Hermitian
 * density matrix is Hermitian; each impulsive mu^x multiplies by i).
 * member = -1 loads all B members from d_canon[B][...]; member >= 0 loads
 * that member from d_canon[1][...] (phase must then equal the handle's).
 * Returns QHFPE_EUNSUPPORTED when max |H_jk - conj(H_kj)| exceeds
 * 1e-12 max |H|.  Synchronous. */
int qhfpe_set_state(qhfpe_t* h, const double* d_canon, int32_t phase, int32_t member);

/* Write the canonical state: the hierarchy elements W^(n)_jk(p, q) of
 * Sec. II, Eq. (heom), n = 0..N, as full complex matrices in (j, k),
 * including the phase factor i^phase of the impulsive excitations (member
 * -1: all, into [B][...]; else one member into [1][...]). */
int qhfpe_get_state(qhfpe_t* h, double* d_canon, int32_t member);
int qhfpe_get_phase(const qhfpe_t* h, int32_t* phase);

/* Per-member Drude bath (Sec. II, Eq. (Drude-J)) for parameter sweeps in one
 * batch: member -1 sets all members.  At create every member takes the
 * params' zeta, gamma, beta; the low_temp_correction flag of the params
 * applies.  Synchronous. */
int qhfpe_set_member_bath(qhfpe_t* h, int32_t member, double zeta, double gamma, double beta);

/* Hierarchy depth of one batch member (Eq. (heom) truncated at its own
 * level N_b, closed there by Eq. (GMFP)), 0 <= depth <= params.depth; at
 * create every member has params.depth.  Members of different depths then
 * share each stage launch: the launch's units run over the levels each
 * member has, and the levels above a member's depth are neither computed
 * nor written (qhfpe_init_thermal leaves them zero; a state loaded with
 * qhfpe_set_state should hold zeros there, since they are carried along
 * unchanged).  Results of a member equal those of a handle of its own
 * depth bit for bit.  Not with a learned closure (QHFPE_EUNSUPPORTED).
 * Synchronous; QHFPE_ESTATE while the handle's stream records a graph;
 * QHFPE_EINVAL for a member or depth out of range.  With members of
 * different depths, qhfpe_apply_rhs and qhfpe_residual clear their scratch
 * state first (and refuse while recording). */
int qhfpe_set_member_depth(qhfpe_t* h, int32_t member, int32_t depth);

/* Potential surfaces from a host function instead of params.poly (Sec. II,
 * Eq. (system-Hamiltonian); the model of Sec. III has displaced Morse
 * diagonals and a Gaussian coupling, see qhfpe_morse_gauss_potential).
 * fn(j, l, x, ctx) must return U_jl(x) (same units as params.poly) for
 * 0 <= j <= l < n_states; U_lj = U_jl is implied.  The library calls fn on
 * the host, during this call only, at every point the r-space multipliers
 * of Eq. (quantum-liouvillian) need: q_i +- r_m / 2 clamped to the q grid,
 * with the Nyquist column averaged as for polynomial surfaces, and
 * replaces the multipliers of the handle.  fn and ctx are not kept.
 * If every off-diagonal U_jl takes one and the same value at all those
 * points, the coupling is applied pointwise as for a constant polynomial;
 * otherwise it is q-dependent and enters the r-space multiply, where
 * -(i/hbar) [U_jl(q + r/2) W_lk - W_jl U_lk(q - r/2)] mixes the diagonal and
 * coherence transforms of a column.  Two variants implement it: the
 * two-state wave variant (tile 1, np = 128 or 256) and the workgroup
 * variant with 2 cells per thread (tile 2, every np, two and three states).
 * The handle moves to one of them if its variant has no such path, and
 * qhfpe_set_tile with another variant fails until a potential with
 * constant couplings is set again.  Synchronous.
 * Errors: QHFPE_EINVAL (fn NULL, a non-finite value); on error the handle
 * keeps its previous surfaces. */
typedef double (*qhfpe_potential_fn)(int32_t j, int32_t l, double x, void* ctx);
int qhfpe_set_potential(qhfpe_t* h, qhfpe_potential_fn fn, void* ctx);

/* Potential surfaces given as the r-space tables of Eq.
 * (quantum-liouvillian) themselves: u_plus[j][l][i][m] = U_jl(q_i + r_m/2)
 * and u_minus[j][l][i][m] = U_jl(q_i - r_m/2), host FP64 arrays of
 * n_states x n_states x nq x np, row-major, with r_m = mh dr, dr =
 * 2 pi hbar / (np dp) and mh = m for m <= np/2, m - np above (the DFT order
 * of the transform along p).  Only the entries with j <= l are read (U_lj =
 * U_jl is implied).  The values are used as given: clamping the arguments
 * to the grid and the Nyquist column are the caller's (qhfpe_set_potential
 * applies the library's readings).  Couplings, variants and errors as for
 * qhfpe_set_potential: constant off-diagonal tables take the pointwise path,
 * anything else the r-space one.  The arrays are read during this call
 * only.  Synchronous.  Errors: QHFPE_EINVAL (NULL array, a non-finite
 * value); on error the handle keeps its previous surfaces. */
int qhfpe_set_potential_tables(qhfpe_t* h, const double* u_plus, const double* u_minus);

/* The two-state surfaces of Sec. III in the dimensionless coordinate:
 *   U_00 = D0 (1 - exp(-a0 (x - q0)))^2
 *   U_11 = D1 (1 - exp(-a1 (x - q1)))^2 + dE
 *   U_01 = dV exp(-(x - qs)^2 / (2 sigma^2)).
 * (The printed exponent is read with the sign and width a_j =
 * omega_j / sqrt(2 D_j omega_0) that reproduce the printed resonance
 * frequencies.)  A qhfpe_potential_fn: ctx points to a qhfpe_morse_gauss;
 * j or l outside {0, 1} returns NaN. */
typedef struct qhfpe_morse_gauss {
  double D0, D1, a0, a1, q0, q1, dE, dV, qs, sigma;
} qhfpe_morse_gauss;
double qhfpe_morse_gauss_potential(int32_t j, int32_t l, double x, void* ctx);

/* Tile variant of the fused RK stage.  2, 4, 8: each thread of a stage
 * workgroup owns cells_per_thread consecutive q columns (2, 4 or 8 for FP32
 * two-state; 2 or 4 for FP64 two-state and FP32 three-state; 2 for FP64
 * three-state).  1: the wave-independent variant, one 64-lane wave per
 * task of q columns, each lane holding np/64 consecutive p nodes: two
 * states at np = 128 or 256 (512/np columns per task); three states with
 * constant couplings at np = 128 (two columns per task) or 256 (one).  0 = default: 1 where available, else 4 (2 for three states); it
 * is also the variant at create.  With a q-dependent coupling only tile 2
 * and, for two states, tile 1 exist (see qhfpe_set_potential).  Variants compute the same operations per
 * cell; results agree to rounding (the compiled instruction order and the
 * grouping of the trace partial sums differ).  QHFPE_EUNSUPPORTED if the
 * variant does not exist for this precision, state count and np. */
int qhfpe_set_tile(qhfpe_t* h, int32_t cells_per_thread);

/* Pick the fastest tile variant for this handle by timing reps stage launches
 * of each (they read the state and write scratch only; the state is not
 * changed).  h_chosen (may be NULL) receives the variant.  Synchronous. */
int qhfpe_autotune(qhfpe_t* h, int32_t reps, int32_t* h_chosen);

/* Member groups of qhfpe_step (batching of independent propagations, as in
 * Sec. III's runs over baths and delays).  The members are split into
 * `groups` contiguous ranges; each range's stage launches go to a stream of
 * its own, created by the library on first use and destroyed with the handle,
 * so that the launches of different ranges overlap on the GPU.  qhfpe_step
 * still runs after earlier work on the handle's stream and before later work
 * (an event fork and join on that stream).  Results do not depend on the
 * grouping: every member is computed by the same kernels in the same order.
 * groups: 1 = one launch per stage for all members; 2..4 = that many ranges
 * (capped at the batch size); 0 = default (one group per member for batches
 * of up to 3 members, 2 groups for 4..16 members, else 1).  Only qhfpe_step (and qhfpe_relax through it) uses the groups.
 * QHFPE_EINVAL if groups is outside [0, 4]. */
int qhfpe_set_streams(qhfpe_t* h, int32_t groups);

/* Member groups qhfpe_step will use (after capping and the default rule). */
int qhfpe_get_streams(const qhfpe_t* h, int32_t* groups);

/* Initial state (Sec. III protocol; harmonic thermal Wigner function):
 * W^(0)_00(p, q) = tanh(b)/(pi hbar) exp(-tanh(b) [p^2/(m hbar omega) + m omega q^2/hbar]),
 * b = beta hbar omega/2 with each member's beta, plus d_noise[i][a] (FP64
 * [nq][np], may be NULL); every other entry 0, phase 0, all members. */
int qhfpe_init_thermal(qhfpe_t* h, double omega, const double* d_noise);

/* Impulsive excitation mu^x W = mu W - W mu on every level and member
 * (Sec. III, the commutator of the Condon dipole; no i/hbar factor).
 * Advances the phase by one. */
int qhfpe_apply_dipole(qhfpe_t* h, int32_t mode);

/* Advance nsteps RK4 steps of dt (Sec. II, Eqs. (heom), (GMFP)).  Each
 * step applies the classical RK4 polynomial in dt L as the product of its
 * two real quadratic factors (four stage launches; equal to Kutta's form
 * up to rounding).
 * If d_resp != NULL it receives, per member, the complex FP64 trace
 * Tr{mu W^(0)} (including i^phase) at t = 0 and after every stride steps:
 * d_resp[B][nsteps/stride + 1][2]; nsteps must be a multiple of stride.
 * Synchronous; returns QHFPE_ENONFINITE if a sample (or, without d_resp,
 * the final trace) is not finite.  QHFPE_ESTATE while the stream records a
 * graph (use qhfpe_step_async). */
int qhfpe_step(qhfpe_t* h, int64_t nsteps, int32_t stride, double* d_resp);

/* The same propagation, enqueued only: no status is read back, so the call
 * returns before the GPU work ends and can be recorded into a graph.  A
 * non-finite sample sets the handle's status flag, which stays set until
 * qhfpe_status (or qhfpe_step, which clears it first) reads it. */
int qhfpe_step_async(qhfpe_t* h, int64_t nsteps, int32_t stride, double* d_resp);

/* Wait for the handle's stream and report the status flag of the
 * propagations enqueued since the last check: QHFPE_ENONFINITE if a trace
 * sample was not finite (the flag is then cleared), else QHFPE_OK.
 * Synchronous (QHFPE_ESTATE while the stream records a graph). */
int qhfpe_status(qhfpe_t* h);

/* Current Tr{mu W^(0)} per member, d_out[B][2] (FP64, including i^phase):
 * the trace of Sec. III, Eqs. (R1) and (R3) at the present time of each
 * member, without the (i/hbar)^k factor. */
int qhfpe_response(qhfpe_t* h, double* d_out);

/* Test hook: state <- L(state), the right-hand side of Eq. (heom)/(GMFP),
 * with no time step. */
int qhfpe_apply_rhs(qhfpe_t* h);

/* h_out[B][2] (host): ||L W||_2 and ||W||_2 per member over the whole
 * hierarchy (canonical complex entries).  Synchronous. */
int qhfpe_residual(qhfpe_t* h, double* h_out);

/* Relax towards the correlated thermal equilibrium of the full hierarchy
 * (Sec. III protocol): step in chunks of check_every until every member has
 * ||L W|| / ||W|| < tol or max_steps is reached.  Outputs may be NULL.
 * Synchronous. */
int qhfpe_relax(qhfpe_t* h, double tol, int64_t max_steps, int32_t check_every,
                int64_t* h_steps_done, double* h_residual);

/* Copy count members src[src_member..] -> dst[dst_member..] device to
 * device (multi-time protocol of Sec. III: the states after G(t1) and
 * G(t2) seed the next propagations).  Both handles must share n_states,
 * nq, np, depth and precision; dst takes src's phase.  The phase is one per
 * handle, so a copy with another phase than dst's must cover all of dst's
 * members unless dst holds no state yet (created and never loaded by
 * qhfpe_set_state, qhfpe_init_thermal or a copy): QHFPE_ESTATE otherwise.
 * Each copied member must have the same depth in both handles
 * (qhfpe_set_member_depth; QHFPE_ESTATE otherwise).
 * Within one handle the two ranges must not overlap (QHFPE_EINVAL).  The
 * copy is a kernel on dst's stream; when the handles' streams differ it
 * waits for src's pending work and src's later work waits for it (events
 * only: the call stays asynchronous and can be recorded into a graph). */
int qhfpe_copy_members(const qhfpe_t* src, int32_t src_member, qhfpe_t* dst,
                       int32_t dst_member, int32_t count);

/* Learned hierarchy terminator (two states, np = 128 or 256).  In place of
 * Eq. (GMFP), which closes the hierarchy with W^(N+1) ~ (zeta p + c0 d/dp)
 * W^(N), a linear convolution F over (q, p) predicts W^(N+1) from W^(N):
 *   F(W)_co(q_i, p_a) = sum_{dq, dp, ci} K[dq][dp][ci][co] X_ci(q_{i+dq-6}, p_{a+dp-6}),
 * dq, dp = 0..12, X = (the packed components H00, H11, Re H01, Im H01 of
 * W^(N), then the same four times p), zero outside the q grid, periodic in p;
 * the output channels are the packed components of W^(N+1).  F acts on the
 * Hermitian part of each member's state (the phase i^k factors out, F being
 * linear).  K is the composition of three 5x5 layers 8 -> 32 -> 32 -> 4
 * without biases or activations (a closure of a linear equation is linear),
 * trained by gradient descent (qhfpe_closure_train) on second-moment
 * statistics of deep-hierarchy runs (qhfpe_closure_stats).  The analytic
 * closure is one such K, so the learned one can only improve the fit. */
enum {
  QHFPE_CLOSURE_KERNEL_FLOATS = 13 * 13 * 8 * 4,          /* K[13][13][8][4] */
  QHFPE_CLOSURE_STATS_DOUBLES = 25 * 25 * 8 * 8 + 13 * 13 * 8 * 4 + 1,
  QHFPE_CLOSURE_TRAIN_FLOATS = 203906
};

/* Accumulate (+=) into d_stats the statistics of the training pairs
 * (level, level + 1) of every member's current state, FP64:
 *   A[dq][dp][ci][cj] = sum_x X_ci(x) X_cj(x + (dq - 12, dp - 12)),  dq, dp = 0..24,
 *   C[dq][dp][ci][co] = sum_x X_ci(x + (dq - 6, dp - 6)) Y_co(x),      dq, dp = 0..12,
 *   yy = sum_x sum_co Y_co(x)^2,
 * stored in that order (X of level `level`, Y the packed level + 1; zero
 * outside the q grid, periodic in p).  The caller zeroes d_stats
 * (QHFPE_CLOSURE_STATS_DOUBLES) before the first call.  0 <= level < depth
 * (QHFPE_EINVAL), and every member must have level + 1
 * (qhfpe_set_member_depth; QHFPE_EUNSUPPORTED).  Asynchronous. */
int qhfpe_closure_stats(qhfpe_t* h, int32_t level, double* d_stats);

/* The kernel K whose closure is Eq. (GMFP), W^(N+1) = zeta p W^(N) +
 * c0 d/dp W^(N) (fourth-order periodic d/dp), for the handle's bath and grid
 * (the params' zeta, gamma, beta): h_kernel[QHFPE_CLOSURE_KERNEL_FLOATS]
 * (host).  The prior of qhfpe_closure_train. */
int qhfpe_closure_gmfp_kernel(const qhfpe_t* h, float* h_kernel);

/* Train the three layers by Adam (iters steps, learning rate decaying
 * geometrically from lr to lr_final, seeded uniform initial layers) on
 *   [ sum (F(X) - Y)^2 + ridge * d * ||K - K0||^2 ] / yy,
 * written through d_stats (in which sum_x X(x + e) X(x + e') is A[e' - e],
 * exact for states that vanish within 12 rows of the q edges), with d the
 * mean zero-offset channel energy (1/8) sum_c A[12][12][c][c] and K0 = d_prior
 * (device FP32 kernel, e.g. qhfpe_closure_gmfp_kernel; NULL = 0).  The ridge
 * term keeps the taps the data do not determine at the prior: a closure fit
 * to the data alone can give the closed hierarchy growing modes.  With a
 * prior the layers start at it (identity through the centre taps of the
 * first two layers, the prior's central 5 x 5 taps in the third; taps of the
 * prior outside them are dropped), plus seeded weights of 1e-3 of that
 * scale; without one from the seeded weights alone.  d_state:
 * QHFPE_CLOSURE_TRAIN_FLOATS of device scratch (layers, gradients,
 * moments).  d_kernel receives the composite K (FP32,
 * QHFPE_CLOSURE_KERNEL_FLOATS), h_loss (may be NULL) its normalised data
 * loss sum (F(X) - Y)^2 / yy.  Runs on stream; synchronous. */
int qhfpe_closure_train(const double* d_stats, const float* d_prior, double ridge, float* d_state, uint64_t seed,
                        int32_t iters, double lr, double lr_final, float* d_kernel, double* h_loss, void* stream);

/* The normalised data loss sum (F(X) - Y)^2 / yy of the kernel d_kernel
 * (device FP32) on the statistics d_stats, into *h_loss; d_state: device
 * scratch of QHFPE_CLOSURE_TRAIN_FLOATS (its layers are not touched).  Runs
 * on stream; synchronous. */
int qhfpe_closure_loss(const double* d_stats, const float* d_kernel, float* d_state, double* h_loss, void* stream);

/* Bytes of the device buffer qhfpe_set_closure needs for these parameters
 * (the BF16 weights and the predicted level of every member).  Host call. */
int qhfpe_closure_buffer_bytes(const qhfpe_params* params, size_t* bytes);

/* Use the closure K (device FP32 K[13][13][8][4], read during this call) at
 * the deepest level of every later stage (qhfpe_step, qhfpe_apply_rhs,
 * qhfpe_residual, qhfpe_relax): before each stage the library evaluates
 * F(W^(N)) of the stage input with BF16 inputs and weights on the matrix
 * cores (FP32 accumulation) into d_buffer (256-byte aligned, at least
 * qhfpe_closure_buffer_bytes, kept alive while the closure is set: the BF16
 * weights, 57344 bytes, then the predicted levels [B][4][nq][np] in the
 * state precision), and the stage uses it as W^(N+1) (no Eq. (GMFP) terms).  d_kernel = NULL switches
 * back to Eq. (GMFP).  The wave variant only (QHFPE_EUNSUPPORTED otherwise);
 * the handle switches to it.  Asynchronous. */
int qhfpe_set_closure(qhfpe_t* h, const float* d_kernel, void* d_buffer, size_t bytes);

/* Device-to-device copy of bytes (d_dst, d_src 16-byte aligned, ranges
 * not overlapping) by the library's streaming kernel: 16-byte loads and
 * stores per lane, every lane's loads issued before its stores.  It is the
 * copy qhfpe_copy_members uses, and the plain copy of known size that
 * bandwidth measurements compare against.  Asynchronous on stream. */
int qhfpe_stream_copy(void* d_dst, const void* d_src, size_t bytes, void* stream);

/* Graphs of the asynchronous calls (the multi-time protocol of Sec. III as
 * one launch).  qhfpe_graph_begin starts recording what this thread
 * enqueues on stream (hipStreamBeginCapture, thread-local mode; stream must
 * not be NULL); library calls on handles of that stream are then recorded,
 * not run.  Synchronous calls fail while recording.  Host-side bookkeeping
 * (each handle's phase) advances at recording time, so a graph replays the
 * recorded sequence: a graph that should give the same result on every
 * launch starts by loading its initial state (e.g. qhfpe_copy_members from
 * a handle that holds it).  qhfpe_graph_end ends the recording and
 * instantiates the graph; qhfpe_graph_launch runs it on a stream;
 * qhfpe_graph_nodes reports its node count. */
typedef struct qhfpe_graph qhfpe_graph_t;
int qhfpe_graph_begin(void* stream);
int qhfpe_graph_end(void* stream, qhfpe_graph_t** out);
int qhfpe_graph_nodes(const qhfpe_graph_t* g, size_t* nodes);
int qhfpe_graph_launch(qhfpe_graph_t* g, void* stream);
int qhfpe_graph_destroy(qhfpe_graph_t* g);

/* Sec. III, Eq. (I1) (and Eq. (transient-absorption) for an R3(t, T, 0)
 * series): d_out[w] = omega_w Im sum_s c_s dt exp(i omega_w s dt) R[s],
 * trapezoid weights c_s, no window.  d_series: complex [n][2], n >= 2
 * (QHFPE_EINVAL otherwise: one sample spans no interval). */
int qhfpe_spectrum_abs(const double* d_series, int64_t n, double dt, const double* d_omega,
                       int32_t n_omega, double* d_out, void* stream);

/* Sec. III, Eqs. (I3), (nonreph), (reph) for one waiting time:
 * d_out[w3][w1] = Im sum_{t1,t3} c c dt1 dt3 e^{i w3 t3} (e^{i w1 t1} + e^{-i w1 t1}) R3[t1][t3].
 * d_r3: complex [n1][n3][2]; d_work: >= n1 * n_w3 * 2 doubles of scratch;
 * n1, n3 >= 2 and n1, n_w3 <= 65535 (QHFPE_EINVAL otherwise). */
int qhfpe_spectrum_corr(const double* d_r3, int32_t n1, int32_t n3, double dt1, double dt3,
                        const double* d_w1, int32_t n_w1, const double* d_w3, int32_t n_w3,
                        double* d_work, double* d_out, void* stream);

/* qhfpe_spectrum_corr without the d_work argument, for callers that cannot
 * allocate device memory (code under graph capture, serving loops, hosts
 * that forbid allocation): the t3 partial sums go to a fixed device array
 * of the library (1 MiB per GPU, held until the process ends), so the call
 * allocates nothing.  Limit: n1 * n_w3 <= 65536 (QHFPE_EINVAL above it);
 * other arguments, results and errors as qhfpe_spectrum_corr.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (on different
 * streams, or from different threads) race and must be ordered by the
 * caller. */
int qhfpe_spectrum_corr_noalloc(const double* d_r3, int32_t n1, int32_t n3, double dt1, double dt3,
                                const double* d_w1, int32_t n_w1, const double* d_w3, int32_t n_w3,
                                double* d_out, void* stream);

/* Message of the last failure on this thread ("" if none). */
const char* qhfpe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QHFPE_H */
