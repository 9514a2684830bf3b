/*
 * nfr.h -- C ABI of the MI355X (gfx950) library for RBF neural fields on surfaces.
 *
 * The library applies and time-steps the discrete nonlocal operator of the
 * discrete collocation scheme (paper section 2.2, eq. NFODETilde; the forcing
 * term enters only through nfr_integrate_forced):
 *
 *     u_i'(t) = -u_i + K_i(u),    K_i(u) = sum_{j=0}^{N-1} w(|x_i - x_j|) q_j f(u_j),
 *
 * over N nodes x_i on a surface with quadrature weights q_j (the mu_j of eq.
 * NFODETilde, produced by RBF-QF, paper section 3; nfr_quad_weights computes
 * them), a radial Mexican-hat kernel w of the chordal distance (or of the
 * doubly periodic distance of eq. dist for nfr_problem_create_periodic) and
 * the sigmoid firing rate f of eq. firing_rate.  The sum runs over every j,
 * j = i included.
 *
 * Conventions shared by every call:
 *   - Every call returns an int status: NFR_OK (0) or a negative NFR_ERR_*.
 *     nfr_last_error() gives a message for the calling thread's last failure.
 *     No C++ exception crosses this interface.
 *   - Pointers named *_dev are device pointers on the context's GPU; pointers
 *     named *_host are host pointers.  All memory is owned by the caller; the
 *     library never allocates device memory and never frees caller memory.
 *     Scratch space comes from a caller-supplied workspace whose size the
 *     matching nfr_*_workspace_size() call returns.
 *   - Device work is enqueued on the stream given at context creation; calls
 *     return after enqueueing (unless stated otherwise) and the caller
 *     synchronises.  Arguments are validated on the host before anything is
 *     enqueued; a failed call enqueues nothing.
 *   - A state array of B states is stored state-major: element (i, b) of an
 *     N x B array lives at [b * N + i] (each state contiguous, FP64).
 *   - One context per thread, or external locking.
 */
#ifndef NFR_H
#define NFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NFR_VERSION_MAJOR 0
#define NFR_VERSION_MINOR 1
#define NFR_VERSION_PATCH 0

enum nfr_status_code {
  NFR_OK = 0,
  NFR_ERR_INVALID_ARG = -1,      /* null pointer, bad size or enum, inconsistent arguments */
  NFR_ERR_NONFINITE = -2,        /* a scalar argument is NaN or infinite */
  NFR_ERR_NO_DEVICE = -3,        /* no HIP device with that index */
  NFR_ERR_UNSUPPORTED_ARCH = -4, /* the device is not gfx950 */
  NFR_ERR_HIP = -5,              /* a HIP runtime call failed */
  NFR_ERR_WORKSPACE = -6,        /* workspace or buffer smaller than required */
  NFR_ERR_INTERNAL = -7
};

/* Kernel families w(r), r = |x - y| chordal distance (unnormalised Mexican hats;
 * the paper's eq. winh is the normalised Gaussian version):
 *   NFR_KERNEL_GAUSS_MH: w(r) = A_e exp(-r^2 / s_e^2) - A_i exp(-r^2 / s_i^2)
 *   NFR_KERNEL_EXP_MH:   w(r) = A_e exp(-r / s_e)     - A_i exp(-r / s_i)      */
enum nfr_kernel_kind { NFR_KERNEL_GAUSS_MH = 0, NFR_KERNEL_EXP_MH = 1 };

typedef struct {
  int kind;            /* nfr_kernel_kind */
  double A_e, s_e;     /* excitatory amplitude and length scale, s_e > 0 */
  double A_i, s_i;     /* inhibitory amplitude and length scale, s_i > 0 */
} nfr_kernel;

/* Sigmoid firing rate f_b(u) = 1 / (1 + exp(-beta (u - theta_b))) (eq. firing_rate).
 * theta_b = theta_dev[b] when theta_dev is non-NULL (device, B doubles), else theta. */
typedef struct {
  double beta;               /* gain, beta >= 0 (beta = 0 gives f = 1/2) */
  double theta;              /* threshold shared by all states */
  const double* theta_dev;   /* optional per-state thresholds (device), may be NULL */
} nfr_firing;

/* How the operator is evaluated.
 *   ONTHEFLY_FP32: kernel values recomputed for every pair in FP32, FP32 sums
 *                  over source tiles, FP64 combination of tile sums.
 *   W_FP32:        W_ij = w(|x_i - x_j|) q_j precomputed once in FP32 (row-major,
 *                  N x Npad) and streamed from HBM at every application.
 *   W_BF16X3 / W_FP16X3: W split as hi + lo in BF16 / FP16 and applied on the
 *                  matrix cores with FP32 accumulation (three products,
 *                  hi*hi + hi*lo + lo*hi; f(u) split the same way).  Meant
 *                  for blocks of states (states are processed 32 or 64 at a
 *                  time; B = 1 works but wastes the matrix cores).
 *   ONTHEFLY_BF16X3 / ONTHEFLY_FP16X3: the same split products on the matrix
 *                  cores, with every W entry evaluated in FP32 on the fly
 *                  and split in registers: no W matrix (w_dev is ignored)
 *                  and no N^2 memory; each kernel value serves 32 or 64
 *                  states at once.
 *   ONTHEFLY_FP32_MFMA: the ONTHEFLY_FP32 arithmetic (FP32 kernel values,
 *                  products and 256-source sums, FP64 beyond) with the
 *                  products on the FP32 matrix cores: for blocks of states
 *                  (32 or 64 at a time), the vector units only evaluate the
 *                  kernel.  No W matrix.
 *   AUTO:          the library picks an FP32-class form that needs no W
 *                  matrix: ONTHEFLY_FP32_MFMA for B > 16, ONTHEFLY_FP32
 *                  otherwise (workspace sizes follow the same choice). */
enum nfr_form {
  NFR_FORM_AUTO = -1,
  NFR_FORM_ONTHEFLY_FP32 = 0,
  NFR_FORM_W_FP32 = 1,
  NFR_FORM_W_BF16X3 = 2,
  NFR_FORM_W_FP16X3 = 3,
  NFR_FORM_ONTHEFLY_BF16X3 = 4,
  NFR_FORM_ONTHEFLY_FP16X3 = 5,
  NFR_FORM_ONTHEFLY_FP32_MFMA = 6
};

typedef struct nfr_context nfr_context;
typedef struct nfr_problem nfr_problem;
typedef struct nfr_batch nfr_batch;

/* ---------------------------------------------------------------- status */

int nfr_version(int* major, int* minor, int* patch);
/* Static string naming a status code (never NULL). */
const char* nfr_status_string(int status);
/* Message of the calling thread's most recent failed call ("" if none). */
const char* nfr_last_error(void);

/* ---------------------------------------------------------------- context */

/* Binds a HIP device and stream.  `hip_stream` is a hipStream_t (NULL = the
 * default stream).  Fails with NFR_ERR_UNSUPPORTED_ARCH unless the device is
 * gfx950.  The context is host memory owned by the library until destroy. */
int nfr_context_create(int device, void* hip_stream, nfr_context** out);
int nfr_context_destroy(nfr_context* ctx);
/* Name of the device architecture the context runs on (e.g. "gfx950"). */
const char* nfr_context_arch(const nfr_context* ctx);

/* Timing of pair-sum launches (the operator's dominant kernel) with HIP events
 * recorded on the context stream around each launch; not recorded for launches
 * replayed from graphs.  When time stepping a single state of at most 4096
 * padded nodes, the timed launch also applies the RK4 stage update (one
 * launch per stage).  set_timing(ctx, 1) starts a fresh measurement;
 * nfr_context_timing synchronises the stream and returns the number of timed
 * launches and their summed duration in milliseconds, then resets. */
int nfr_context_set_timing(nfr_context* ctx, int enable);
int nfr_context_timing(nfr_context* ctx, int64_t* launches, double* total_ms);

/* Size of the HIP graph that the last graph-replayed nfr_integrate or
 * nfr_batch_integrate call on this context replayed: its node count (kernel
 * launches) and the RK4 steps it holds (both 0 if none yet).  Host-only. */
int nfr_context_last_graph(const nfr_context* ctx, int64_t* nodes, int64_t* steps);

/* Roofline microbenchmarks (synchronous).  Rates returned in *rate:
 *   FMA, EXP, SQRT: FP32 lane-operations per second (v_fma / v_exp / v_sqrt),
 *                   `size` = iterations of 8 independent chains per thread;
 *   HBM_READ:       bytes per second reading `size` floats from buf_dev;
 *   HBM_COPY:       bytes per second (read + write) copying `size` floats from
 *                   the first half of buf_dev to the second half;
 *   MFMA_BF16:      FLOP per second of 32x32x16 BF16 MFMA, `size` iterations;
 *   FMA_VOP3:       as FMA with the three-operand encoding (x <- x*m + b);
 *   FMA_EXP:        lane-operations per second of a mix of one exp2 and three
 *                   accumulating FMAs per chain and iteration;
 *   MFMA_F32:       FLOP per second of 32x32x2 FP32 MFMA, `size` iterations;
 *   MFMA_F32_FMA:   MFMA FLOP per second of two 32x32x2 FP32 MFMA chains run
 *                   beside eight FMA chains (32 FMAs per iteration, no data
 *                   shared): equal to MFMA_F32 if the vector units run while
 *                   the matrix cores do, half of it if the two alternate;
 *   MFMA_BF16_FMA:  the same with four 32x32x16 BF16 MFMAs per iteration;
 *   MFMA_BF16_DOT2: the four BF16 MFMAs beside 32 v_dot2c_f32_bf16 (eight
 *                   chains) per iteration;
 *   MFMA_BF16_MASK: the four BF16 MFMAs beside 16 masks and 16 FMAs (eight
 *                   chains of x <- x - 2^-30 (x & 0xffff0000)) per iteration.
 * buf_dev must hold 4*size bytes plus one float per thread of a grid of
 * 8 workgroups per compute unit (HBM_READ), 8*size bytes (HBM_COPY), or one
 * float per thread (others). */
enum nfr_probe_kind {
  NFR_PROBE_FMA = 0,
  NFR_PROBE_EXP = 1,
  NFR_PROBE_SQRT = 2,
  NFR_PROBE_HBM_READ = 3,
  NFR_PROBE_HBM_COPY = 4,
  NFR_PROBE_MFMA_BF16 = 5,
  NFR_PROBE_FMA_VOP3 = 6,
  NFR_PROBE_FMA_EXP = 7,
  NFR_PROBE_MFMA_F32 = 8,
  NFR_PROBE_MFMA_F32_FMA = 9,
  NFR_PROBE_MFMA_BF16_FMA = 10,
  NFR_PROBE_MFMA_BF16_DOT2 = 11,
  NFR_PROBE_MFMA_BF16_MASK = 12
};
int nfr_probe(nfr_context* ctx, int which, int64_t size, void* buf_dev, size_t buf_bytes, double* rate);

/* ---------------------------------------------------------------- problem */

/* Bytes of device memory a packed problem of n nodes occupies. */
size_t nfr_problem_bytes(int64_t n);

/* Packs a node set (paper section 2.1: nodes Xi; section 2.2: weights mu_j)
 * into `pack_dev` (caller-owned, >= nfr_problem_bytes(n) bytes, 256-byte
 * aligned):  coordinates become FP32 (x, y, z) padded to a multiple of 256
 * nodes, weights stay FP64; padding nodes carry weight 0 and never
 * contribute.  xyz_dev: n x 3 row-major FP64 (device); q_dev: n FP64 (device).
 * The inputs are read by a kernel enqueued on the context stream and may be
 * freed once it has run.  The handle (host memory) references pack_dev, which
 * must stay allocated until nfr_problem_destroy.  The pack also holds a tile
 * order of the nodes (recursive bisection along each segment's longest axis
 * down to blocks of 16 nodes, built on the device by bitonic sorts), in which
 * the fused BF16 form runs so that blocks of nearby nodes can skip the steep
 * exponential; every call still takes and returns states in the caller's
 * node order. */
int nfr_problem_create(nfr_context* ctx, int64_t n, const double* xyz_dev, const double* q_dev,
                       void* pack_dev, size_t pack_bytes, nfr_problem** out);

/* As nfr_problem_create, for a node set on a doubly periodic plane: the flat
 * domains of the paper's section 4 with the distance of eq. dist, the length
 * of x - y + L (i, j, 0) minimised over i, j in {-1, 0, 1}, L = `period`.
 * Every pair kernel, W build and adjoint of this problem then uses that
 * distance; z enters unchanged (the paper's flat domains have z = 0).  The
 * packed x and y are reduced by whole periods to [-L/2, L/2] (the same points
 * of the periodic plane), so the nine shifts find the nearest image for any
 * input coordinates.  period = 0 is nfr_problem_create; period < 0 or
 * non-finite is NFR_ERR_INVALID_ARG / NFR_ERR_NONFINITE.  Distances are
 * evaluated in FP32 from FP32 coordinates on the on-the-fly path, so the
 * rounding of a coordinate is about L 2^-25: keep L / s_e moderate (the
 * kernel's relative error grows like (r / s_e) (L / s_e) 2^-24). */
int nfr_problem_create_periodic(nfr_context* ctx, int64_t n, const double* xyz_dev, const double* q_dev,
                                double period, void* pack_dev, size_t pack_bytes, nfr_problem** out);
/* The period of a problem (0: not periodic; -1 for NULL). */
double nfr_problem_period(const nfr_problem* prob);
int nfr_problem_destroy(nfr_problem* prob);
int64_t nfr_problem_n(const nfr_problem* prob);
/* Padded node count (multiple of 256): the row stride of a W matrix. */
int64_t nfr_problem_npad(const nfr_problem* prob);

/* Far blocks of the fused BF16 form (ONTHEFLY_BF16X3) for this problem and
 * kernel: an application evaluates W in blocks of 32 target rows by 16 source
 * columns of the tile order, and a block whose bounding spheres are so far
 * apart that every pair has (1 - rho) t > 27 - log2|kappa| (paper eq. winh's
 * Mexican hat with the excitatory exponential the steeper one: t =
 * r^2 log2(e) / s_e^2, rho = s_e^2 / s_i^2, kappa = -A_i / A_e) takes only the
 * inhibitory exponential, the excitatory one being below half a unit in the
 * last place of the FP32 sum.  Returns the number of such blocks and of all
 * blocks ((npad / 32) x (npad / 16)); far_blocks = 0 when the kernel is not
 * eligible (not Gaussian, periodic, an integer length ratio, rho > 3/4,
 * |kappa| < 2^-20, or coordinates so large against s_e that the kernel
 * evaluates r^2 from differences: log2(e) max|x|^2 / s_e^2 > 96).  ws_dev: caller-owned device scratch of at least
 * nfr_far_blocks_workspace_size(prob) bytes.  Synchronises the context stream;
 * a diagnostic (the cost scales as npad^2 / 512), not part of the hot path. */
size_t nfr_far_blocks_workspace_size(const nfr_problem* prob);
int nfr_far_blocks(nfr_problem* prob, const nfr_kernel* kernel, void* ws_dev, size_t ws_bytes,
                   int64_t* far_blocks, int64_t* total_blocks);

/* ---------------------------------------------------------------- W form */

/* Bytes of a precomputed W for n nodes in a W_* form (0 for other forms). */
size_t nfr_w_bytes(int64_t n, int form);

/* Builds W_ij = w(|x_i - x_j|) q_j (paper eq. NFODETilde: kernel times quadrature
 * weight) for targets i < n and sources j < npad into `w_dev` (caller-owned,
 * >= nfr_w_bytes(n, form), 256-byte aligned).  Rows are targets, row stride
 * npad elements.  For W_BF16X3 / W_FP16X3 the buffer holds a 256-byte header
 * then the hi and lo matrices, each npad x npad (rows >= n zero), as 32 x 16
 * tiles in matrix-core operand order, hi and lo tiles interleaved in groups
 * of four row blocks (an opaque layout: only nfr_apply / nfr_integrate read
 * it);
 * W is scaled by 2^s, s = 14 - ceil(log2((|A_e| + |A_i|) max|q|)) for FP16
 * (0 for BF16), so that FP16 neither overflows nor underflows; s is stored in
 * the header and undone when W is applied. */
int nfr_w_build(nfr_problem* prob, const nfr_kernel* kernel, int form, void* w_dev, size_t w_bytes);

/* ---------------------------------------------------------------- operator */

size_t nfr_apply_workspace_size(const nfr_problem* prob, int B, int form);

/* One operator application (paper eq. NFODETilde, the sum K~):
 *   y_dev[b*n + i] = sum_j w(|x_i - x_j|) q_j f_b(u_dev[b*n + j]),  i < n, b < B.
 * u_dev, y_dev: n x B FP64 (device, state-major, must not overlap).  For W_*
 * forms `w_dev` is the matrix from nfr_w_build with the same kernel (it is
 * ignored otherwise and may be NULL). */
int nfr_apply(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B,
              const double* u_dev, double* y_dev, int form, const void* w_dev,
              void* ws_dev, size_t ws_bytes);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): nfr_apply without a
 * workspace.  Same arguments, kernels and results as nfr_apply (bit for bit);
 * its scratch (the sources g and the partial sums) lives in a fixed device
 * array of NFR_APPLY_NOALLOC_MAX_BYTES inside the library, one per GPU,
 * held until the process ends.  An application whose
 * nfr_apply_workspace_size exceeds that size fails with NFR_ERR_WORKSPACE
 * before anything is enqueued.  The call allocates nothing (no hipMalloc, no
 * library allocation).  Every call on one GPU shares that GPU's array and the
 * kernels overwrite every scratch byte they read (nothing needs clearing), so
 * calls whose work overlaps on one GPU (other streams, other threads, other
 * contexts on the same device) race: serialise them. */
#define NFR_APPLY_NOALLOC_MAX_BYTES (64u << 20)
int nfr_apply_noalloc(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B,
                      const double* u_dev, double* y_dev, int form, const void* w_dev);

/* ---------------------------------------------------------------- time stepping */

size_t nfr_integrate_workspace_size(const nfr_problem* prob, int B, int form);

/* Classical fourth-order Runge-Kutta with fixed step dt for `steps` steps of
 * u' = -u + K(u) (paper eq. NFODETilde; the stepper is this library's choice):
 *   k_s = -v_s + K(v_s),  v_1 = u,  v_2 = u + dt/2 k_1,  v_3 = u + dt/2 k_2,
 *   v_4 = u + dt k_3,     u <- u + dt/6 (k_1 + 2 k_2 + 2 k_3 + k_4),
 * with every state update in FP64.  u_dev (n x B FP64) holds u(0) on entry and
 * u(steps * dt) on exit; integration can resume from any state.  If ckpt_dev is
 * non-NULL it receives u at steps 0, ckpt_every, 2 ckpt_every, ... (each n x B,
 * consecutive; 1 + steps / ckpt_every of them).  use_graph != 0 (a
 * non-default stream is required) replays groups of up to 64 RK4 steps from
 * one captured HIP graph (with checkpoints the group length divides
 * ckpt_every); the graph is kept with the problem and replayed again by later
 * calls with the same arguments and workspace, so repeated integrations pay
 * one capture.  Steps beyond the last whole group are launched directly.
 * Results are bitwise those of use_graph == 0. */
int nfr_integrate(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B,
                  double* u_dev, double dt, int64_t steps, int form, const void* w_dev,
                  double* ckpt_dev, int64_t ckpt_every, int use_graph,
                  void* ws_dev, size_t ws_bytes);

/* RK4 for the forced equation u' = -u + K(u) + gamma(t) (paper eq. NFODETilde
 * with its forcing term gamma_i(t) = g(t, x_i); used with manufactured
 * solutions, eq. manufactured_system).  forcing_dev (device, FP64) holds, for
 * every step n, gamma at t_n, t_n + dt/2 and t_n + dt: layout
 * [steps][3][B][n].  The workspace is nfr_integrate_workspace_size's; other
 * arguments as nfr_integrate (no checkpoints, no graph replay). */
int nfr_integrate_forced(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, double* u_dev,
                         double dt, int64_t steps, const double* forcing_dev, int form, const void* w_dev,
                         void* ws_dev, size_t ws_bytes);

/* Adams-Bashforth 5 with fixed step dt for `steps` steps of u' = -u + K(u), the
 * stepper the paper's section 5.1 showcase uses: one operator application per
 * step, u_{n+1} = u_n + dt/720 (1901 F_n - 2774 F_{n-1} + 2616 F_{n-2}
 * - 1274 F_{n-3} + 251 F_{n-4}), F(u) = -u + K(u), state updates in FP64.  The
 * first four steps are classical RK4 (whose first stage gives F(u_n)).
 * Arguments as nfr_integrate (no checkpoints, no graph replay). */
size_t nfr_integrate_ab5_workspace_size(const nfr_problem* prob, int B, int form);
int nfr_integrate_ab5(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, double* u_dev,
                      double dt, int64_t steps, int form, const void* w_dev, void* ws_dev, size_t ws_bytes);

/* Neural field with synaptic depression (paper section 5.2, eq. nfsyndep), the
 * efficacy a acting on the presynaptic side of the integral:
 *   u' = -u + sum_j w_ij q_j a_j f(u_j),    tau a' = 1 - a - beta_d a f(u),
 * classical RK4 on the pair, on-the-fly FP32 pair sums, FP64 state updates.
 * u_dev and a_dev: n x B FP64 (device), advanced in place. */
size_t nfr_integrate_syndep_workspace_size(const nfr_problem* prob, int B);
int nfr_integrate_syndep(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, double* u_dev,
                         double* a_dev, double tau, double beta_d, double dt, int64_t steps, void* ws_dev,
                         size_t ws_bytes);

/* ---------------------------------------------------------------- uneven batch */

/* Groups P problems of one context (any mix of node counts, kernels, firing
 * rates and state counts B[p]) that are time-stepped together: each RK4 stage
 * is one persistent on-the-fly pair-sum launch over a cost-sorted list of work
 * items (problem, target tile, source chunk, state block) plus one combine
 * launch for all problems.  Arrays are copied; the problems must outlive the
 * batch.  Host memory only. */
int nfr_batch_create(nfr_context* ctx, int P, nfr_problem* const* probs, const nfr_kernel* kernels,
                     const nfr_firing* firings, const int* B, nfr_batch** out);
int nfr_batch_destroy(nfr_batch* batch);
/* Workspace bytes for nfr_batch_integrate / nfr_batch_tune (any configuration). */
size_t nfr_batch_workspace_size(const nfr_batch* batch);
/* Tile configuration: source-chunk length (multiple of 256, >= 1024) and
 * persistent workgroups per compute unit. */
int nfr_batch_set_config(nfr_batch* batch, int64_t chunk, int wgs_per_cu);
int nfr_batch_get_config(const nfr_batch* batch, int64_t* chunk, int* wgs_per_cu);
/* Autotuner: times one pair-sum launch of every candidate configuration on the
 * given states (which are read, not modified) and keeps the fastest; its time
 * in ms goes to *best_ms (may be NULL).  Synchronous. */
int nfr_batch_tune(nfr_batch* batch, double* const* u_devs, void* ws_dev, size_t ws_bytes, double* best_ms);
/* RK4 (as nfr_integrate, on-the-fly FP32 pair sums, FP64 states) for every
 * problem of the batch: u_devs[p] points to problem p's B[p] x n_p state
 * (device), advanced in place by `steps` steps of size dt.  use_graph != 0
 * replays each step from a captured HIP graph (needs a non-default stream;
 * then the call returns after the work has run). */
int nfr_batch_integrate(nfr_batch* batch, double* const* u_devs, double dt, int64_t steps, int use_graph,
                        void* ws_dev, size_t ws_bytes);

/* ---------------------------------------------------------------- adjoint */

/* Workspace bytes of nfr_adjoint: the stage inputs of one checkpoint segment
 * (4 x ckpt_every x n FP64) plus the transpose kernel's per-tile partial sums,
 * 4 x npad^2 / 256 FP64 (8.6 GB at n = 262144; it grows quadratically). */
size_t nfr_adjoint_workspace_size(const nfr_problem* prob, int64_t steps, int64_t ckpt_every);

/* Gradients of a scalar loss L(u(T)) through `steps` RK4 steps of a single
 * state (B = 1), by the discrete adjoint of the time stepper.  The forward
 * trajectory is the one nfr_integrate computes with NFR_FORM_ONTHEFLY_FP32
 * from the same inputs; ckpt_dev holds its checkpoints (u at steps 0,
 * ckpt_every, 2 ckpt_every, ...: 1 + steps / ckpt_every arrays of n doubles,
 * as nfr_integrate writes them).  Each segment is recomputed forward from its
 * checkpoint (keeping its RK4 stage inputs), then swept in reverse: every
 * reverse stage applies the transposed operator z_j = sum_i w_ij lambda_i
 * (w is symmetric, so this is the same pair sum with lambda as the source
 * weights) and accumulates the kernel-parameter derivatives in the same pass.
 * The kernel and firing rate are those of the paper's eq. NFODETilde setting
 * described above; the motivation is model inversion / connectivity
 * inference (paper sections 1 and 6).
 *   ubarT_dev: dL/du(T), n doubles (device);  ubar0_dev: receives dL/du(0).
 *   pbar_host: receives dL/d(A_e, s_e, A_i, s_i, theta) (5 doubles, host).
 * firing->theta_dev must be NULL (one threshold).  On a context with a
 * non-default stream the recompute and the reverse sweep of a segment are
 * captured once per segment length and replayed as HIP graphs (the same
 * results).  Synchronous: returns after the gradients are written. */
int nfr_adjoint(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, const double* ckpt_dev,
                int64_t ckpt_every, int64_t steps, double dt, const double* ubarT_dev, double* ubar0_dev,
                double* pbar_host, void* ws_dev, size_t ws_bytes);

/* ---------------------------------------------------------------- autotuner */

/* The multi-state on-the-fly pair sum (B >= 2) has one free launch parameter:
 * how many workgroups the work is cut into (source chunks per target tile).
 * Tuning results live in a process-wide table that every later plan consults
 * (the entry nearest in log n and log B); workspace sizes follow the plan, so
 * query them after tuning.  Tile shapes of the other kernels are fixed at
 * build time; the uneven batch has its own tuner (nfr_batch_tune). */

/* Workspace bytes of nfr_tune (0 if the sizes are unsupported). */
size_t nfr_tune_workspace_size(int64_t n_max, int B_max);

/* Times the candidate workgroup targets (256 ... 4096) of the multi-state pair
 * sum on synthetic problems (spherical Fibonacci nodes, n = n_max/16, n_max/4,
 * n_max, at least 1024; B = 2, 4, 16, 64, 256 up to B_max; Gaussian Mexican
 * hat), installs the fastest per (n, B) in the process-wide table and, if
 * cache_path is non-NULL, writes them there as JSON.  1024 <= n_max <= 4e6,
 * 2 <= B_max.  Synchronous. */
int nfr_tune(nfr_context* ctx, const char* cache_path, int64_t n_max, int B_max, void* ws_dev, size_t ws_bytes);
/* Installs the entries of a cache written by nfr_tune (host only). */
int nfr_tune_load(const char* cache_path);
/* The workgroup target the planner uses for n nodes and B >= 2 states
 * (1024 without tuning); -1 for invalid sizes. */
int64_t nfr_tune_target(int64_t n, int B);
/* Empties the process-wide table (plans return to the built-in target). */
int nfr_tune_clear(void);

/* ---------------------------------------------------------------- quadrature weights */

/* Projection of a flat triangle's plane onto the surface (section 3.3). */
enum nfr_projection {
  NFR_PROJ_PLANES = 0,      /* central projection from the cutting planes' common point */
  NFR_PROJ_ORIGIN = 1,      /* central projection from the origin (star-shaped surfaces) */
  NFR_PROJ_ORTHOGONAL = 2   /* orthogonal projection along each triangle's normal */
};

/* Workspace bytes for nfr_quad_weights (0 if the sizes are unsupported). */
size_t nfr_quad_workspace_size(int64_t n, int64_t ntri, int k);

/* Surface quadrature weights q (paper section 3.3, eqs. integral and
 * functional_stencil) on the GPU, all arithmetic FP64:
 *   - for every triangle E_j (vertices a, b, c = tri_host[3j..3j+2], oriented
 *     so that (b - a) x (c - a) points outward), its stencil is the k nodes
 *     nearest to the centroid (a + b + c) / 3, ranked by the squared distance
 *     (dx dx + dy dy) + dz dz evaluated without fused multiply-add, ties by
 *     node index;
 *   - projection point p_j, by `projection` (enum nfr_projection):
 *     NFR_PROJ_ORIGIN: the origin (star-shaped surfaces: every ray from the
 *     origin meets the surface once);
 *     NFR_PROJ_PLANES: the common point of the three cutting planes through
 *     E_j's edges, the plane of edge e containing that edge with normal
 *     n_j - n_j' (j' the neighbour across it); if that 3 x 3 system has
 *     condition number above 1e8 the triangle uses orthogonal projection
 *     onto its plane instead (a NaN row in proj_dev);
 *     NFR_PROJ_ORTHOGONAL: every triangle projects orthogonally onto its own
 *     plane (p_j at infinity along n_j; a NaN row in proj_dev), with the
 *     Jacobian 1 / |n(x) . n_j|;
 *   - the stencil is pulled back to E_j's plane along rays from p_j, planar
 *     RBF-QF with phi = r^3 and polynomials of degree <= 2 gives one weight
 *     per stencil node (a (k+6) x (k+6) saddle-point solve, LU with partial
 *     pivoting), each weight is multiplied by the Jacobian of the projection
 *     at that node (using the exact unit normals nrm_dev), and q_i adds node
 *     i's weights over all triangles in increasing (triangle, slot) order.
 * xyz_dev, nrm_dev: n x 3 FP64 row-major (device).  tri_host: ntri x 3 int32
 * (host; read during the call).  The triangulation must be closed and
 * consistently oriented for NFR_PROJ_PLANES (NFR_ERR_INVALID_ARG otherwise);
 * any other `projection` value is NFR_ERR_INVALID_ARG.
 * 6 <= k <= 57, k <= n.  Outputs (device, caller-owned): q_dev (n FP64);
 * stencil_dev (ntri x k int32, may be NULL) receives the stencils; proj_dev
 * (ntri x 3 FP64, may be NULL) the projection points.  ws_dev: >=
 * nfr_quad_workspace_size bytes, 256-byte aligned.  Enqueued on the context
 * stream; the host triangle array may be reused when the call returns. */
int nfr_quad_weights(nfr_context* ctx, int64_t n, const double* xyz_dev, const double* nrm_dev, int64_t ntri,
                     const int32_t* tri_host, int projection, int k, double* q_dev, int32_t* stencil_dev,
                     double* proj_dev, void* ws_dev, size_t ws_bytes);

#ifdef __cplusplus
}
#endif

#endif /* NFR_H */
