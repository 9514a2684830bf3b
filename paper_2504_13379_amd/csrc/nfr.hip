// C ABI of the neural-field library: validation, planning and launches.
// The operator and the time stepper are specified in include/nfr.h.
#include "nfr.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "kernels_core.h"
#include "kernels_mfma.h"
#include "kernels_probe.h"
#include "kernels_adjoint.h"
#include "kernels_batch.h"
#include "kernels_quad.h"
#include "kernels_tile.h"

#include <algorithm>

using namespace nfr;

struct nfr_context {
  int device = 0;
  hipStream_t stream = nullptr;
  int cu_count = 0;
  char arch[64] = {0};
  // optional event timing of the pair-sum launches (not inside graph capture)
  bool timing = false;
  bool capturing = false;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
  // nodes and RK4 steps of the graph the last graph-replayed call used (0: none yet)
  int64_t last_graph_nodes = 0;
  int64_t last_graph_steps = 0;
};

// Everything a captured RK4 graph of nfr_integrate depends on: the kernel
// arguments it baked in (pointers, parameters, the launch plan) and its length.
struct StepGraphKey {
  int form, B, kind;
  double dt, A_e, s_e, A_i, s_i, beta, theta;
  const void* theta_dev;
  const void* u;
  const void* w;
  const void* ws;
  int64_t steps_per_graph, otf_chunk, otf_tiles;
  int nsplit, otf_bs, otf_nsb;
};

struct nfr_problem {
  nfr_context* ctx = nullptr;
  ProblemView view;
  void* pack = nullptr;
  // the last RK4 graph nfr_integrate captured for this problem, reused while
  // the key matches (zero-filled before assignment so memcmp sees no padding)
  hipGraphExec_t step_graph = nullptr;
  StepGraphKey step_key;
  int64_t step_graph_nodes = 0;
};

namespace {

thread_local std::string t_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}

#define NFR_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(NFR_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define NFR_HIP_LAUNCH()                                                                    \
  do {                                                                                      \
    hipError_t e_ = hipGetLastError();                                                      \
    if (e_ != hipSuccess) return fail(NFR_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

constexpr int64_t kMaxN = 4000000;   // keeps every grid dimension below 65536 blocks
constexpr int kMaxB = 4096;
// node indices and segment counts fit the tile order's sort keys (kernels_tile.h)
static_assert(kMaxN <= (int64_t(1) << kTileNodeBits) && kMaxN / kTileLeaf < (int64_t(1) << kTileSegBits), "tile keys");

bool is_finite_d(double x) { return std::isfinite(x); }

int check_kernel(const nfr_kernel* k) {
  if (!k) return fail(NFR_ERR_INVALID_ARG, "kernel is NULL");
  if (k->kind != NFR_KERNEL_GAUSS_MH && k->kind != NFR_KERNEL_EXP_MH)
    return fail(NFR_ERR_INVALID_ARG, "unknown kernel kind %d", k->kind);
  if (!is_finite_d(k->A_e) || !is_finite_d(k->s_e) || !is_finite_d(k->A_i) || !is_finite_d(k->s_i))
    return fail(NFR_ERR_NONFINITE, "kernel parameters must be finite");
  if (!(k->s_e > 0.0) || !(k->s_i > 0.0)) return fail(NFR_ERR_INVALID_ARG, "kernel length scales must be > 0");
  return NFR_OK;
}

int check_firing(const nfr_firing* f) {
  if (!f) return fail(NFR_ERR_INVALID_ARG, "firing is NULL");
  if (!is_finite_d(f->beta) || !is_finite_d(f->theta)) return fail(NFR_ERR_NONFINITE, "firing parameters must be finite");
  if (f->beta < 0.0) return fail(NFR_ERR_INVALID_ARG, "beta must be >= 0");
  return NFR_OK;
}

int check_form(int form) {
  if (form < NFR_FORM_AUTO || form > NFR_FORM_ONTHEFLY_FP32_MFMA) return fail(NFR_ERR_INVALID_ARG, "unknown form %d", form);
  if (is_mfma_form(form) && !kMfmaAvailable) return fail(NFR_ERR_INVALID_ARG, "form %d is not available in this build", form);
  return NFR_OK;
}

PairParams pair_params(const nfr_kernel& k, const ProblemView& pv) {
  PairParams p;
  if (k.kind == NFR_KERNEL_GAUSS_MH) {
    p.sig = (float)(std::sqrt(kLog2e) / k.s_e);
    p.rho = (float)((k.s_e / k.s_i) * (k.s_e / k.s_i));
  } else {
    p.sig = (float)(kLog2e / k.s_e);
    p.rho = (float)(k.s_e / k.s_i);
  }
  p.Ae = k.A_e;
  p.Ai = k.A_i;
  p.per = (float)(pv.period * (double)p.sig);
  p.kappa = k.A_e != 0.0 ? (float)(-k.A_i / k.A_e) : 0.0f;
  p.amp = k.A_e;
  return p;
}

// The forward pair sums accumulate w / A_e (PairParams); a kernel without an
// excitatory part is rewritten as its single inhibitory term, -A_i exp(.. s_i ..)
// in the excitatory slot.
nfr_kernel norm_kernel(const nfr_kernel& k) {
  if (k.A_e != 0.0) return k;
  nfr_kernel n = k;
  n.A_e = -k.A_i;
  n.s_e = k.s_i;
  n.A_i = 0.0;
  return n;
}

// pair_params for the kernels that take a sym_pow code: with an integer
// length ratio the coordinates (and the period) are scaled by the inhibitory
// length instead (see sym_pow).
PairParams pair_params_pow(const nfr_kernel& k, const ProblemView& pv);

// Template code of the pair kernels: kernel kind, + 2 for a periodic problem.
int kind_code(const nfr_kernel& k, const ProblemView& pv) { return k.kind + (pv.period > 0.0 ? 2 : 0); }

// m - 1 when the length scales are in the ratio rho = 1/m, m in {2, 3, 4}
// (rho = s_e/s_i, squared for the Gaussian), else 0; the symmetric kernel then
// derives the excitatory exponential from the inhibitory one.
int sym_pow_code(const nfr_kernel& k) {
  double rho = k.s_e / k.s_i;
  if (k.kind == NFR_KERNEL_GAUSS_MH) rho *= rho;
  if (!(rho > 0.0)) return 0;
  const double m = 1.0 / rho;
  const long mi = std::lround(m);
  if (mi >= 2 && mi <= 4 && std::fabs(m - (double)mi) <= 1e-12 * (double)mi) return (int)mi - 1;
  return 0;
}

PairParams pair_params_pow(const nfr_kernel& k, const ProblemView& pv) {
  PairParams pp = pair_params(k, pv);
  if (sym_pow_code(k)) {
    const double sig_i = k.kind == NFR_KERNEL_GAUSS_MH ? std::sqrt(kLog2e) / k.s_i : kLog2e / k.s_i;
    pp.sig = (float)sig_i;
    pp.per = (float)(pv.period * sig_i);
  }
  return pp;
}

// Far blocks of the fused BF16 form (kernels_tile.h) apply to a Gaussian
// kernel with two exponentials on a non-periodic problem whose broad
// exponential is the inhibitory one, with rho <= 3/4 (then the near entries
// e1' / kappa_i + e2' stay within FP32 range) and |kappa| >= 2^-20 (k is
// normalised).  Returns the squared distance beyond which every pair has
// (1 - rho) t > 27 - log2|kappa|, two bits of margin over the 25 at which the
// steep term falls below half an ulp of the broad one; 0 when not eligible.
float far_d2(const nfr_kernel& k, const ProblemView& pv, int form) {
  if (form != NFR_FORM_ONTHEFLY_BF16X3 || kind_code(k, pv) != 0 || sym_pow_code(k) != 0) return 0.0f;
  const PairParams pp = pair_params_pow(k, pv);
  const double kap = std::fabs((double)pp.kappa), rho = pp.rho;
  if (!(kap >= 0x1p-20) || !(rho > 0.0) || !(rho <= 0.75)) return 0.0f;
  const double s2 = (double)pp.sig * pp.sig;
  return (float)((27.0 - std::log2(kap)) / ((1.0 - rho) * s2));
}

// Calls of the fused BF16 form run in the problem's tile order when its far
// blocks apply (states gathered at the start, scattered back at the end).
bool use_tile_order(const nfr_kernel& k_in, const ProblemView& pv, int form) {
  return far_d2(norm_kernel(k_in), pv, form) > 0.0f;
}

KernelF64 kernel64(const nfr_kernel& k, const ProblemView& pv) {
  return KernelF64{k.kind, k.A_e, k.s_e, k.A_i, k.s_i, pv.period};
}

Firing firing_of(const nfr_firing& f) { return Firing{f.beta, f.theta, f.theta_dev}; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ---------------------------------------------------------------- fixed scratch

// Device memory of nfr_apply_noalloc: one file-scope array that every GPU the
// library runs on holds (its own copy) until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is a
// stand-in, not a device address); it uses the address hipGetSymbolAddress
// returns for the device, taken once per device by nfr_context_create.
constexpr size_t kScratchBytes = NFR_APPLY_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // by device ordinal; null until a context is created there

// Takes the scratch array's device address for `device` (once), with that
// device current; the caller's current device is restored.
int scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)device < g_scratch_ptr.size() && g_scratch_ptr[(size_t)device]) return NFR_OK;
  int prev = 0;
  NFR_HIP(hipGetDevice(&prev));
  NFR_HIP(hipSetDevice(device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  NFR_HIP(hipSetDevice(prev));
  if (e != hipSuccess) return fail(NFR_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  if (!p) return fail(NFR_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
  if (g_scratch_ptr.size() <= (size_t)device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  g_scratch_ptr[(size_t)device] = p;
  return NFR_OK;
}

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (size_t)device < g_scratch_ptr.size() ? g_scratch_ptr[(size_t)device] : nullptr;
}

// ---------------------------------------------------------------- plans

constexpr int64_t kTargetWGs = 1024;   // about four workgroups per compute unit
constexpr int64_t kGraphMaxSteps = 64;  // RK4 steps per captured graph of nfr_integrate
constexpr int64_t kBatchGraphMaxSteps = 16;  // RK4 steps per captured graph of nfr_batch_integrate

struct OtfPlan {
  int bs = 1, nsb = 1;
  int64_t tiles = 0, chunk = 0;
  int nsplit = 1;
};

// States per block of the on-the-fly pair sum: one kernel evaluation serves
// every state of a block, so larger blocks cost fewer evaluations per pair
// interaction; targets per thread shrink as blocks grow (registers).
int otf_bs(int B) { return B == 1 ? 1 : (B == 2 ? 2 : (B <= 4 ? 4 : (B <= 8 ? 8 : 16))); }

// Tuned workgroup targets of the multi-state on-the-fly pair sum (its one
// free launch parameter: how many source chunks the work is cut into), keyed
// by padded node count and state count; process-wide, filled by nfr_tune or
// nfr_tune_load.  A plan uses the entry nearest in (log npad, log B).
struct TuneEntry {
  int64_t npad;
  int B;
  int64_t target;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

int64_t otf_target_wgs(int64_t npad, int B) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  int64_t best = kTargetWGs;
  double best_d = 1e300;
  for (const TuneEntry& e : g_tune) {
    const double d = std::fabs(std::log2((double)npad / (double)e.npad)) + std::fabs(std::log2((double)B / (double)e.B));
    if (d < best_d) {
      best_d = d;
      best = e.target;
    }
  }
  return best;
}

OtfPlan plan_otf_target(int64_t npad, int B, int64_t target) {
  OtfPlan p;
  p.bs = otf_bs(B);
  p.nsb = (int)ceil_div(B, p.bs);
  p.tiles = ceil_div(npad, (int64_t)kWG * otf_tpt(p.bs));
  int64_t want = ceil_div(target, p.tiles * p.nsb);
  const int64_t max_split = npad / kWG;
  if (want < 1) want = 1;
  if (want > max_split) want = max_split;
  p.chunk = round_up(ceil_div(npad, want), kWG);
  p.nsplit = (int)ceil_div(npad, p.chunk);
  return p;
}

OtfPlan plan_otf(int64_t npad, int B) { return plan_otf_target(npad, B, B == 1 ? kTargetWGs : otf_target_wgs(npad, B)); }

struct GemvPlan {
  int bs = 1, nsb = 1;
  int64_t rowblocks = 0, chunk = 0;
  int nsplit = 1;
};

GemvPlan plan_gemv(int64_t n, int64_t npad, int B) {
  GemvPlan p;
  p.bs = B == 1 ? 1 : (B == 2 ? 2 : 4);
  p.nsb = (int)ceil_div(B, p.bs);
  p.rowblocks = ceil_div(n, kGemvRows);
  int64_t want = ceil_div(2 * kTargetWGs, p.rowblocks * p.nsb);
  const int64_t max_split = ceil_div(npad, kColStep);
  if (want < 1) want = 1;
  if (want > max_split) want = max_split;
  p.chunk = round_up(ceil_div(npad, want), kColStep);
  p.nsplit = (int)ceil_div(npad, p.chunk);
  return p;
}

// AUTO: FP32-class accuracy with no W matrix.  From 17 states on the FP32
// matrix-core form (32 or 64 states per kernel value; at N = 65536, B = 64
// 5.1 against 12.3 ms per application); below, the vector-unit sum.
int resolve_form(int form, int64_t n, int B) {
  if (form != NFR_FORM_AUTO) return form;
  (void)n;
  return B > 16 ? NFR_FORM_ONTHEFLY_FP32_MFMA : NFR_FORM_ONTHEFLY_FP32;
}

// The forward symmetric kernel uses tiles of 64 nodes up to kSymSmallMaxNpad
// padded nodes (see kSymSmallTPT), of kSymTile above; the adjoint's transpose
// kernel always uses kSymTile.  Measured (sphere, B = 1, pair kernel per
// launch, large / small shape): N = 2000 12.7 / 7.9 us, 4096 12.7 / 11.8,
// 6144 19.1 / 16.6, 8192 25.8 / 25.3, 16384 65.0 / 71.6.
#ifndef NFR_SYM_SMALL_MAX
#define NFR_SYM_SMALL_MAX 6144
#endif
constexpr int64_t kSymSmallMaxNpad = NFR_SYM_SMALL_MAX;
bool sym_small(int64_t npad) { return npad <= kSymSmallMaxNpad; }
int64_t sym_tiles(int64_t npad) { return ceil_div(npad, sym_small(npad) ? 64 * kSymSmallTPT : kSymTile); }
int64_t adj_tiles(int64_t npad) { return ceil_div(npad, kSymTile); }

// Up to this many padded nodes one state's pair sum is the one-sided
// k_otf_small (kSmallRows targets per workgroup, one slot per node) instead of
// the symmetric kernel.  RK4 step on the sphere, one-sided (one launch per
// stage) / symmetric (pair kernel + combine): N = 1000 18.5 / 35.6 us,
// 2000 25.7 / 37.1, 4096 43.4 / 57.4; with 8 targets per workgroup 6144
// 73.3 / 74.9 and 8192 113 / 108.
#ifndef NFR_SMALL_ONESIDED_MAX
#define NFR_SMALL_ONESIDED_MAX 4096
#endif
constexpr int64_t kSmallOneSidedMaxNpad = NFR_SMALL_ONESIDED_MAX;
bool small_onesided(int64_t npad) { return npad <= kSmallOneSidedMaxNpad; }

template <int K>
void launch_sym(const ProblemView& pv, const PairParams& pp, const float* g, double* part, hipStream_t s) {
  static_assert(kPad % kSmallRows == 0, "whole target blocks");
  if (small_onesided(pv.npad)) {
    hipLaunchKernelGGL((k_otf_small<K, false>), dim3((unsigned)(pv.npad / kSmallRows)), dim3(kWG), 0, s, pv.src, g,
                       pv.n, pv.npad, pp, part, Rk4Stage{}, nullptr);
    return;
  }
  const dim3 grid((unsigned)sym_pairs(sym_tiles(pv.npad)));
  if (sym_small(pv.npad))
    hipLaunchKernelGGL((k_otf_sym<K, kSymSmallTPT, kSymSmallSplit>), grid, dim3(64 * kSymSmallSplit), 0, s, pv.src, g,
                       pv.npad, pp, part);
  else
    hipLaunchKernelGGL((k_otf_sym<K, kSymTPT, kSymSplit>), grid, dim3(kSymThreads), 0, s, pv.src, g, pv.npad, pp, part);
}

// B = 1 on the fly uses the symmetric kernel: one FP64 slot per tile and node,
// npad^2 / kSymTile * 8 bytes, which grows quadratically; beyond 8 GiB of
// slots (N above about 520k) the one-sided kernel, whose partial sums stay
// small, is used instead.
constexpr double kSymMaxSlotBytes = 8.0 * 1024 * 1024 * 1024;
bool use_sym(int form, int B, int64_t npad) {
  return form == NFR_FORM_ONTHEFLY_FP32 && B == 1 && (double)sym_tiles(npad) * (double)npad * 8.0 <= kSymMaxSlotBytes;
}

// Forms whose FP32 source array g holds q f(u) (the on-the-fly FP32 forms);
// the W forms hold f(u) (q sits in W).
bool sources_carry_q(int form) { return form == NFR_FORM_ONTHEFLY_FP32 || form == NFR_FORM_ONTHEFLY_FP32_MFMA; }

// Partial-sum slots per node of one pair launch; `otf` is the plan of the
// multi-state on-the-fly FP32 sum (the only plan that reads the tune table).
int nsplit_of(const ProblemView& pv, int B, int form, const OtfPlan& otf) {
  if (use_sym(form, B, pv.npad)) return small_onesided(pv.npad) ? 1 : (int)sym_tiles(pv.npad);
  if (form == NFR_FORM_ONTHEFLY_FP32) return otf.nsplit;
  if (form == NFR_FORM_W_FP32) return plan_gemv(pv.n, pv.npad, B).nsplit;
  return mfma_nsplit(form);
}

// A carved workspace also fixes the launch plan of the call that carved it:
// the tune table is read once, in carve(), and every pair launch and combine
// of that call uses `otf` and `nsplit` from here, so a concurrent nfr_tune*
// on another thread cannot change the slot count between the launch that
// writes the partial sums and the combine that adds them.
struct Workspace {
  float* g = nullptr;
  float* g2 = nullptr;         // second source buffer of the one-launch small stage (null: two launches)
  double* part = nullptr;
  double* v = nullptr;
  double* ksum = nullptr;
  double* ut = nullptr;        // fused BF16 form: states in the tile order (n x B)
  double* yt = nullptr;        // fused BF16 form, one application: the result in the tile order
  OtfPlan otf;                 // multi-state on-the-fly FP32 plan (unused by other forms)
  int nsplit = 1;              // partial-sum slots per node and state in `part`
  size_t bytes = 0;
};

// Small single-state problems on the one-sided path step each RK4 stage in
// one launch (k_otf_small with STAGE), alternating the sources between g and
// g2: stages 1 and 3 read g and write g2, stages 2 and 4 the reverse, so
// every step starts and ends with the sources in g.
bool use_small_stage(const ProblemView& pv, int form, int B) {
  return use_sym(form, B, pv.npad) && small_onesided(pv.npad);
}

Workspace carve(void* base, const ProblemView& pv, int B, int form, bool stepping) {
  Workspace w;
  char* p = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* r = p ? p + off : nullptr;
    off += align256(bytes);
    return r;
  };
  if (form == NFR_FORM_ONTHEFLY_FP32 && !use_sym(form, B, pv.npad)) w.otf = plan_otf(pv.npad, B);
  w.nsplit = nsplit_of(pv, B, form, w.otf);
  const size_t gbytes = is_mfma_form(form) ? mfma_g_bytes(pv.npad, B) : size_t(pv.npad) * B * sizeof(float);
  w.g = reinterpret_cast<float*>(take(gbytes));
  // the fused split forms keep FP32 partial sums, every other form FP64
  const size_t part_elem = (form == NFR_FORM_ONTHEFLY_BF16X3 || form == NFR_FORM_ONTHEFLY_FP16X3) ? sizeof(float)
                                                                                                  : sizeof(double);
  w.part = reinterpret_cast<double*>(take(size_t(w.nsplit) * B * pv.npad * part_elem));
  if (stepping) {
    w.v = reinterpret_cast<double*>(take(size_t(pv.n) * B * sizeof(double)));
    w.ksum = reinterpret_cast<double*>(take(size_t(pv.n) * B * sizeof(double)));
    if (use_small_stage(pv, form, B)) w.g2 = reinterpret_cast<float*>(take(gbytes));
  }
  if (form == NFR_FORM_ONTHEFLY_BF16X3) {
    w.ut = reinterpret_cast<double*>(take(size_t(pv.n) * B * sizeof(double)));
    if (!stepping) w.yt = reinterpret_cast<double*>(take(size_t(pv.n) * B * sizeof(double)));
  }
  w.bytes = off;
  return w;
}

// ---------------------------------------------------------------- launches

template <int KIND>
void launch_otf_kind(const ProblemView& pv, const PairParams& pp, int B, const float* g, double* part,
                     const OtfPlan& pl, hipStream_t s) {
  dim3 grid((unsigned)pl.tiles, (unsigned)pl.nsplit, (unsigned)pl.nsb);
  if (pl.bs == 1)
    hipLaunchKernelGGL((k_otf_pair_sum<KIND, otf_tpt(1), 1>), grid, dim3(kWG), 0, s, pv.src, g, pv.npad, B, pl.chunk, pp, part);
  else if (pl.bs == 2)
    hipLaunchKernelGGL((k_otf_pair_sum<KIND, otf_tpt(2), 2>), grid, dim3(kWG), 0, s, pv.src, g, pv.npad, B, pl.chunk, pp, part);
  else if (pl.bs == 4)
    hipLaunchKernelGGL((k_otf_pair_sum<KIND, otf_tpt(4), 4>), grid, dim3(kWG), 0, s, pv.src, g, pv.npad, B, pl.chunk, pp, part);
  else if (pl.bs == 8)
    hipLaunchKernelGGL((k_otf_pair_sum<KIND, otf_tpt(8), 8>), grid, dim3(kWG), 0, s, pv.src, g, pv.npad, B, pl.chunk, pp, part);
  else
    hipLaunchKernelGGL((k_otf_pair_sum<KIND, otf_tpt(16), 16>), grid, dim3(kWG), 0, s, pv.src, g, pv.npad, B, pl.chunk, pp, part);
}

void launch_gemv(const ProblemView& pv, const float* W, int B, const float* G, double* part, const GemvPlan& pl,
                 hipStream_t s) {
  dim3 grid((unsigned)pl.rowblocks, (unsigned)pl.nsplit, (unsigned)pl.nsb);
  if (pl.bs == 1)
    hipLaunchKernelGGL((k_w_gemv_f32<1>), grid, dim3(kWG), 0, s, W, G, pv.n, pv.npad, B, pl.chunk, part);
  else if (pl.bs == 2)
    hipLaunchKernelGGL((k_w_gemv_f32<2>), grid, dim3(kWG), 0, s, W, G, pv.n, pv.npad, B, pl.chunk, part);
  else
    hipLaunchKernelGGL((k_w_gemv_f32<4>), grid, dim3(kWG), 0, s, W, G, pv.n, pv.npad, B, pl.chunk, part);
}

// Source preparation for a given form; `v_copy` may be null.
int launch_prep(const ProblemView& pv, int form, int B, const double* u, const Firing& fr, const Workspace& w,
                double* v_copy, hipStream_t s) {
  if (is_mfma_form(form)) {
    launch_mfma_prep(pv, form, B, u, fr, w.g, v_copy, s);
  } else {
    const int with_q = sources_carry_q(form) ? 1 : 0;
    const int64_t total = pv.npad * (int64_t)B;
    hipLaunchKernelGGL(k_source_prep, dim3((unsigned)ceil_div(total, kWG)), dim3(kWG), 0, s, u, pv.n, pv.npad, B,
                       pv.q, with_q, fr, w.g, v_copy);
  }
  NFR_HIP_LAUNCH();
  return NFR_OK;
}

// States between the problem's node order and its tile order.
void launch_tile_gather(const ProblemView& pv, int B, const double* u, double* ut, hipStream_t s) {
  const int64_t total = pv.n * (int64_t)B;
  hipLaunchKernelGGL(k_tile_gather, dim3((unsigned)ceil_div(total, kWG)), dim3(kWG), 0, s, u, pv.perm, pv.n, total, ut);
}
void launch_tile_scatter(const ProblemView& pv, int B, const double* ut, double* u, hipStream_t s) {
  const int64_t total = pv.n * (int64_t)B;
  hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)ceil_div(total, kWG)), dim3(kWG), 0, s, ut, pv.perm, pv.n, total, u);
}

// Pair sums into w.part for the current w.g.
int timing_mark(nfr_context* ctx) {
  if (!ctx->timing || ctx->capturing) return NFR_OK;
  if (ctx->events_used == ctx->events.size()) {
    hipEvent_t e;
    NFR_HIP(hipEventCreate(&e));
    ctx->events.push_back(e);
  }
  NFR_HIP(hipEventRecord(ctx->events[ctx->events_used++], ctx->stream));
  return NFR_OK;
}

int launch_pairs_raw(const ProblemView& pv, const nfr_kernel& k_in, int form, int B, const void* W, const Workspace& w,
                     hipStream_t s) {
  const nfr_kernel k = norm_kernel(k_in);
  if (use_sym(form, B, pv.npad)) {
    const PairParams pp = pair_params_pow(k, pv);
#define NFR_SYM_CASE(K) \
  case K: launch_sym<K>(pv, pp, w.g, w.part, s); break;
    switch (kind_code(k, pv) | (sym_pow_code(k) << 2)) {
      NFR_SYM_CASE(0) NFR_SYM_CASE(1) NFR_SYM_CASE(2) NFR_SYM_CASE(3)
      NFR_SYM_CASE(4) NFR_SYM_CASE(5) NFR_SYM_CASE(6) NFR_SYM_CASE(7)
      NFR_SYM_CASE(8) NFR_SYM_CASE(9) NFR_SYM_CASE(10) NFR_SYM_CASE(11)
      NFR_SYM_CASE(12) NFR_SYM_CASE(13) NFR_SYM_CASE(14) NFR_SYM_CASE(15)
      default: return fail(NFR_ERR_INTERNAL, "no symmetric kernel for this kernel code");
    }
#undef NFR_SYM_CASE
  } else if (form == NFR_FORM_ONTHEFLY_FP32) {
    const OtfPlan& pl = w.otf;
    const PairParams pp = pair_params(k, pv);
    switch (kind_code(k, pv)) {
      case 0: launch_otf_kind<0>(pv, pp, B, w.g, w.part, pl, s); break;
      case 1: launch_otf_kind<1>(pv, pp, B, w.g, w.part, pl, s); break;
      case 2: launch_otf_kind<2>(pv, pp, B, w.g, w.part, pl, s); break;
      default: launch_otf_kind<3>(pv, pp, B, w.g, w.part, pl, s); break;
    }
  } else if (form == NFR_FORM_W_FP32) {
    launch_gemv(pv, static_cast<const float*>(W), B, w.g, w.part, plan_gemv(pv.n, pv.npad, B), s);
  } else if (form == NFR_FORM_ONTHEFLY_FP32_MFMA) {
    const PairParams pp = pair_params_pow(k, pv);
#define NFR_F32M_CASE(K) \
  case K: launch_mfma_otf_f32<K>(pv, pp, B, w.g, w.part, s); break;
    switch (kind_code(k, pv) | (sym_pow_code(k) << 2)) {
      NFR_F32M_CASE(0) NFR_F32M_CASE(1) NFR_F32M_CASE(2) NFR_F32M_CASE(3)
      NFR_F32M_CASE(4) NFR_F32M_CASE(5) NFR_F32M_CASE(6) NFR_F32M_CASE(7)
      NFR_F32M_CASE(8) NFR_F32M_CASE(9) NFR_F32M_CASE(10) NFR_F32M_CASE(11)
      NFR_F32M_CASE(12) NFR_F32M_CASE(13) NFR_F32M_CASE(14) NFR_F32M_CASE(15)
      default: return fail(NFR_ERR_INTERNAL, "no FP32 matrix-core kernel for this kernel code");
    }
#undef NFR_F32M_CASE
  } else if (!mfma_has_w(form)) {
    const PairParams pp = pair_params_pow(k, pv);
    const float d2 = pv.tiled ? far_d2(k, pv, form) : 0.0f;
    const MfmaOtfParams op{pp.sig, pp.rho, pp.per, pp.kappa, pp.amp, pv.qmax,
                           d2 > 0.0f ? pv.bnd32 : nullptr, d2 > 0.0f ? pv.bnd16 : nullptr, d2};
#define NFR_MFMA_OTF_CASE(K) \
  case K: launch_mfma_otf<K>(pv, form, op, B, w.g, w.part, s); break;
    switch (kind_code(k, pv) | (sym_pow_code(k) << 2)) {
      NFR_MFMA_OTF_CASE(0) NFR_MFMA_OTF_CASE(1) NFR_MFMA_OTF_CASE(2) NFR_MFMA_OTF_CASE(3)
      NFR_MFMA_OTF_CASE(4) NFR_MFMA_OTF_CASE(5) NFR_MFMA_OTF_CASE(6) NFR_MFMA_OTF_CASE(7)
      NFR_MFMA_OTF_CASE(8) NFR_MFMA_OTF_CASE(9) NFR_MFMA_OTF_CASE(10) NFR_MFMA_OTF_CASE(11)
      NFR_MFMA_OTF_CASE(12) NFR_MFMA_OTF_CASE(13) NFR_MFMA_OTF_CASE(14) NFR_MFMA_OTF_CASE(15)
      default: return fail(NFR_ERR_INTERNAL, "no fused kernel for this kernel code");
    }
#undef NFR_MFMA_OTF_CASE
  } else {
    launch_mfma_apply(pv, form, B, W, w.g, w.part, s);
  }
  NFR_HIP_LAUNCH();
  return NFR_OK;
}

// The pair-sum launch of one operator application, bracketed by timing events when enabled.
int launch_pairs(nfr_context* ctx, const ProblemView& pv, const nfr_kernel& k, int form, int B, const void* W,
                 const Workspace& w) {
  int st;
  if ((st = timing_mark(ctx))) return st;
  if ((st = launch_pairs_raw(pv, k, form, B, W, w, ctx->stream))) return st;
  return timing_mark(ctx);
}

// Lanes per element for adding nsplit partial-sum slots (see slot_sum).
int slot_lanes(int nsplit) { return nsplit <= 4 ? 1 : (nsplit <= 16 ? 4 : (nsplit <= 64 ? 8 : 16)); }

// Launches KERNEL<L> with L = slot_lanes(nsplit) and n*B*L threads.
#define NFR_LAUNCH_SLOTS(KERNEL, nsplit, total, s, ...)                                                      \
  do {                                                                                                      \
    const int L_ = slot_lanes(nsplit);                                                                      \
    const dim3 g_((unsigned)ceil_div((total) * L_, kWG));                                                   \
    if (L_ == 1) hipLaunchKernelGGL(KERNEL<1>, g_, dim3(kWG), 0, s, __VA_ARGS__);                           \
    else if (L_ == 4) hipLaunchKernelGGL(KERNEL<4>, g_, dim3(kWG), 0, s, __VA_ARGS__);                      \
    else if (L_ == 8) hipLaunchKernelGGL(KERNEL<8>, g_, dim3(kWG), 0, s, __VA_ARGS__);                      \
    else hipLaunchKernelGGL(KERNEL<16>, g_, dim3(kWG), 0, s, __VA_ARGS__);                                  \
  } while (0)

int launch_combine(const ProblemView& pv, int form, int B, int stage, double dt, double* u, const Workspace& w,
                   const Firing& fr, hipStream_t s, double* k1_out = nullptr, const double* gamma = nullptr) {
  const int nsplit = w.nsplit;
  const int64_t total = pv.n * (int64_t)B;
  if (is_mfma_form(form)) {
    launch_mfma_combine(pv, form, B, stage, dt, u, w.v, w.ksum, w.part, nsplit, fr, w.g, k1_out, gamma, s);
  } else {
    const Rk4Stage st{stage, dt, u, w.v, w.ksum, pv.q, sources_carry_q(form) ? 1 : 0, fr, k1_out, gamma};
    NFR_LAUNCH_SLOTS(k_rk4_combine, nsplit, total, s, w.part, nsplit, pv.n, pv.npad, B, st, w.g);
  }
  NFR_HIP_LAUNCH();
  return NFR_OK;
}

// One RK4 stage: pair sums of the current sources, then the stage combination
// (one launch for small single-state problems, see use_small_stage, else two).
int launch_stage(nfr_context* ctx, const ProblemView& pv, const nfr_kernel& k_in, int form, int B, const void* W,
                 const Workspace& w, int stage, double dt, double* u, const Firing& fr, double* k1_out = nullptr,
                 const double* gamma = nullptr) {
  int st;
  if (!w.g2) {
    if ((st = launch_pairs(ctx, pv, k_in, form, B, W, w))) return st;
    return launch_combine(pv, form, B, stage, dt, u, w, fr, ctx->stream, k1_out, gamma);
  }
  const nfr_kernel k = norm_kernel(k_in);
  const PairParams pp = pair_params_pow(k, pv);
  const Rk4Stage rs{stage, dt, u, w.v, w.ksum, pv.q, sources_carry_q(form) ? 1 : 0, fr, k1_out, gamma};
  const float* g_in = (stage & 1) ? w.g : w.g2;
  float* g_out = (stage & 1) ? w.g2 : w.g;
  const dim3 grid((unsigned)(pv.npad / kSmallRows));
  hipStream_t s = ctx->stream;
  if ((st = timing_mark(ctx))) return st;
#define NFR_STAGE_CASE(K) \
  case K: hipLaunchKernelGGL((k_otf_small<K, true>), grid, dim3(kWG), 0, s, pv.src, g_in, pv.n, pv.npad, pp, w.part, rs, g_out); break;
  switch (kind_code(k, pv) | (sym_pow_code(k) << 2)) {
    NFR_STAGE_CASE(0) NFR_STAGE_CASE(1) NFR_STAGE_CASE(2) NFR_STAGE_CASE(3)
    NFR_STAGE_CASE(4) NFR_STAGE_CASE(5) NFR_STAGE_CASE(6) NFR_STAGE_CASE(7)
    NFR_STAGE_CASE(8) NFR_STAGE_CASE(9) NFR_STAGE_CASE(10) NFR_STAGE_CASE(11)
    NFR_STAGE_CASE(12) NFR_STAGE_CASE(13) NFR_STAGE_CASE(14) NFR_STAGE_CASE(15)
    default: return fail(NFR_ERR_INTERNAL, "no small stage kernel for this kernel code");
  }
#undef NFR_STAGE_CASE
  NFR_HIP_LAUNCH();
  return timing_mark(ctx);
}

// One Adams-Bashforth 5 step from the partial sums of K(u_n); n_step >= 4.
int launch_ab5(const ProblemView& pv, int form, int B, int64_t n_step, double dt, double* u, double* hist,
               const Workspace& w, const Firing& fr, hipStream_t s) {
  const Ab5Weights wt{{1901.0 / 720.0, -2774.0 / 720.0, 2616.0 / 720.0, -1274.0 / 720.0, 251.0 / 720.0}};
  auto slot = [&](int64_t m) { return (int)(m % 5); };
  const int4 s03 = make_int4(slot(n_step), slot(n_step - 1), slot(n_step - 2), slot(n_step - 3));
  const int s4 = slot(n_step - 4);
  const int nsplit = w.nsplit;
  const int64_t total = pv.n * (int64_t)B;
  if (is_mfma_form(form)) {
    launch_mfma_ab5(pv, form, B, dt, wt, s03, s4, u, hist, w.part, nsplit, fr, w.g, s);
  } else {
    const int with_q = sources_carry_q(form) ? 1 : 0;
    NFR_LAUNCH_SLOTS(k_ab5_combine, nsplit, total, s, w.part, nsplit, pv.n, pv.npad, B, dt, wt, s03, s4, u, hist,
                     pv.q, with_q, fr, w.g);
  }
  NFR_HIP_LAUNCH();
  return NFR_OK;
}

int check_problem(const nfr_problem* p) {
  if (!p || !p->ctx) return fail(NFR_ERR_INVALID_ARG, "problem is NULL");
  return NFR_OK;
}

int check_w(const nfr_problem* p, int form, const void* w_dev) {
  if (form == NFR_FORM_ONTHEFLY_FP32 || form == NFR_FORM_ONTHEFLY_FP32_MFMA || (is_mfma_form(form) && !mfma_has_w(form)))
    return NFR_OK;
  if (!w_dev) return fail(NFR_ERR_INVALID_ARG, "form %d needs a W matrix (w_dev is NULL)", form);
  (void)p;
  return NFR_OK;
}

}  // namespace

// ================================================================ C ABI

namespace {
// Regions of a problem's pack buffer, in order: packed coordinates, weights,
// FP64 coordinates, the two maxima, then the tile order (kernels_tile.h):
// slot -> node, coordinates and weights in slot order, block bounds, the
// bounding box and the sort keys (used while the problem is created).
struct PackLayout {
  size_t src, q, xyz, qmax, perm, src_t, q_t, bnd32, bnd16, box, keys, bytes;
};
PackLayout pack_layout(int64_t n) {
  const int64_t npad = round_up(n, kPad);
  PackLayout L;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t r = off;
    off += align256(b);
    return r;
  };
  L.src = take(npad * sizeof(float4));
  L.q = take(npad * sizeof(double));
  L.xyz = take(3 * npad * sizeof(double));
  L.qmax = take(2 * sizeof(double));
  L.perm = take(npad * sizeof(int));
  L.src_t = take(npad * sizeof(float4));
  L.q_t = take(npad * sizeof(double));
  L.bnd32 = take(npad / kTileRowBlock * sizeof(float4));
  L.bnd16 = take(npad / kTileColBlock * sizeof(float4));
  L.box = take(size_t(6) * (size_t(1) << tile_levels(n)) * sizeof(double));   // one box per segment
  L.keys = take(tile_pow2(npad) * sizeof(uint64_t));
  L.bytes = off;
  return L;
}
}  // namespace

extern "C" {

int nfr_version(int* major, int* minor, int* patch) {
  if (!major || !minor || !patch) return fail(NFR_ERR_INVALID_ARG, "NULL output pointer");
  *major = NFR_VERSION_MAJOR;
  *minor = NFR_VERSION_MINOR;
  *patch = NFR_VERSION_PATCH;
  return NFR_OK;
}

const char* nfr_status_string(int status) {
  switch (status) {
    case NFR_OK: return "NFR_OK";
    case NFR_ERR_INVALID_ARG: return "NFR_ERR_INVALID_ARG";
    case NFR_ERR_NONFINITE: return "NFR_ERR_NONFINITE";
    case NFR_ERR_NO_DEVICE: return "NFR_ERR_NO_DEVICE";
    case NFR_ERR_UNSUPPORTED_ARCH: return "NFR_ERR_UNSUPPORTED_ARCH";
    case NFR_ERR_HIP: return "NFR_ERR_HIP";
    case NFR_ERR_WORKSPACE: return "NFR_ERR_WORKSPACE";
    case NFR_ERR_INTERNAL: return "NFR_ERR_INTERNAL";
    default: return "NFR_ERR_UNKNOWN";
  }
}

const char* nfr_last_error(void) { return t_err.c_str(); }

int nfr_context_create(int device, void* hip_stream, nfr_context** out) {
  if (!out) return fail(NFR_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(NFR_ERR_NO_DEVICE, "no HIP device");
  if (device < 0 || device >= count) return fail(NFR_ERR_NO_DEVICE, "device %d out of range (count %d)", device, count);
  hipDeviceProp_t prop;
  NFR_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(NFR_ERR_UNSUPPORTED_ARCH, "device %d is %s, this library is built for gfx950", device, prop.gcnArchName);
  int st;
  if ((st = scratch_init(device))) return st;
  nfr_context* c = new (std::nothrow) nfr_context;
  if (!c) return fail(NFR_ERR_INTERNAL, "out of host memory");
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->cu_count = prop.multiProcessorCount;
  std::snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
  *out = c;
  return NFR_OK;
}

int nfr_context_destroy(nfr_context* ctx) {
  if (ctx)
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  delete ctx;
  return NFR_OK;
}

int nfr_context_set_timing(nfr_context* ctx, int enable) {
  if (!ctx) return fail(NFR_ERR_INVALID_ARG, "context is NULL");
  ctx->timing = enable != 0;
  ctx->events_used = 0;
  return NFR_OK;
}

int nfr_context_last_graph(const nfr_context* ctx, int64_t* nodes, int64_t* steps) {
  if (!ctx || !nodes || !steps) return fail(NFR_ERR_INVALID_ARG, "NULL argument");
  *nodes = ctx->last_graph_nodes;
  *steps = ctx->last_graph_steps;
  return NFR_OK;
}

int nfr_context_timing(nfr_context* ctx, int64_t* launches, double* total_ms) {
  if (!ctx || !launches || !total_ms) return fail(NFR_ERR_INVALID_ARG, "NULL argument");
  NFR_HIP(hipSetDevice(ctx->device));
  NFR_HIP(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  for (size_t i = 0; i + 1 < ctx->events_used; i += 2) {
    float ms = 0.0f;
    NFR_HIP(hipEventElapsedTime(&ms, ctx->events[i], ctx->events[i + 1]));
    tot += ms;
  }
  *launches = (int64_t)(ctx->events_used / 2);
  *total_ms = tot;
  ctx->events_used = 0;
  return NFR_OK;
}

int nfr_probe(nfr_context* ctx, int which, int64_t size, void* buf_dev, size_t buf_bytes, double* rate) {
  if (!ctx || !buf_dev || !rate) return fail(NFR_ERR_INVALID_ARG, "NULL argument");
  if (which < NFR_PROBE_FMA || which > NFR_PROBE_MFMA_BF16_MASK) return fail(NFR_ERR_INVALID_ARG, "unknown probe %d", which);
  if (size < 1) return fail(NFR_ERR_INVALID_ARG, "size must be >= 1");
  const int64_t grid = (int64_t)ctx->cu_count * 8;
  const size_t out_bytes = size_t(grid) * kWG * sizeof(float);
  const bool memprobe = which == NFR_PROBE_HBM_READ || which == NFR_PROBE_HBM_COPY;
  if (memprobe && size % 4) return fail(NFR_ERR_INVALID_ARG, "size must be a multiple of 4 floats");
  const size_t need = memprobe ? (which == NFR_PROBE_HBM_READ ? size_t(size) * 4 + out_bytes : size_t(size) * 8)
                               : out_bytes;
  if (buf_bytes < need) return fail(NFR_ERR_WORKSPACE, "probe buffer has %zu bytes, needs %zu", buf_bytes, need);
  NFR_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  hipEvent_t e0, e1;
  NFR_HIP(hipEventCreate(&e0));
  NFR_HIP(hipEventCreate(&e1));
  float* f = static_cast<float*>(buf_dev);
  NFR_HIP(hipEventRecord(e0, s));
  const dim3 g((unsigned)grid), b(kWG);
  switch (which) {
    case NFR_PROBE_FMA: hipLaunchKernelGGL(k_probe_fma, g, b, 0, s, size, f); break;
    case NFR_PROBE_EXP: hipLaunchKernelGGL(k_probe_exp, g, b, 0, s, size, f); break;
    case NFR_PROBE_SQRT: hipLaunchKernelGGL(k_probe_sqrt, g, b, 0, s, size, f); break;
    case NFR_PROBE_HBM_READ: hipLaunchKernelGGL(k_probe_read, g, b, 0, s, f, size, f + size); break;
    case NFR_PROBE_HBM_COPY: hipLaunchKernelGGL(k_probe_copy, g, b, 0, s, f, f + size, size); break;
    case NFR_PROBE_FMA_VOP3: hipLaunchKernelGGL(k_probe_fma_vop3, g, b, 0, s, size, f); break;
    case NFR_PROBE_FMA_EXP: hipLaunchKernelGGL(k_probe_fma_exp, g, b, 0, s, size, f); break;
    case NFR_PROBE_MFMA_F32: hipLaunchKernelGGL(k_probe_mfma_f32, g, b, 0, s, size, f); break;
    case NFR_PROBE_MFMA_F32_FMA: hipLaunchKernelGGL(k_probe_mfma_f32_fma, g, b, 0, s, size, f); break;
    case NFR_PROBE_MFMA_BF16_FMA: hipLaunchKernelGGL(k_probe_mfma_bf16_fma, g, b, 0, s, size, f); break;
    case NFR_PROBE_MFMA_BF16_DOT2: hipLaunchKernelGGL(k_probe_mfma_bf16_vop<0>, g, b, 0, s, size, f); break;
    case NFR_PROBE_MFMA_BF16_MASK: hipLaunchKernelGGL(k_probe_mfma_bf16_vop<1>, g, b, 0, s, size, f); break;
    default: hipLaunchKernelGGL(k_probe_mfma, g, b, 0, s, size, f); break;
  }
  hipError_t le = hipGetLastError();
  NFR_HIP(hipEventRecord(e1, s));
  NFR_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  NFR_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (le != hipSuccess) return fail(NFR_ERR_HIP, "probe launch failed: %s", hipGetErrorString(le));
  const double sec = ms * 1e-3;
  const double lanes = double(grid) * kWG;
  switch (which) {
    case NFR_PROBE_FMA:
    case NFR_PROBE_EXP:
    case NFR_PROBE_SQRT:
    case NFR_PROBE_FMA_VOP3: *rate = lanes * kProbeChains * double(size) / sec; break;
    case NFR_PROBE_FMA_EXP: *rate = lanes * kProbeChains * 4.0 * double(size) / sec; break;
    case NFR_PROBE_HBM_READ: *rate = double(size) * 4 / sec; break;
    case NFR_PROBE_HBM_COPY: *rate = double(size) * 8 / sec; break;
    case NFR_PROBE_MFMA_F32: *rate = double(grid) * (kWG / 64) * 4 * double(size) * (32.0 * 32 * 2 * 2) / sec; break;
    case NFR_PROBE_MFMA_F32_FMA: *rate = double(grid) * (kWG / 64) * 2 * double(size) * (32.0 * 32 * 2 * 2) / sec; break;
    case NFR_PROBE_MFMA_BF16_FMA:
    case NFR_PROBE_MFMA_BF16_DOT2:
    case NFR_PROBE_MFMA_BF16_MASK:
      *rate = double(grid) * (kWG / 64) * 4 * double(size) * (32.0 * 32 * 16 * 2) / sec;
      break;
    default: *rate = double(grid) * (kWG / 64) * 4 * double(size) * (32.0 * 32 * 16 * 2) / sec; break;
  }
  return NFR_OK;
}

const char* nfr_context_arch(const nfr_context* ctx) { return ctx ? ctx->arch : ""; }


size_t nfr_problem_bytes(int64_t n) {
  if (n < 1 || n > kMaxN) return 0;
  return pack_layout(n).bytes;
}

int nfr_problem_create_periodic(nfr_context* ctx, int64_t n, const double* xyz_dev, const double* q_dev,
                                double period, void* pack_dev, size_t pack_bytes, nfr_problem** out) {
  if (!out) return fail(NFR_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!is_finite_d(period)) return fail(NFR_ERR_NONFINITE, "period must be finite");
  if (period < 0.0) return fail(NFR_ERR_INVALID_ARG, "period must be >= 0 (0: no periodicity)");
  if (!ctx) return fail(NFR_ERR_INVALID_ARG, "context is NULL");
  if (n < 1 || n > kMaxN) return fail(NFR_ERR_INVALID_ARG, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxN);
  if (!xyz_dev || !q_dev || !pack_dev) return fail(NFR_ERR_INVALID_ARG, "NULL device pointer");
  if (reinterpret_cast<uintptr_t>(pack_dev) % 256) return fail(NFR_ERR_INVALID_ARG, "pack buffer must be 256-byte aligned");
  const size_t need = nfr_problem_bytes(n);
  if (pack_bytes < need) return fail(NFR_ERR_WORKSPACE, "pack buffer has %zu bytes, needs %zu", pack_bytes, need);
  NFR_HIP(hipSetDevice(ctx->device));
  nfr_problem* p = new (std::nothrow) nfr_problem;
  if (!p) return fail(NFR_ERR_INTERNAL, "out of host memory");
  const int64_t npad = round_up(n, kPad);
  char* base = static_cast<char*>(pack_dev);
  p->ctx = ctx;
  p->pack = pack_dev;
  p->view.n = n;
  p->view.npad = npad;
  p->view.period = period;
  const PackLayout L = pack_layout(n);
  float4* src = reinterpret_cast<float4*>(base + L.src);
  double* q = reinterpret_cast<double*>(base + L.q);
  double* xyz = reinterpret_cast<double*>(base + L.xyz);
  double* qmax = reinterpret_cast<double*>(base + L.qmax);
  int* perm = reinterpret_cast<int*>(base + L.perm);
  float4* src_t = reinterpret_cast<float4*>(base + L.src_t);
  double* q_t = reinterpret_cast<double*>(base + L.q_t);
  float4* bnd32 = reinterpret_cast<float4*>(base + L.bnd32);
  float4* bnd16 = reinterpret_cast<float4*>(base + L.bnd16);
  double* box = reinterpret_cast<double*>(base + L.box);
  uint64_t* keys = reinterpret_cast<uint64_t*>(base + L.keys);
  p->view.src = src;
  p->view.q = q;
  p->view.xyz = xyz;
  p->view.qmax = qmax;
  p->view.perm = perm;
  p->view.src_t = src_t;
  p->view.q_t = q_t;
  p->view.bnd32 = bnd32;
  p->view.bnd16 = bnd16;
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)ceil_div(npad, kWG)), dim3(kWG), 0, st, xyz_dev, q_dev, n, npad, period, src, q,
                     xyz);
  hipLaunchKernelGGL(k_qmax, dim3(1), dim3(kWG), 0, st, q, src, npad, qmax);
  // tile order (kernels_tile.h): recursive bisection, each level a bitonic sort
  // of (segment, coordinate along the segment's longest axis, node) keys;
  // then the slot arrays and block bounds
  const int64_t np2 = tile_pow2(npad);
  const dim3 gk((unsigned)ceil_div(np2, kWG));
  hipLaunchKernelGGL(k_tile_init, dim3((unsigned)ceil_div(n, kWG)), dim3(kWG), 0, st, n, perm);
  const int levels = tile_levels(n);
  for (int l = 0; l < levels; ++l) {
    hipLaunchKernelGGL(k_tile_seg_box, dim3((unsigned)(int64_t(1) << l)), dim3(kWG), 0, st, src, perm, n, l, box);
    hipLaunchKernelGGL(k_tile_seg_keys, gk, dim3(kWG), 0, st, src, perm, n, np2, l, box, keys);
    for (int64_t k = 2; k <= np2; k <<= 1)
      for (int64_t j = k >> 1; j > 0; j >>= 1) hipLaunchKernelGGL(k_bitonic, gk, dim3(kWG), 0, st, keys, np2, k, j);
    hipLaunchKernelGGL(k_tile_take, dim3((unsigned)ceil_div(n, kWG)), dim3(kWG), 0, st, keys, n, perm);
  }
  hipLaunchKernelGGL(k_tile_build, dim3((unsigned)ceil_div(npad, kWG)), dim3(kWG), 0, st, n, npad, src, q, perm, src_t,
                     q_t);
  const int64_t nb32 = npad / kTileRowBlock, nb16 = npad / kTileColBlock;
  hipLaunchKernelGGL(k_tile_bounds<kTileRowBlock>, dim3((unsigned)ceil_div(nb32, kWG)), dim3(kWG), 0, st, src_t, n, nb32,
                     bnd32);
  hipLaunchKernelGGL(k_tile_bounds<kTileColBlock>, dim3((unsigned)ceil_div(nb16, kWG)), dim3(kWG), 0, st, src_t, n, nb16,
                     bnd16);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    delete p;
    return fail(NFR_ERR_HIP, "pack launch failed: %s", hipGetErrorString(e));
  }
  *out = p;
  return NFR_OK;
}

int nfr_problem_create(nfr_context* ctx, int64_t n, const double* xyz_dev, const double* q_dev, void* pack_dev,
                       size_t pack_bytes, nfr_problem** out) {
  return nfr_problem_create_periodic(ctx, n, xyz_dev, q_dev, 0.0, pack_dev, pack_bytes, out);
}

double nfr_problem_period(const nfr_problem* prob) { return prob ? prob->view.period : -1.0; }

int nfr_problem_destroy(nfr_problem* prob) {
  if (prob && prob->step_graph) {
    // the executable graph may only be released once its launches have run
    (void)hipSetDevice(prob->ctx->device);
    (void)hipStreamSynchronize(prob->ctx->stream);
    (void)hipGraphExecDestroy(prob->step_graph);
  }
  delete prob;
  return NFR_OK;
}

int64_t nfr_problem_n(const nfr_problem* prob) { return prob ? prob->view.n : -1; }
int64_t nfr_problem_npad(const nfr_problem* prob) { return prob ? prob->view.npad : -1; }

size_t nfr_far_blocks_workspace_size(const nfr_problem* prob) {
  if (!prob) return 0;
  return align256(size_t(prob->view.npad / kTileRowBlock) * sizeof(int64_t));
}

int nfr_far_blocks(nfr_problem* prob, const nfr_kernel* kernel, void* ws_dev, size_t ws_bytes, int64_t* far_blocks,
                   int64_t* total_blocks) {
  int st;
  if ((st = check_problem(prob)) || (st = check_kernel(kernel))) return st;
  if (!far_blocks || !total_blocks) return fail(NFR_ERR_INVALID_ARG, "NULL output pointer");
  const ProblemView& pv = prob->view;
  const int64_t nrow = pv.npad / kTileRowBlock, ncol = pv.npad / kTileColBlock;
  *total_blocks = nrow * ncol;
  *far_blocks = 0;
  const nfr_kernel kn = norm_kernel(*kernel);
  const float d2 = far_d2(kn, pv, NFR_FORM_ONTHEFLY_BF16X3);
  if (!(d2 > 0.0f)) return NFR_OK;
  const size_t need = nfr_far_blocks_workspace_size(prob);
  if (!ws_dev || ws_bytes < need) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  NFR_HIP(hipSetDevice(prob->ctx->device));
  hipStream_t s = prob->ctx->stream;
  // the kernel takes far blocks only on its norm expansion path, as it decides
  // on the device: sig^2 max(1, rho) max_j |x_j|^2 <= kNormMaxT
  double qm[2];
  NFR_HIP(hipMemcpyAsync(qm, pv.qmax, sizeof qm, hipMemcpyDeviceToHost, s));
  NFR_HIP(hipStreamSynchronize(s));
  const PairParams pp = pair_params_pow(kn, pv);
  const double s2d = (double)pp.sig * pp.sig;
  if (!(s2d * std::fmax(1.0, (double)pp.rho) * qm[1] <= kNormMaxT)) return NFR_OK;
  int64_t* counts = static_cast<int64_t*>(ws_dev);
  hipLaunchKernelGGL(k_tile_far_count, dim3((unsigned)ceil_div(nrow, kWG)), dim3(kWG), 0, s, pv.bnd32, pv.bnd16, nrow, ncol,
                     d2, counts);
  NFR_HIP_LAUNCH();
  std::vector<int64_t> h(nrow);
  NFR_HIP(hipMemcpyAsync(h.data(), counts, nrow * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  NFR_HIP(hipStreamSynchronize(s));
  int64_t sum = 0;
  for (int64_t v : h) sum += v;
  *far_blocks = sum;
  return NFR_OK;
}

size_t nfr_w_bytes(int64_t n, int form) {
  if (n < 1 || n > kMaxN) return 0;
  const int64_t npad = round_up(n, kPad);
  if (form == NFR_FORM_W_FP32) return align256(size_t(n) * npad * sizeof(float));
  if (mfma_has_w(form)) return mfma_w_bytes(n, npad);
  return 0;
}

int nfr_w_build(nfr_problem* prob, const nfr_kernel* kernel, int form, void* w_dev, size_t w_bytes) {
  int st;
  if ((st = check_problem(prob)) || (st = check_kernel(kernel))) return st;
  if ((st = check_form(form))) return st;
  if (form != NFR_FORM_W_FP32 && !mfma_has_w(form)) return fail(NFR_ERR_INVALID_ARG, "form %d has no W matrix", form);
  if (!w_dev) return fail(NFR_ERR_INVALID_ARG, "w_dev is NULL");
  if (reinterpret_cast<uintptr_t>(w_dev) % 256) return fail(NFR_ERR_INVALID_ARG, "W buffer must be 256-byte aligned");
  const ProblemView& pv = prob->view;
  const size_t need = nfr_w_bytes(pv.n, form);
  if (w_bytes < need) return fail(NFR_ERR_WORKSPACE, "W buffer has %zu bytes, needs %zu", w_bytes, need);
  NFR_HIP(hipSetDevice(prob->ctx->device));
  hipStream_t s = prob->ctx->stream;
  if (form == NFR_FORM_W_FP32) {
    hipLaunchKernelGGL(k_w_build_f32, dim3((unsigned)pv.n, (unsigned)ceil_div(pv.npad, kWG)), dim3(kWG), 0, s, pv.xyz,
                       pv.q, pv.n, pv.npad, kernel64(*kernel, pv), static_cast<float*>(w_dev));
  } else {
    launch_mfma_w_build(pv, form, kernel64(*kernel, pv), w_dev, s);
  }
  NFR_HIP_LAUNCH();
  return NFR_OK;
}

size_t nfr_apply_workspace_size(const nfr_problem* prob, int B, int form) {
  if (!prob || B < 1 || B > kMaxB) return 0;
  form = resolve_form(form, prob->view.n, B);
  return carve(nullptr, prob->view, B, form, false).bytes;
}

}  // extern "C"

namespace {

// Argument checks shared by nfr_apply and nfr_apply_noalloc; resolves AUTO.
int apply_check(const nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, const double* u_dev,
                const double* y_dev, int* form, const void* w_dev) {
  int st;
  if ((st = check_problem(prob)) || (st = check_kernel(kernel)) || (st = check_firing(firing)) || (st = check_form(*form)))
    return st;
  if (B < 1 || B > kMaxB) return fail(NFR_ERR_INVALID_ARG, "B = %d outside [1, %d]", B, kMaxB);
  if (!u_dev || !y_dev) return fail(NFR_ERR_INVALID_ARG, "NULL state pointer");
  *form = resolve_form(*form, prob->view.n, B);
  return check_w(prob, *form, w_dev);
}

// Prep, pair sums and reduction of one application into y_dev, with the
// scratch of `w` (carved by the caller).
int apply_launch(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, const double* u_dev,
                 double* y_dev, int form, const void* w_dev, const Workspace& w) {
  int st;
  const bool tiled = use_tile_order(*kernel, prob->view, form);
  const ProblemView pv = tiled ? tile_view(prob->view) : prob->view;
  NFR_HIP(hipSetDevice(prob->ctx->device));
  hipStream_t s = prob->ctx->stream;
  const Firing fr = firing_of(*firing);
  const double* u_in = u_dev;
  double* y_out = y_dev;
  if (tiled) {
    launch_tile_gather(pv, B, u_dev, w.ut, s);
    u_in = w.ut;
    y_out = w.yt;
  }
  if ((st = launch_prep(pv, form, B, u_in, fr, w, nullptr, s))) return st;
  if ((st = launch_pairs(prob->ctx, pv, *kernel, form, B, w_dev, w))) return st;
  const int nsplit = w.nsplit;
  const int64_t total = pv.n * (int64_t)B;
  if (is_mfma_form(form))
    launch_mfma_reduce(pv, form, B, w.part, nsplit, y_out, s);
  else
    NFR_LAUNCH_SLOTS(k_reduce_partials, nsplit, total, s, w.part, nsplit, pv.n, pv.npad, B, y_out);
  if (tiled) launch_tile_scatter(pv, B, w.yt, y_dev, s);
  NFR_HIP_LAUNCH();
  return NFR_OK;
}

}  // namespace

extern "C" {

int nfr_apply(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, const double* u_dev,
              double* y_dev, int form, const void* w_dev, void* ws_dev, size_t ws_bytes) {
  int st;
  if ((st = apply_check(prob, kernel, firing, B, u_dev, y_dev, &form, w_dev))) return st;
  const Workspace w = carve(ws_dev, prob->view, B, form, false);
  if (!ws_dev || ws_bytes < w.bytes) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, w.bytes);
  return apply_launch(prob, kernel, firing, B, u_dev, y_dev, form, w_dev, w);
}

int nfr_apply_noalloc(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B,
                      const double* u_dev, double* y_dev, int form, const void* w_dev) {
  int st;
  if ((st = apply_check(prob, kernel, firing, B, u_dev, y_dev, &form, w_dev))) return st;
  void* base = scratch_of(prob->ctx->device);
  if (!base) return fail(NFR_ERR_INTERNAL, "no scratch address for device %d", prob->ctx->device);
  // carved once (the plan is read once); nothing is launched unless it fits
  const Workspace w = carve(base, prob->view, B, form, false);
  if (w.bytes > kScratchBytes)
    return fail(NFR_ERR_WORKSPACE, "this application needs %zu scratch bytes; the fixed scratch holds %zu (use nfr_apply with a workspace)",
                w.bytes, kScratchBytes);
  return apply_launch(prob, kernel, firing, B, u_dev, y_dev, form, w_dev, w);
}

size_t nfr_integrate_workspace_size(const nfr_problem* prob, int B, int form) {
  if (!prob || B < 1 || B > kMaxB) return 0;
  form = resolve_form(form, prob->view.n, B);
  return carve(nullptr, prob->view, B, form, true).bytes;
}

int nfr_integrate(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, double* u_dev,
                  double dt, int64_t steps, int form, const void* w_dev, double* ckpt_dev, int64_t ckpt_every,
                  int use_graph, void* ws_dev, size_t ws_bytes) {
  int st;
  if ((st = check_problem(prob)) || (st = check_kernel(kernel)) || (st = check_firing(firing)) || (st = check_form(form)))
    return st;
  if (B < 1 || B > kMaxB) return fail(NFR_ERR_INVALID_ARG, "B = %d outside [1, %d]", B, kMaxB);
  if (!u_dev) return fail(NFR_ERR_INVALID_ARG, "u_dev is NULL");
  if (!is_finite_d(dt)) return fail(NFR_ERR_NONFINITE, "dt must be finite");
  if (!(dt > 0.0)) return fail(NFR_ERR_INVALID_ARG, "dt must be > 0");
  if (steps < 0) return fail(NFR_ERR_INVALID_ARG, "steps must be >= 0");
  if (ckpt_dev && ckpt_every < 1) return fail(NFR_ERR_INVALID_ARG, "ckpt_every must be >= 1");
  form = resolve_form(form, prob->view.n, B);
  // the fused BF16 form steps the states in the tile order (w.ut)
  const bool tiled = use_tile_order(*kernel, prob->view, form);
  const ProblemView pv = tiled ? tile_view(prob->view) : prob->view;
  if ((st = check_w(prob, form, w_dev))) return st;
  const Workspace w = carve(ws_dev, pv, B, form, true);
  if (!ws_dev || ws_bytes < w.bytes) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, w.bytes);
  if (use_graph && prob->ctx->stream == nullptr)
    return fail(NFR_ERR_INVALID_ARG, "graph replay needs a non-default stream");
  NFR_HIP(hipSetDevice(prob->ctx->device));
  hipStream_t s = prob->ctx->stream;
  const Firing fr = firing_of(*firing);
  const size_t state_bytes = size_t(pv.n) * B * sizeof(double);
  if (ckpt_dev) NFR_HIP(hipMemcpyAsync(ckpt_dev, u_dev, state_bytes, hipMemcpyDeviceToDevice, s));
  if (steps == 0) return NFR_OK;
  double* u_run = u_dev;
  if (tiled) {
    launch_tile_gather(pv, B, u_dev, w.ut, s);
    NFR_HIP_LAUNCH();
    u_run = w.ut;
  }
  if ((st = launch_prep(pv, form, B, u_run, fr, w, w.v, s))) return st;

  auto one_step = [&]() -> int {
    for (int stage = 1; stage <= 4; ++stage) {
      int r;
      if ((r = launch_stage(prob->ctx, pv, *kernel, form, B, w_dev, w, stage, dt, u_run, fr))) return r;
    }
    return NFR_OK;
  };
  auto checkpoint = [&](int64_t done) -> int {
    if (ckpt_dev && done % ckpt_every == 0) {
      double* dst = ckpt_dev + (done / ckpt_every) * (int64_t)pv.n * B;
      if (tiled) {
        launch_tile_scatter(pv, B, u_run, dst, s);
        NFR_HIP_LAUNCH();
      } else {
        NFR_HIP(hipMemcpyAsync(dst, u_dev, state_bytes, hipMemcpyDeviceToDevice, s));
      }
    }
    return NFR_OK;
  };

  // Graph replay: groups of g consecutive RK4 steps are captured once into one
  // graph, kept with the problem and replayed by this and later calls with the
  // same arguments (one graph launch per g steps).  With checkpoints g divides
  // ckpt_every, so every checkpoint falls between two replays; the steps left
  // over after the last whole group are launched directly (same kernels).
  int64_t g = 0;
  if (use_graph) {
    g = std::min<int64_t>(steps, kGraphMaxSteps);
    if (ckpt_dev)
      while (ckpt_every % g) --g;
  }
  if (g > 0) {
    StepGraphKey key;
    std::memset(&key, 0, sizeof key);
    key.form = form;
    key.B = B;
    key.kind = kernel->kind;
    key.dt = dt;
    key.A_e = kernel->A_e;
    key.s_e = kernel->s_e;
    key.A_i = kernel->A_i;
    key.s_i = kernel->s_i;
    key.beta = firing->beta;
    key.theta = firing->theta;
    key.theta_dev = firing->theta_dev;
    key.u = u_dev;
    key.w = w_dev;
    key.ws = ws_dev;
    key.steps_per_graph = g;
    key.otf_chunk = w.otf.chunk;
    key.otf_tiles = w.otf.tiles;
    key.nsplit = w.nsplit;
    key.otf_bs = w.otf.bs;
    key.otf_nsb = w.otf.nsb;
    if (prob->step_graph && std::memcmp(&key, &prob->step_key, sizeof key) != 0) {
      NFR_HIP(hipStreamSynchronize(s));   // earlier replays of the old graph must have run
      (void)hipGraphExecDestroy(prob->step_graph);
      prob->step_graph = nullptr;
    }
    if (!prob->step_graph) {
      hipGraph_t graph = nullptr;
      NFR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      prob->ctx->capturing = true;
      int r = NFR_OK;
      for (int64_t i = 0; i < g && r == NFR_OK; ++i) r = one_step();
      prob->ctx->capturing = false;
      const hipError_t e_end = hipStreamEndCapture(s, &graph);
      if (r) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
      }
      if (e_end != hipSuccess) return fail(NFR_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e_end));
      size_t nodes = 0;
      (void)hipGraphGetNodes(graph, nullptr, &nodes);
      hipGraphExec_t exec = nullptr;
      const hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e_inst != hipSuccess) return fail(NFR_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e_inst));
      prob->step_graph = exec;
      prob->step_key = key;
      prob->step_graph_nodes = (int64_t)nodes;
    }
    prob->ctx->last_graph_nodes = prob->step_graph_nodes;
    prob->ctx->last_graph_steps = g;
  }
  int64_t done = 0;
  if (g > 0) {
    for (; done + g <= steps; done += g) {
      NFR_HIP(hipGraphLaunch(prob->step_graph, s));
      if ((st = checkpoint(done + g))) return st;
    }
  }
  for (; done < steps; ++done) {
    if ((st = one_step())) return st;
    if ((st = checkpoint(done + 1))) return st;
  }
  if (tiled) {
    launch_tile_scatter(pv, B, u_run, u_dev, s);
    NFR_HIP_LAUNCH();
  }
  return NFR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- adjoint

namespace {

struct AdjWorkspace {
  Workspace fwd;
  double* store = nullptr;   // C x 4 x n stage inputs of one segment
  double* useg = nullptr;
  double* lam = nullptr;
  float* lam32 = nullptr;
  double* ubar = nullptr;
  double* unbar = nullptr;
  double* apart = nullptr;   // 4 x nsplit x npad
  double* pblk = nullptr;    // nblocks x 8
  double* pbar = nullptr;    // 8
  size_t bytes = 0;
};

// Workgroups of one reverse-stage combine (slot_lanes lanes per node).
int64_t adj_blocks(int64_t n, int nsplit) { return ceil_div(n * slot_lanes(nsplit), kWG); }

AdjWorkspace carve_adjoint(void* base, const ProblemView& pv, int64_t ckpt_every) {
  AdjWorkspace a;
  a.fwd = carve(base, pv, 1, NFR_FORM_ONTHEFLY_FP32, true);
  char* p = static_cast<char*>(base);
  size_t off = a.fwd.bytes;
  auto take = [&](size_t bytes) {
    char* r = p ? p + off : nullptr;
    off += align256(bytes);
    return r;
  };
  const int nsplit = (int)adj_tiles(pv.npad);
  const int64_t nblocks = adj_blocks(pv.n, nsplit);
  a.store = reinterpret_cast<double*>(take(size_t(ckpt_every) * 4 * pv.n * sizeof(double)));
  a.useg = reinterpret_cast<double*>(take(size_t(pv.n) * sizeof(double)));
  a.lam = reinterpret_cast<double*>(take(size_t(pv.n) * sizeof(double)));
  a.lam32 = reinterpret_cast<float*>(take(size_t(pv.npad) * sizeof(float)));
  a.ubar = reinterpret_cast<double*>(take(size_t(pv.n) * sizeof(double)));
  a.unbar = reinterpret_cast<double*>(take(size_t(pv.n) * sizeof(double)));
  a.apart = reinterpret_cast<double*>(take(size_t(4) * nsplit * pv.npad * sizeof(double)));
  a.pblk = reinterpret_cast<double*>(take(size_t(nblocks) * 8 * sizeof(double)));
  a.pbar = reinterpret_cast<double*>(take(8 * sizeof(double)));
  a.bytes = off;
  return a;
}

AdjCoef adj_coef(const nfr_kernel& k) {
  AdjCoef c;
  c.Ae = k.A_e;
  c.Ai = k.A_i;
  if (k.kind == NFR_KERNEL_GAUSS_MH) {
    c.kse = 2.0 / (k.s_e * kLog2e);
    c.ksi = 2.0 * k.s_e * k.s_e / (k.s_i * k.s_i * k.s_i * kLog2e);
  } else {
    c.kse = 1.0 / (k.s_e * kLog2e);
    c.ksi = k.s_e / (k.s_i * k.s_i * kLog2e);
  }
  // rho = 1/m: the pair kernel's T sums are in the inhibitory argument, t / m
  if (const int code = sym_pow_code(k)) {
    c.kse *= code + 1;
    c.ksi *= code + 1;
  }
  return c;
}

}  // namespace

extern "C" {

size_t nfr_adjoint_workspace_size(const nfr_problem* prob, int64_t steps, int64_t ckpt_every) {
  if (!prob || steps < 0 || ckpt_every < 1) return 0;
  return carve_adjoint(nullptr, prob->view, ckpt_every).bytes;
}

int nfr_adjoint(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, const double* ckpt_dev,
                int64_t ckpt_every, int64_t steps, double dt, const double* ubarT_dev, double* ubar0_dev,
                double* pbar_host, void* ws_dev, size_t ws_bytes) {
  int st;
  if ((st = check_problem(prob)) || (st = check_kernel(kernel)) || (st = check_firing(firing))) return st;
  if (firing->theta_dev) return fail(NFR_ERR_INVALID_ARG, "the adjoint supports one shared threshold (theta_dev must be NULL)");
  if (!ckpt_dev || !ubarT_dev || !ubar0_dev || !pbar_host) return fail(NFR_ERR_INVALID_ARG, "NULL argument");
  if (ckpt_every < 1) return fail(NFR_ERR_INVALID_ARG, "ckpt_every must be >= 1");
  if (steps < 0) return fail(NFR_ERR_INVALID_ARG, "steps must be >= 0");
  if (!is_finite_d(dt)) return fail(NFR_ERR_NONFINITE, "dt must be finite");
  if (!(dt > 0.0)) return fail(NFR_ERR_INVALID_ARG, "dt must be > 0");
  const ProblemView& pv = prob->view;
  const AdjWorkspace a = carve_adjoint(ws_dev, pv, ckpt_every);
  if (!ws_dev || ws_bytes < a.bytes) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, a.bytes);
  NFR_HIP(hipSetDevice(prob->ctx->device));
  nfr_context* ctx = prob->ctx;
  hipStream_t s = ctx->stream;
  const Firing fr = firing_of(*firing);
  const PairParams pp = pair_params_pow(*kernel, pv);
  const AdjCoef co = adj_coef(*kernel);
  const int nt = (int)adj_tiles(pv.npad);
  const int adj_code = kind_code(*kernel, pv) | (sym_pow_code(*kernel) << 2);
  const int64_t n = pv.n;
  const int64_t nblocks = adj_blocks(n, nt);
  const size_t vbytes = size_t(n) * sizeof(double);
  const int form = NFR_FORM_ONTHEFLY_FP32;

  hipLaunchKernelGGL(k_adj_init, dim3((unsigned)ceil_div(pv.npad, kWG)), dim3(kWG), 0, s, ubarT_dev, n, pv.npad, dt,
                     a.ubar, a.unbar, a.lam, a.lam32);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)ceil_div(nblocks * 8, kWG)), dim3(kWG), 0, s, a.pblk, nblocks * 8);
  NFR_HIP_LAUNCH();

  // recompute of one segment of `len` steps from a.useg, keeping every stage input
  auto recompute = [&](int64_t len) -> int {
    int r;
    for (int64_t l = 0; l < len; ++l) {
      for (int stage = 1; stage <= 4; ++stage) {
        NFR_HIP(hipMemcpyAsync(a.store + (l * 4 + stage - 1) * n, a.fwd.v, vbytes, hipMemcpyDeviceToDevice, s));
        if ((r = launch_stage(ctx, pv, *kernel, form, 1, nullptr, a.fwd, stage, dt, a.useg, fr))) return r;
      }
    }
    return NFR_OK;
  };
  // reverse sweep over one segment of `len` steps
  auto reverse = [&](int64_t len) -> int {
    int r;
    for (int64_t l = len - 1; l >= 0; --l) {
      for (int stage = 4; stage >= 1; --stage) {
        if ((r = timing_mark(ctx))) return r;
        const dim3 agrid((unsigned)sym_pairs(nt));
#define NFR_ADJ_CASE(K) \
  case K: hipLaunchKernelGGL(k_sym_adjoint<K>, agrid, dim3(kAdjThreads), 0, s, pv.src, a.lam32, pv.npad, nt, pp, a.apart); break;
        switch (adj_code) {
          NFR_ADJ_CASE(0) NFR_ADJ_CASE(1) NFR_ADJ_CASE(2) NFR_ADJ_CASE(3)
          NFR_ADJ_CASE(4) NFR_ADJ_CASE(5) NFR_ADJ_CASE(6) NFR_ADJ_CASE(7)
          NFR_ADJ_CASE(8) NFR_ADJ_CASE(9) NFR_ADJ_CASE(10) NFR_ADJ_CASE(11)
          NFR_ADJ_CASE(12) NFR_ADJ_CASE(13) NFR_ADJ_CASE(14) NFR_ADJ_CASE(15)
          default: return fail(NFR_ERR_INTERNAL, "no adjoint kernel for this kernel code");
        }
#undef NFR_ADJ_CASE
        NFR_HIP_LAUNCH();
        if ((r = timing_mark(ctx))) return r;
        NFR_LAUNCH_SLOTS(k_adj_combine, nt, n, s, a.apart, nt, n, pv.npad,
                           stage, dt, co, pv.q, fr, a.store + (l * 4 + stage - 1) * n, a.ubar, a.unbar, a.lam,
                           a.lam32, a.pblk);
        NFR_HIP_LAUNCH();
      }
    }
    return NFR_OK;
  };

  // On a non-default stream the recompute and the reverse sweep of a segment
  // are captured once per segment length (every segment uses the same
  // buffers) and replayed; the null stream cannot be captured, so there every
  // kernel is launched.
  struct SegGraphs {
    int64_t len = -1;
    hipGraphExec_t rec = nullptr, rev = nullptr;
  };
  struct GraphCache {
    hipStream_t stream;
    SegGraphs g[2];
    ~GraphCache() {
      bool any = false;
      for (auto& e : g) any = any || e.rec || e.rev;
      if (!any) return;
      (void)hipStreamSynchronize(stream);   // executable graphs are released once their launches have run
      for (auto& e : g) {
        if (e.rec) (void)hipGraphExecDestroy(e.rec);
        if (e.rev) (void)hipGraphExecDestroy(e.rev);
      }
    }
  } cache{s, {}};
  auto capture = [&](auto&& body, int64_t len, hipGraphExec_t* out) -> int {
    hipGraph_t graph = nullptr;
    NFR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    const int r = body(len);
    ctx->capturing = false;
    const hipError_t e_end = hipStreamEndCapture(s, &graph);
    if (r) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    if (e_end != hipSuccess) return fail(NFR_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e_end));
    const hipError_t e_inst = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e_inst != hipSuccess) return fail(NFR_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e_inst));
    return NFR_OK;
  };
  auto graphs_for = [&](int64_t len, SegGraphs** out) -> int {
    for (auto& e : cache.g)
      if (e.len == len) {
        *out = &e;
        return NFR_OK;
      }
    SegGraphs& e = cache.g[0].len < 0 ? cache.g[0] : cache.g[1];
    e.len = len;
    int r;
    if ((r = capture(recompute, len, &e.rec)) || (r = capture(reverse, len, &e.rev))) return r;
    *out = &e;
    return NFR_OK;
  };

  const int64_t nseg = ceil_div(steps, ckpt_every);
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t s0 = seg * ckpt_every;
    const int64_t len = (steps - s0) < ckpt_every ? (steps - s0) : ckpt_every;
    NFR_HIP(hipMemcpyAsync(a.useg, ckpt_dev + seg * n, vbytes, hipMemcpyDeviceToDevice, s));
    if ((st = launch_prep(pv, form, 1, a.useg, fr, a.fwd, a.fwd.v, s))) return st;
    if (s != nullptr) {
      SegGraphs* gs = nullptr;
      if ((st = graphs_for(len, &gs))) return st;
      NFR_HIP(hipGraphLaunch(gs->rec, s));
      NFR_HIP(hipGraphLaunch(gs->rev, s));
    } else {
      if ((st = recompute(len)) || (st = reverse(len))) return st;
    }
  }
  NFR_HIP(hipMemcpyAsync(ubar0_dev, a.ubar, vbytes, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_adj_finalize, dim3(1), dim3(64), 0, s, a.pblk, nblocks, a.pbar);
  NFR_HIP_LAUNCH();
  NFR_HIP(hipMemcpyAsync(pbar_host, a.pbar, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
  NFR_HIP(hipStreamSynchronize(s));
  return NFR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- uneven batch

struct nfr_batch {
  nfr_context* ctx = nullptr;
  std::vector<nfr_problem*> probs;
  std::vector<nfr_kernel> kernels;
  std::vector<nfr_firing> firings;
  std::vector<int> B;
  int64_t chunk = 2048;
  int wgs_per_cu = 4;
  std::vector<BatchProblemDev> table;
  std::vector<BatchItem> items;
};

namespace {

constexpr int64_t kBatchChunks[] = {1024, 2048, 4096, 8192};
constexpr int kBatchWgs[] = {2, 4, 8};
constexpr int64_t kBatchMinChunk = 1024;

struct BatchLayout {
  size_t table_off = 0, items_off = 0, bytes = 0;
  std::vector<size_t> g_off, part_off, v_off, ksum_off;
  size_t max_items = 0;
};

int64_t batch_items_for(const nfr_problem* p, int B, int64_t chunk) {
  const int64_t npad = p->view.npad;
  const int bs = batch_bs(B);
  return ceil_div(npad, (int64_t)kWG * batch_tpt(bs)) * ceil_div(npad, chunk) * ceil_div(B, bs);
}

BatchLayout batch_layout(const nfr_batch* b) {
  BatchLayout L;
  const int P = (int)b->probs.size();
  size_t off = 0;
  L.table_off = off;
  off += align256(sizeof(BatchProblemDev) * P);
  for (int p = 0; p < P; ++p) L.max_items += batch_items_for(b->probs[p], b->B[p], kBatchMinChunk);
  L.items_off = off;
  off += align256(sizeof(BatchItem) * L.max_items);
  for (int p = 0; p < P; ++p) {
    const ProblemView& pv = b->probs[p]->view;
    const int Bp = b->B[p];
    L.g_off.push_back(off);
    off += align256(size_t(pv.npad) * Bp * sizeof(float));
    L.part_off.push_back(off);
    off += align256(size_t(ceil_div(pv.npad, kBatchMinChunk)) * Bp * pv.npad * sizeof(double));
    L.v_off.push_back(off);
    off += align256(size_t(pv.n) * Bp * sizeof(double));
    L.ksum_off.push_back(off);
    off += align256(size_t(pv.n) * Bp * sizeof(double));
  }
  L.bytes = off;
  return L;
}

// Fills the host table and the sorted item list for the batch's current chunk.
void batch_build(nfr_batch* b, const BatchLayout& L, char* ws, double* const* u_devs) {
  const int P = (int)b->probs.size();
  b->table.assign(P, BatchProblemDev{});
  b->items.clear();
  std::vector<double> cost;
  int64_t eoff = 0, goff = 0;
  for (int p = 0; p < P; ++p) {
    const ProblemView& pv = b->probs[p]->view;
    const int Bp = b->B[p];
    BatchProblemDev& d = b->table[p];
    d.src = pv.src;
    d.q = pv.q;
    d.n = pv.n;
    d.npad = pv.npad;
    d.B = Bp;
    d.bs = batch_bs(Bp);
    const nfr_kernel kn = norm_kernel(b->kernels[p]);
    d.kind = kind_code(kn, pv);
    d.chunk = b->chunk;
    d.nsplit = (int)ceil_div(pv.npad, b->chunk);
    d.pp = pair_params(kn, pv);
    d.fr = firing_of(b->firings[p]);
    d.g = reinterpret_cast<float*>(ws + L.g_off[p]);
    d.part = reinterpret_cast<double*>(ws + L.part_off[p]);
    d.u = u_devs ? u_devs[p] : nullptr;
    d.v = reinterpret_cast<double*>(ws + L.v_off[p]);
    d.ksum = reinterpret_cast<double*>(ws + L.ksum_off[p]);
    d.elem_off = eoff;
    d.gel_off = goff;
    eoff += pv.n * Bp;
    goff += pv.npad * Bp;
    const int tpt = batch_tpt(d.bs);
    const int64_t tiles = ceil_div(pv.npad, (int64_t)kWG * tpt);
    const int sbs = (int)ceil_div(Bp, d.bs);
    for (int64_t t = 0; t < tiles; ++t)
      for (int sp = 0; sp < d.nsplit; ++sp)
        for (int sb = 0; sb < sbs; ++sb) {
          const double tg = (double)std::min<int64_t>(kWG * tpt, pv.npad - t * kWG * tpt);
          const double sc = (double)std::min<int64_t>(b->chunk, pv.npad - sp * b->chunk);
          const double st = (double)std::min(d.bs, Bp - sb * d.bs);
          const double per_pair = ((d.kind & 1) ? 1.3 : 1.0) + ((d.kind & 2) ? 0.2 : 0.0) + 0.25 * (st - 1.0);
          b->items.push_back(BatchItem{p, (int)t, sp, sb});
          cost.push_back(tg * sc * per_pair);
        }
  }
  std::vector<size_t> order(b->items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
  std::vector<BatchItem> sorted(order.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = b->items[order[i]];
  b->items.swap(sorted);
}

int64_t batch_total(const nfr_batch* b, bool padded) {
  int64_t t = 0;
  for (size_t p = 0; p < b->probs.size(); ++p)
    t += (padded ? b->probs[p]->view.npad : b->probs[p]->view.n) * b->B[p];
  return t;
}

int batch_upload(nfr_batch* b, const BatchLayout& L, char* ws, hipStream_t s) {
  NFR_HIP(hipMemcpyAsync(ws + L.table_off, b->table.data(), sizeof(BatchProblemDev) * b->table.size(),
                         hipMemcpyHostToDevice, s));
  NFR_HIP(hipMemcpyAsync(ws + L.items_off, b->items.data(), sizeof(BatchItem) * b->items.size(),
                         hipMemcpyHostToDevice, s));
  // the host vectors are reused by the next call: finish the copies first
  NFR_HIP(hipStreamSynchronize(s));
  return NFR_OK;
}

void batch_launch_pairs(const nfr_batch* b, const BatchLayout& L, char* ws, hipStream_t s) {
  const int nitems = (int)b->items.size();
  int grid = b->ctx->cu_count * b->wgs_per_cu;
  if (grid > nitems) grid = nitems;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_batch_pairs, dim3((unsigned)grid), dim3(kWG), 0, s,
                     reinterpret_cast<const BatchProblemDev*>(ws + L.table_off),
                     reinterpret_cast<const BatchItem*>(ws + L.items_off), nitems);
}

int check_batch_states(const nfr_batch* b, double* const* u_devs) {
  if (!u_devs) return fail(NFR_ERR_INVALID_ARG, "u_devs is NULL");
  for (size_t p = 0; p < b->probs.size(); ++p)
    if (!u_devs[p]) return fail(NFR_ERR_INVALID_ARG, "state pointer %zu is NULL", p);
  return NFR_OK;
}

}  // namespace

extern "C" {

int nfr_batch_create(nfr_context* ctx, int P, nfr_problem* const* probs, const nfr_kernel* kernels,
                     const nfr_firing* firings, const int* B, nfr_batch** out) {
  if (!out) return fail(NFR_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx || !probs || !kernels || !firings || !B) return fail(NFR_ERR_INVALID_ARG, "NULL argument");
  if (P < 1 || P > 65536) return fail(NFR_ERR_INVALID_ARG, "P = %d outside [1, 65536]", P);
  int st;
  for (int p = 0; p < P; ++p) {
    if ((st = check_problem(probs[p]))) return st;
    if (probs[p]->ctx != ctx) return fail(NFR_ERR_INVALID_ARG, "problem %d belongs to another context", p);
    if ((st = check_kernel(&kernels[p])) || (st = check_firing(&firings[p]))) return st;
    if (B[p] < 1 || B[p] > kMaxB) return fail(NFR_ERR_INVALID_ARG, "B[%d] = %d outside [1, %d]", p, B[p], kMaxB);
  }
  nfr_batch* b = new (std::nothrow) nfr_batch;
  if (!b) return fail(NFR_ERR_INTERNAL, "out of host memory");
  b->ctx = ctx;
  b->probs.assign(probs, probs + P);
  b->kernels.assign(kernels, kernels + P);
  b->firings.assign(firings, firings + P);
  b->B.assign(B, B + P);
  *out = b;
  return NFR_OK;
}

int nfr_batch_destroy(nfr_batch* b) {
  delete b;
  return NFR_OK;
}

size_t nfr_batch_workspace_size(const nfr_batch* b) { return b ? batch_layout(b).bytes : 0; }

int nfr_batch_set_config(nfr_batch* b, int64_t chunk, int wgs_per_cu) {
  if (!b) return fail(NFR_ERR_INVALID_ARG, "batch is NULL");
  if (chunk < kBatchMinChunk || chunk % kWG || chunk > (int64_t(1) << 24))
    return fail(NFR_ERR_INVALID_ARG, "chunk must be a multiple of %d, >= %lld", kWG, (long long)kBatchMinChunk);
  if (wgs_per_cu < 1 || wgs_per_cu > 64) return fail(NFR_ERR_INVALID_ARG, "wgs_per_cu outside [1, 64]");
  b->chunk = chunk;
  b->wgs_per_cu = wgs_per_cu;
  return NFR_OK;
}

int nfr_batch_get_config(const nfr_batch* b, int64_t* chunk, int* wgs_per_cu) {
  if (!b || !chunk || !wgs_per_cu) return fail(NFR_ERR_INVALID_ARG, "NULL argument");
  *chunk = b->chunk;
  *wgs_per_cu = b->wgs_per_cu;
  return NFR_OK;
}

int nfr_batch_tune(nfr_batch* b, double* const* u_devs, void* ws_dev, size_t ws_bytes, double* best_ms) {
  if (!b) return fail(NFR_ERR_INVALID_ARG, "batch is NULL");
  int st;
  if ((st = check_batch_states(b, u_devs))) return st;
  const BatchLayout L = batch_layout(b);
  if (!ws_dev || ws_bytes < L.bytes) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.bytes);
  NFR_HIP(hipSetDevice(b->ctx->device));
  hipStream_t s = b->ctx->stream;
  char* ws = static_cast<char*>(ws_dev);
  hipEvent_t e0, e1;
  NFR_HIP(hipEventCreate(&e0));
  NFR_HIP(hipEventCreate(&e1));
  double best = 1e300;
  int64_t best_chunk = b->chunk;
  int best_wgs = b->wgs_per_cu;
  for (int64_t chunk : kBatchChunks) {
    for (int wgs : kBatchWgs) {
      b->chunk = chunk;
      b->wgs_per_cu = wgs;
      batch_build(b, L, ws, u_devs);
      if ((st = batch_upload(b, L, ws, s))) return st;
      const int64_t gtot = batch_total(b, true);
      hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)ceil_div(gtot, kWG)), dim3(kWG), 0, s,
                         reinterpret_cast<const BatchProblemDev*>(ws + L.table_off), (int)b->probs.size(), gtot);
      float ms = 0.0f;
      for (int rep = 0; rep < 2; ++rep) {
        NFR_HIP(hipEventRecord(e0, s));
        batch_launch_pairs(b, L, ws, s);
        NFR_HIP(hipEventRecord(e1, s));
        NFR_HIP(hipEventSynchronize(e1));
        NFR_HIP(hipEventElapsedTime(&ms, e0, e1));
      }
      NFR_HIP_LAUNCH();
      if (ms < best) {
        best = ms;
        best_chunk = chunk;
        best_wgs = wgs;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->chunk = best_chunk;
  b->wgs_per_cu = best_wgs;
  if (best_ms) *best_ms = best;
  return NFR_OK;
}

int nfr_batch_integrate(nfr_batch* b, double* const* u_devs, double dt, int64_t steps, int use_graph, void* ws_dev,
                        size_t ws_bytes) {
  if (!b) return fail(NFR_ERR_INVALID_ARG, "batch is NULL");
  int st;
  if ((st = check_batch_states(b, u_devs))) return st;
  if (!is_finite_d(dt)) return fail(NFR_ERR_NONFINITE, "dt must be finite");
  if (!(dt > 0.0)) return fail(NFR_ERR_INVALID_ARG, "dt must be > 0");
  if (steps < 0) return fail(NFR_ERR_INVALID_ARG, "steps must be >= 0");
  const BatchLayout L = batch_layout(b);
  if (!ws_dev || ws_bytes < L.bytes) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.bytes);
  if (use_graph && b->ctx->stream == nullptr) return fail(NFR_ERR_INVALID_ARG, "graph replay needs a non-default stream");
  NFR_HIP(hipSetDevice(b->ctx->device));
  hipStream_t s = b->ctx->stream;
  char* ws = static_cast<char*>(ws_dev);
  batch_build(b, L, ws, u_devs);
  if ((st = batch_upload(b, L, ws, s))) return st;
  if (steps == 0) return NFR_OK;
  const int P = (int)b->probs.size();
  const auto* table = reinterpret_cast<const BatchProblemDev*>(ws + L.table_off);
  const int64_t gtot = batch_total(b, true);
  const int64_t etot = batch_total(b, false);
  hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)ceil_div(gtot, kWG)), dim3(kWG), 0, s, table, P, gtot);
  NFR_HIP_LAUNCH();

  auto one_step = [&]() -> int {
    for (int stage = 1; stage <= 4; ++stage) {
      int r;
      if ((r = timing_mark(b->ctx))) return r;
      batch_launch_pairs(b, L, ws, s);
      NFR_HIP_LAUNCH();
      if ((r = timing_mark(b->ctx))) return r;
      hipLaunchKernelGGL(k_batch_combine, dim3((unsigned)ceil_div(etot, kWG)), dim3(kWG), 0, s, table, P, etot, stage,
                         dt);
      NFR_HIP_LAUNCH();
    }
    return NFR_OK;
  };

  // Graph replay: g consecutive steps captured into one graph per call, the
  // steps left over after the last whole group launched directly.
  const int64_t g = use_graph ? std::min<int64_t>(steps, kBatchGraphMaxSteps) : 0;
  hipGraphExec_t exec = nullptr;
  if (g > 0) {
    hipGraph_t graph = nullptr;
    NFR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    b->ctx->capturing = true;
    int r = NFR_OK;
    for (int64_t i = 0; i < g && r == NFR_OK; ++i) r = one_step();
    b->ctx->capturing = false;
    const hipError_t e_end = hipStreamEndCapture(s, &graph);
    if (r) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    if (e_end != hipSuccess) return fail(NFR_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e_end));
    size_t nodes = 0;
    (void)hipGraphGetNodes(graph, nullptr, &nodes);
    const hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e_inst != hipSuccess) return fail(NFR_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e_inst));
    b->ctx->last_graph_nodes = (int64_t)nodes;
    b->ctx->last_graph_steps = g;
  }
  int result = NFR_OK;
  int64_t done = 0;
  if (exec) {
    for (; done + g <= steps; done += g) {
      const hipError_t e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) {
        result = fail(NFR_ERR_HIP, "hipGraphLaunch failed: %s", hipGetErrorString(e));
        break;
      }
    }
  }
  for (; result == NFR_OK && done < steps; ++done) result = one_step();
  if (exec) {
    // the executable graph may only be released once its launches have run
    const hipError_t e = hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(exec);
    if (e != hipSuccess && result == NFR_OK) result = fail(NFR_ERR_HIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
  }
  return result;
}

}  // extern "C"

// ---------------------------------------------------------------- Adams-Bashforth 5

extern "C" {

size_t nfr_integrate_ab5_workspace_size(const nfr_problem* prob, int B, int form) {
  if (!prob || B < 1 || B > kMaxB) return 0;
  form = resolve_form(form, prob->view.n, B);
  return carve(nullptr, prob->view, B, form, true).bytes + align256(size_t(5) * prob->view.n * B * sizeof(double));
}

int nfr_integrate_ab5(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, double* u_dev,
                      double dt, int64_t steps, int form, const void* w_dev, void* ws_dev, size_t ws_bytes) {
  int st;
  if ((st = check_problem(prob)) || (st = check_kernel(kernel)) || (st = check_firing(firing)) || (st = check_form(form)))
    return st;
  if (B < 1 || B > kMaxB) return fail(NFR_ERR_INVALID_ARG, "B = %d outside [1, %d]", B, kMaxB);
  if (!u_dev) return fail(NFR_ERR_INVALID_ARG, "u_dev is NULL");
  if (!is_finite_d(dt)) return fail(NFR_ERR_NONFINITE, "dt must be finite");
  if (!(dt > 0.0)) return fail(NFR_ERR_INVALID_ARG, "dt must be > 0");
  if (steps < 0) return fail(NFR_ERR_INVALID_ARG, "steps must be >= 0");
  const ProblemView& pv = prob->view;
  form = resolve_form(form, pv.n, B);
  if ((st = check_w(prob, form, w_dev))) return st;
  const Workspace w = carve(ws_dev, pv, B, form, true);
  const size_t need = nfr_integrate_ab5_workspace_size(prob, B, form);
  if (!ws_dev || ws_bytes < need) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  double* hist = reinterpret_cast<double*>(static_cast<char*>(ws_dev) + w.bytes);
  NFR_HIP(hipSetDevice(prob->ctx->device));
  hipStream_t s = prob->ctx->stream;
  const Firing fr = firing_of(*firing);
  if (steps == 0) return NFR_OK;
  if ((st = launch_prep(pv, form, B, u_dev, fr, w, w.v, s))) return st;
  const int64_t nb = pv.n * (int64_t)B;
  for (int64_t n = 0; n < steps; ++n) {
    if (n < 4) {
      // classical RK4 start-up; its first stage is F(u_n), kept for the multistep formula
      for (int stage = 1; stage <= 4; ++stage) {
        if ((st = launch_stage(prob->ctx, pv, *kernel, form, B, w_dev, w, stage, dt, u_dev, fr, hist + (n % 5) * nb)))
          return st;
      }
    } else {
      if ((st = launch_pairs(prob->ctx, pv, *kernel, form, B, w_dev, w))) return st;
      if ((st = launch_ab5(pv, form, B, n, dt, u_dev, hist, w, fr, s))) return st;
    }
  }
  return NFR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- synaptic depression

extern "C" {

size_t nfr_integrate_syndep_workspace_size(const nfr_problem* prob, int B) {
  if (!prob || B < 1 || B > kMaxB) return 0;
  return carve(nullptr, prob->view, B, NFR_FORM_ONTHEFLY_FP32, true).bytes +
         2 * align256(size_t(prob->view.n) * B * sizeof(double));
}

int nfr_integrate_syndep(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, double* u_dev,
                         double* a_dev, double tau, double beta_d, double dt, int64_t steps, void* ws_dev,
                         size_t ws_bytes) {
  int st;
  if ((st = check_problem(prob)) || (st = check_kernel(kernel)) || (st = check_firing(firing))) return st;
  if (B < 1 || B > kMaxB) return fail(NFR_ERR_INVALID_ARG, "B = %d outside [1, %d]", B, kMaxB);
  if (!u_dev || !a_dev) return fail(NFR_ERR_INVALID_ARG, "NULL state pointer");
  if (!is_finite_d(dt) || !is_finite_d(tau) || !is_finite_d(beta_d)) return fail(NFR_ERR_NONFINITE, "dt, tau and beta_d must be finite");
  if (!(dt > 0.0) || !(tau > 0.0)) return fail(NFR_ERR_INVALID_ARG, "dt and tau must be > 0");
  if (beta_d < 0.0) return fail(NFR_ERR_INVALID_ARG, "beta_d must be >= 0");
  if (steps < 0) return fail(NFR_ERR_INVALID_ARG, "steps must be >= 0");
  const ProblemView& pv = prob->view;
  const int form = NFR_FORM_ONTHEFLY_FP32;
  const Workspace w = carve(ws_dev, pv, B, form, true);
  const size_t need = nfr_integrate_syndep_workspace_size(prob, B);
  if (!ws_dev || ws_bytes < need) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  char* extra = static_cast<char*>(ws_dev) + w.bytes;
  double* va = reinterpret_cast<double*>(extra);
  double* ka_sum = reinterpret_cast<double*>(extra + align256(size_t(pv.n) * B * sizeof(double)));
  NFR_HIP(hipSetDevice(prob->ctx->device));
  hipStream_t s = prob->ctx->stream;
  const Firing fr = firing_of(*firing);
  if (steps == 0) return NFR_OK;
  hipLaunchKernelGGL(k_syndep_prep, dim3((unsigned)ceil_div(pv.npad * (int64_t)B, kWG)), dim3(kWG), 0, s, u_dev, a_dev,
                     pv.n, pv.npad, B, pv.q, fr, w.g, w.v, va);
  NFR_HIP_LAUNCH();
  const int nsplit = w.nsplit;
  const int64_t total = pv.n * (int64_t)B;
  for (int64_t n = 0; n < steps; ++n) {
    for (int stage = 1; stage <= 4; ++stage) {
      if ((st = launch_pairs(prob->ctx, pv, *kernel, form, B, nullptr, w))) return st;
      NFR_LAUNCH_SLOTS(k_syndep_combine, nsplit, total, s, w.part, nsplit, pv.n, pv.npad, B, stage, dt, 1.0 / tau,
                       beta_d, u_dev, a_dev, w.v, va, w.ksum, ka_sum, pv.q, fr, w.g);
      NFR_HIP_LAUNCH();
    }
  }
  return NFR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- forcing

extern "C" {

int nfr_integrate_forced(nfr_problem* prob, const nfr_kernel* kernel, const nfr_firing* firing, int B, double* u_dev,
                         double dt, int64_t steps, const double* forcing_dev, int form, const void* w_dev,
                         void* ws_dev, size_t ws_bytes) {
  int st;
  if ((st = check_problem(prob)) || (st = check_kernel(kernel)) || (st = check_firing(firing)) || (st = check_form(form)))
    return st;
  if (B < 1 || B > kMaxB) return fail(NFR_ERR_INVALID_ARG, "B = %d outside [1, %d]", B, kMaxB);
  if (!u_dev || !forcing_dev) return fail(NFR_ERR_INVALID_ARG, "NULL device pointer");
  if (!is_finite_d(dt)) return fail(NFR_ERR_NONFINITE, "dt must be finite");
  if (!(dt > 0.0)) return fail(NFR_ERR_INVALID_ARG, "dt must be > 0");
  if (steps < 0) return fail(NFR_ERR_INVALID_ARG, "steps must be >= 0");
  const ProblemView& pv = prob->view;
  form = resolve_form(form, pv.n, B);
  if ((st = check_w(prob, form, w_dev))) return st;
  const Workspace w = carve(ws_dev, pv, B, form, true);
  if (!ws_dev || ws_bytes < w.bytes) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, w.bytes);
  NFR_HIP(hipSetDevice(prob->ctx->device));
  hipStream_t s = prob->ctx->stream;
  const Firing fr = firing_of(*firing);
  if (steps == 0) return NFR_OK;
  if ((st = launch_prep(pv, form, B, u_dev, fr, w, w.v, s))) return st;
  const int64_t nb = pv.n * (int64_t)B;
  static const int slot_of_stage[5] = {0, 0, 1, 1, 2};
  for (int64_t n = 0; n < steps; ++n) {
    for (int stage = 1; stage <= 4; ++stage) {
      const double* gam = forcing_dev + (n * 3 + slot_of_stage[stage]) * nb;
      if ((st = launch_stage(prob->ctx, pv, *kernel, form, B, w_dev, w, stage, dt, u_dev, fr, nullptr, gam))) return st;
    }
  }
  return NFR_OK;
}

}  // extern "C"

// ================================================================ quadrature weights

namespace {

struct QuadWorkspace {
  int* tri = nullptr;
  int* nbr = nullptr;
  double* cen = nullptr;
  double* nrm_tri = nullptr;
  double* proj = nullptr;
  int* st = nullptr;
  double* wE = nullptr;
  int* cnt = nullptr;
  int* cursor = nullptr;
  int64_t* off = nullptr;
  int64_t* bsum = nullptr;
  int* list = nullptr;
  QuadGrid* grid = nullptr;   // node grid of the k-nearest search
  int* gcnt = nullptr;        // nodes per cell
  int* gcursor = nullptr;
  int64_t* gstart = nullptr;  // first node of each cell in gnodes
  int64_t* gbsum = nullptr;
  int* gnodes = nullptr;      // node indices grouped by cell
  size_t bytes = 0;
};

int64_t quad_max_cells(int64_t n) { return 2 * n + 1; }

QuadWorkspace carve_quad(void* base, int64_t n, int64_t ntri, int k) {
  QuadWorkspace w;
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? b + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const size_t tk = size_t(ntri) * k;
  w.tri = static_cast<int*>(take(3 * size_t(ntri) * sizeof(int)));
  w.nbr = static_cast<int*>(take(3 * size_t(ntri) * sizeof(int)));
  w.cen = static_cast<double*>(take(3 * size_t(ntri) * sizeof(double)));
  w.nrm_tri = static_cast<double*>(take(3 * size_t(ntri) * sizeof(double)));
  w.proj = static_cast<double*>(take(3 * size_t(ntri) * sizeof(double)));
  w.st = static_cast<int*>(take(tk * sizeof(int)));
  w.wE = static_cast<double*>(take(tk * sizeof(double)));
  w.cnt = static_cast<int*>(take(size_t(n) * sizeof(int)));
  w.cursor = static_cast<int*>(take(size_t(n) * sizeof(int)));
  w.off = static_cast<int64_t*>(take(size_t(n) * sizeof(int64_t)));
  w.bsum = static_cast<int64_t*>(take(size_t(ceil_div(n, kWG)) * sizeof(int64_t)));
  w.list = static_cast<int*>(take(tk * sizeof(int)));
  const int64_t mc = quad_max_cells(n);
  w.grid = static_cast<QuadGrid*>(take(sizeof(QuadGrid)));
  w.gcnt = static_cast<int*>(take(size_t(mc) * sizeof(int)));
  w.gcursor = static_cast<int*>(take(size_t(mc) * sizeof(int)));
  w.gstart = static_cast<int64_t*>(take(size_t(mc) * sizeof(int64_t)));
  w.gbsum = static_cast<int64_t*>(take(size_t(ceil_div(mc, kWG)) * sizeof(int64_t)));
  w.gnodes = static_cast<int*>(take(size_t(n) * sizeof(int)));
  w.bytes = off;
  return w;
}

bool quad_sizes_ok(int64_t n, int64_t ntri, int k) {
  return n >= 3 && n <= kMaxN && ntri >= 1 && ntri <= 4 * kMaxN && k >= 6 && k <= kQuadMaxK && k <= n &&
         ntri * (int64_t)k < (int64_t(1) << 31);
}

// Neighbour across every edge e (vertex e -> vertex e+1) of every triangle: the
// triangle holding the reverse directed edge.  Fails unless every directed
// edge occurs once and its reverse once (a closed, consistently oriented surface).
// Triangle across each edge: the triangle that holds the reversed directed
// edge.  Directed edges are grouped by their first vertex (a counting sort),
// so the reverse of (a, b) is looked for among the few edges that start at b;
// a repeated directed edge or a missing reverse is reported.
int quad_neighbours(const int32_t* tri, int64_t ntri, int64_t n, std::vector<int>& nbr) {
  const int64_t ne = 3 * ntri;
  std::vector<int64_t> start(size_t(n) + 1, 0);
  for (int64_t e = 0; e < ne; ++e) ++start[size_t(tri[e]) + 1];
  for (int64_t v = 0; v < n; ++v) start[size_t(v) + 1] += start[size_t(v)];
  std::vector<int64_t> fill(start.begin(), start.end() - 1);
  std::vector<int64_t> by_first(static_cast<size_t>(ne));
  for (int64_t e = 0; e < ne; ++e) by_first[size_t(fill[size_t(tri[e])]++)] = e;
  auto head = [&](int64_t e) { return tri[e]; };
  auto tail = [&](int64_t e) { return tri[3 * (e / 3) + (e % 3 + 1) % 3]; };
  for (int64_t v = 0; v < n; ++v)
    for (int64_t p = start[size_t(v)]; p < start[size_t(v) + 1]; ++p)
      for (int64_t r = p + 1; r < start[size_t(v) + 1]; ++r)
        if (tail(by_first[size_t(p)]) == tail(by_first[size_t(r)]))
          return fail(NFR_ERR_INVALID_ARG, "directed edge (%d, %d) occurs twice: the triangulation is not consistently oriented",
                      (int)v, tail(by_first[size_t(p)]));
  nbr.assign(size_t(ne), -1);
  for (int64_t e = 0; e < ne; ++e) {
    const int32_t a = head(e), b = tail(e);
    for (int64_t p = start[size_t(b)]; p < start[size_t(b) + 1]; ++p)
      if (tail(by_first[size_t(p)]) == a) {
        nbr[size_t(e)] = (int)(by_first[size_t(p)] / 3);
        break;
      }
    if (nbr[size_t(e)] < 0)
      return fail(NFR_ERR_INVALID_ARG, "edge (%d, %d) has no reverse: the triangulation is not closed", (int)a, (int)b);
  }
  return NFR_OK;
}

}  // namespace

extern "C" {

size_t nfr_quad_workspace_size(int64_t n, int64_t ntri, int k) {
  if (!quad_sizes_ok(n, ntri, k)) return 0;
  return carve_quad(nullptr, n, ntri, k).bytes;
}

int nfr_quad_weights(nfr_context* ctx, int64_t n, const double* xyz_dev, const double* nrm_dev, int64_t ntri,
                     const int32_t* tri_host, int projection, int k, double* q_dev, int32_t* stencil_dev,
                     double* proj_dev, void* ws_dev, size_t ws_bytes) {
  if (!xyz_dev || !nrm_dev || !tri_host || !q_dev) return fail(NFR_ERR_INVALID_ARG, "NULL argument");
  if (projection != NFR_PROJ_PLANES && projection != NFR_PROJ_ORIGIN && projection != NFR_PROJ_ORTHOGONAL)
    return fail(NFR_ERR_INVALID_ARG, "unknown projection %d", projection);
  const bool planes = projection == NFR_PROJ_PLANES;
  if (!quad_sizes_ok(n, ntri, k))
    return fail(NFR_ERR_INVALID_ARG, "sizes n = %lld, ntri = %lld, k = %d outside the supported range (6 <= k <= %d, k <= n)",
                (long long)n, (long long)ntri, k, kQuadMaxK);
  for (int64_t i = 0; i < 3 * ntri; ++i)
    if (tri_host[i] < 0 || tri_host[i] >= n)
      return fail(NFR_ERR_INVALID_ARG, "triangle %lld has vertex %d outside [0, %lld)", (long long)(i / 3), tri_host[i],
                  (long long)n);
  for (int64_t t = 0; t < ntri; ++t) {
    const int32_t a = tri_host[3 * t], b = tri_host[3 * t + 1], c = tri_host[3 * t + 2];
    if (a == b || b == c || a == c) return fail(NFR_ERR_INVALID_ARG, "triangle %lld repeats a vertex", (long long)t);
  }
  std::vector<int> nbr;
  int st;
  if (planes && (st = quad_neighbours(tri_host, ntri, n, nbr))) return st;
  if (!ctx) return fail(NFR_ERR_INVALID_ARG, "context is NULL");
  const QuadWorkspace w = carve_quad(ws_dev, n, ntri, k);
  if (!ws_dev || ws_bytes < w.bytes) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, w.bytes);
  if (reinterpret_cast<uintptr_t>(ws_dev) % 256) return fail(NFR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  NFR_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  int* stn = stencil_dev ? stencil_dev : w.st;
  double* proj = proj_dev ? proj_dev : w.proj;
  const size_t tk = size_t(ntri) * k;
  NFR_HIP(hipMemcpyAsync(w.tri, tri_host, 3 * size_t(ntri) * sizeof(int), hipMemcpyHostToDevice, s));
  if (planes)
    NFR_HIP(hipMemcpyAsync(w.nbr, nbr.data(), 3 * size_t(ntri) * sizeof(int), hipMemcpyHostToDevice, s));
  NFR_HIP(hipMemsetAsync(w.cnt, 0, size_t(n) * sizeof(int), s));
  NFR_HIP(hipMemsetAsync(w.cursor, 0, size_t(n) * sizeof(int), s));
  const int64_t mc = quad_max_cells(n);
  NFR_HIP(hipMemsetAsync(w.gcnt, 0, size_t(mc) * sizeof(int), s));
  NFR_HIP(hipMemsetAsync(w.gcursor, 0, size_t(mc) * sizeof(int), s));
  const unsigned tb = (unsigned)ceil_div(ntri, kWG);
  hipLaunchKernelGGL(k_quad_centroids, dim3(tb), dim3(kWG), 0, s, xyz_dev, w.tri, ntri, w.cen, w.nrm_tri);
  hipLaunchKernelGGL(k_quad_proj, dim3(tb), dim3(kWG), 0, s, xyz_dev, w.tri, w.nbr, w.cen, w.nrm_tri, ntri,
                     projection, 1e8, proj);
  // k nearest nodes: bin the nodes into a grid, then search rings of cells
  const unsigned nbn = (unsigned)ceil_div(n, kWG);
  const int64_t nbc = ceil_div(mc, kWG);
  hipLaunchKernelGGL(k_quad_grid, dim3(1), dim3(kWG), 0, s, xyz_dev, n, mc, w.grid);
  hipLaunchKernelGGL(k_quad_bin_count, dim3(nbn), dim3(kWG), 0, s, xyz_dev, n, w.grid, w.gcnt);
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nbc), dim3(kWG), 0, s, w.gcnt, mc, w.gbsum);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kWG), 0, s, w.gbsum, nbc);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nbc), dim3(kWG), 0, s, w.gcnt, mc, w.gbsum, w.gstart);
  hipLaunchKernelGGL(k_quad_bin_fill, dim3(nbn), dim3(kWG), 0, s, xyz_dev, n, w.grid, w.gstart, w.gcursor, w.gnodes);
  hipLaunchKernelGGL(k_quad_knn, dim3((unsigned)ceil_div(ntri, kWG / 64)), dim3(kWG), 0, s, xyz_dev, w.grid, w.gcnt,
                     w.gstart, w.gnodes, w.cen, ntri, k, stn);
  const size_t lds = (size_t(k + 6) * (k + 7) + 2 * size_t(k)) * sizeof(double);
  hipLaunchKernelGGL(k_quad_elements, dim3((unsigned)ntri), dim3(64), lds, s, xyz_dev, nrm_dev, w.tri, w.cen,
                     w.nrm_tri, proj, stn, n, ntri, k, w.wE);
  const unsigned eb = (unsigned)ceil_div((int64_t)tk, kWG);
  const int64_t nb = ceil_div(n, kWG);
  hipLaunchKernelGGL(k_quad_count, dim3(eb), dim3(kWG), 0, s, stn, (int64_t)tk, n, w.cnt);
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kWG), 0, s, w.cnt, n, w.bsum);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kWG), 0, s, w.bsum, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kWG), 0, s, w.cnt, n, w.bsum, w.off);
  hipLaunchKernelGGL(k_quad_fill, dim3(eb), dim3(kWG), 0, s, stn, (int64_t)tk, n, w.off, w.cursor, w.list);
  hipLaunchKernelGGL(k_quad_sum, dim3((unsigned)nb), dim3(kWG), 0, s, w.off, w.cnt, n, w.list, w.wE, q_dev);
  NFR_HIP_LAUNCH();
  return NFR_OK;
}

}  // extern "C"

// ================================================================ autotuner

namespace {

constexpr int kTuneB[] = {2, 4, 16, 64, 256};
constexpr int64_t kTuneTargets[] = {256, 512, 1024, 2048, 4096};
constexpr int kTuneMaxSplit = 16;

std::vector<int64_t> tune_sizes(int64_t n_max) {
  std::vector<int64_t> out;
  for (int64_t d : {16, 4, 1}) {
    const int64_t n = std::max<int64_t>(1024, n_max / d);
    if (out.empty() || out.back() != n) out.push_back(n);
  }
  return out;
}

struct TuneLayout {
  size_t xyz = 0, q = 0, pack = 0, g = 0, part = 0, bytes = 0;
};

TuneLayout tune_layout(int64_t n_max, int B_max) {
  TuneLayout L;
  const int64_t npad = round_up(n_max, kPad);
  const int Bm = std::min(B_max, 256);
  size_t off = 0;
  L.xyz = off;
  off += align256(size_t(3) * n_max * sizeof(double));
  L.q = off;
  off += align256(size_t(n_max) * sizeof(double));
  L.pack = off;
  off += align256(nfr_problem_bytes(n_max));
  L.g = off;
  off += align256(size_t(npad) * Bm * sizeof(float));
  L.part = off;
  off += align256(size_t(kTuneMaxSplit) * Bm * npad * sizeof(double));
  L.bytes = off;
  return L;
}

bool tune_sizes_ok(int64_t n_max, int B_max) { return n_max >= 1024 && n_max <= kMaxN && B_max >= 2 && B_max <= kMaxB; }

void tune_install(const std::vector<TuneEntry>& add) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const TuneEntry& e : add) {
    bool replaced = false;
    for (TuneEntry& f : g_tune)
      if (f.npad == e.npad && f.B == e.B) {
        f.target = e.target;
        replaced = true;
      }
    if (!replaced) g_tune.push_back(e);
  }
}

// Integer value following "key": in text from position pos; -1 if absent.
long long json_int_after(const std::string& text, size_t pos, size_t end, const char* key) {
  const std::string k = std::string("\"") + key + "\"";
  const size_t at = text.find(k, pos);
  if (at == std::string::npos || at >= end) return -1;
  size_t c = text.find(':', at + k.size());
  if (c == std::string::npos || c >= end) return -1;
  ++c;
  while (c < end && (text[c] == ' ' || text[c] == '\t' || text[c] == '\n' || text[c] == '\r')) ++c;
  long long v = 0;
  bool any = false;
  while (c < end && text[c] >= '0' && text[c] <= '9') {
    v = v * 10 + (text[c] - '0');
    any = true;
    if (v > (1LL << 40)) return -1;
    ++c;
  }
  return any ? v : -1;
}

}  // namespace

extern "C" {

size_t nfr_tune_workspace_size(int64_t n_max, int B_max) {
  if (!tune_sizes_ok(n_max, B_max)) return 0;
  return tune_layout(n_max, B_max).bytes;
}

int nfr_tune(nfr_context* ctx, const char* cache_path, int64_t n_max, int B_max, void* ws_dev, size_t ws_bytes) {
  if (!ctx) return fail(NFR_ERR_INVALID_ARG, "context is NULL");
  if (!tune_sizes_ok(n_max, B_max))
    return fail(NFR_ERR_INVALID_ARG, "n_max = %lld, B_max = %d outside [1024, %lld] x [2, %d]", (long long)n_max, B_max,
                (long long)kMaxN, kMaxB);
  const TuneLayout L = tune_layout(n_max, B_max);
  if (!ws_dev || ws_bytes < L.bytes) return fail(NFR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.bytes);
  if (reinterpret_cast<uintptr_t>(ws_dev) % 256) return fail(NFR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  NFR_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  char* base = static_cast<char*>(ws_dev);
  double* xyz_dev = reinterpret_cast<double*>(base + L.xyz);
  double* q_dev = reinterpret_cast<double*>(base + L.q);
  float* g = reinterpret_cast<float*>(base + L.g);
  double* part = reinterpret_cast<double*>(base + L.part);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  NFR_HIP(hipEventCreate(&ev0));
  hipError_t e = hipEventCreate(&ev1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev0);
    return fail(NFR_ERR_HIP, "hipEventCreate failed: %s", hipGetErrorString(e));
  }
  struct Events {
    hipEvent_t a, b;
    ~Events() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } events{ev0, ev1};
  const nfr_kernel kern{NFR_KERNEL_GAUSS_MH, 1.0, 0.15, 0.5, 0.4};
  std::vector<TuneEntry> found;
  std::vector<double> found_ms;
  for (int64_t n : tune_sizes(n_max)) {
    // a synthetic surface: spherical Fibonacci nodes, equal weights
    std::vector<double> xyz(size_t(3) * n), q(size_t(n), 4.0 * M_PI / (double)n);
    const double golden = (1.0 + std::sqrt(5.0)) / 2.0;
    for (int64_t i = 0; i < n; ++i) {
      const double z = 1.0 - (2.0 * i + 1.0) / (double)n;
      const double r = std::sqrt(std::max(0.0, 1.0 - z * z));
      const double phi = 2.0 * M_PI * (double)i / golden;
      xyz[3 * i] = r * std::cos(phi);
      xyz[3 * i + 1] = r * std::sin(phi);
      xyz[3 * i + 2] = z;
    }
    NFR_HIP(hipMemcpyAsync(xyz_dev, xyz.data(), xyz.size() * sizeof(double), hipMemcpyHostToDevice, s));
    NFR_HIP(hipMemcpyAsync(q_dev, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice, s));
    NFR_HIP(hipStreamSynchronize(s));   // the host arrays go out of scope with this iteration
    nfr_problem* prob = nullptr;
    int st = nfr_problem_create(ctx, n, xyz_dev, q_dev, base + L.pack, nfr_problem_bytes(n), &prob);
    if (st) return st;
    struct ProbGuard {
      nfr_problem* p;
      ~ProbGuard() { nfr_problem_destroy(p); }
    } guard{prob};
    const ProblemView& pv = prob->view;
    const PairParams pp = pair_params(norm_kernel(kern), pv);
    for (int B : kTuneB) {
      if (B > B_max) break;
      NFR_HIP(hipMemsetAsync(g, 0, size_t(pv.npad) * B * sizeof(float), s));
      int64_t best_t = kTargetWGs;
      double best_ms = 1e300;
      int64_t last_split = -1;
      for (int64_t target : kTuneTargets) {
        const OtfPlan pl = plan_otf_target(pv.npad, B, target);
        if (pl.nsplit > kTuneMaxSplit || pl.nsplit == last_split) continue;   // same launch as the previous target
        last_split = pl.nsplit;
        launch_otf_kind<0>(pv, pp, B, g, part, pl, s);
        NFR_HIP(hipEventRecord(ev0, s));
        for (int r = 0; r < 3; ++r) launch_otf_kind<0>(pv, pp, B, g, part, pl, s);
        NFR_HIP(hipEventRecord(ev1, s));
        NFR_HIP_LAUNCH();
        NFR_HIP(hipEventSynchronize(ev1));
        float ms = 0.0f;
        NFR_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        if (ms / 3.0 < best_ms) {
          best_ms = ms / 3.0;
          best_t = target;
        }
      }
      found.push_back(TuneEntry{pv.npad, B, best_t});
      found_ms.push_back(best_ms);
    }
  }
  tune_install(found);
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "w");
    if (!f) return fail(NFR_ERR_INVALID_ARG, "cannot write %s", cache_path);
    std::fprintf(f, "{\"library\": \"nfr\", \"arch\": \"%s\", \"tuned\": \"multi-state on-the-fly pair sum, workgroup target\",\n \"entries\": [\n", ctx->arch);
    for (size_t i = 0; i < found.size(); ++i)
      std::fprintf(f, "  {\"npad\": %lld, \"B\": %d, \"target_wgs\": %lld, \"ms\": %.6f}%s\n", (long long)found[i].npad,
                   found[i].B, (long long)found[i].target, found_ms[i], i + 1 < found.size() ? "," : "");
    std::fprintf(f, " ]\n}\n");
    if (std::fclose(f) != 0) return fail(NFR_ERR_INVALID_ARG, "cannot write %s", cache_path);
  }
  return NFR_OK;
}

int nfr_tune_load(const char* cache_path) {
  if (!cache_path) return fail(NFR_ERR_INVALID_ARG, "cache_path is NULL");
  FILE* f = std::fopen(cache_path, "r");
  if (!f) return fail(NFR_ERR_INVALID_ARG, "cannot read %s", cache_path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  std::vector<TuneEntry> add;
  size_t pos = 0;
  while ((pos = text.find('{', pos + 1)) != std::string::npos) {
    const size_t end = text.find('}', pos);
    if (end == std::string::npos) break;
    if (text.find("\"npad\"", pos) >= end) continue;
    const long long npad = json_int_after(text, pos, end, "npad");
    const long long B = json_int_after(text, pos, end, "B");
    const long long t = json_int_after(text, pos, end, "target_wgs");
    if (npad < kPad || npad % kPad || npad > round_up(kMaxN, kPad) || B < 2 || B > kMaxB || t < 1 || t > (1 << 20))
      return fail(NFR_ERR_INVALID_ARG, "malformed tuning entry in %s", cache_path);
    add.push_back(TuneEntry{(int64_t)npad, (int)B, (int64_t)t});
  }
  if (add.empty()) return fail(NFR_ERR_INVALID_ARG, "no tuning entries in %s", cache_path);
  tune_install(add);
  return NFR_OK;
}

int64_t nfr_tune_target(int64_t n, int B) {
  if (n < 1 || n > kMaxN || B < 2 || B > kMaxB) return -1;
  return otf_target_wgs(round_up(n, kPad), B);
}

int nfr_tune_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  return NFR_OK;
}

}  // extern "C"
