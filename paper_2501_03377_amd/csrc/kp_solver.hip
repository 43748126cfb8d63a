// Plan, workspace and the PCG driver of the kpcg C ABI (include/kpcg.h).
//
// A plan is the preconditioner's initialisation (Algs. 4-5): closed-form
// eigenbases uploaded once.  A solve is Algorithm 1 enqueued on the plan's
// stream; the scalar recurrences stay on the device, and the host only reads
// the per-RHS done flags between chunks of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/kpcg.h"
#include "kp_common.h"
#include "kp_internal.h"

using namespace kp;

namespace kp {

// Per-plan launch timer: a begin and an end event around every traced launch
// on the plan's stream; elapsed times are folded into per-class totals once
// the stream has been synchronised.
struct Tracer {
  struct Rec { int cls; hipEvent_t a, b; bool pooled; };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  std::vector<Rec>* capture = nullptr;   // records of a graph being captured
  hipEvent_t cur = nullptr;
  double ms[KC_COUNT] = {};
  int64_t cnt[KC_COUNT] = {};

  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int, hipStream_t s) { cur = get(); (void)hipEventRecord(cur, s); }
  void end(int cls, hipStream_t s) {
    hipEvent_t e = get();
    (void)hipEventRecord(e, s);
    if (capture) capture->push_back({cls, cur, e, false});   // owned by the graph
    else pending.push_back({cls, cur, e, true});
    cur = nullptr;
  }
  void collect() {
    for (const Rec& r : pending) {
      float f = 0.f;
      if (hipEventElapsedTime(&f, r.a, r.b) == hipSuccess) {
        ms[r.cls] += f;
        cnt[r.cls] += 1;
      }
      if (r.pooled) {
        pool.push_back(r.a);
        pool.push_back(r.b);
      }
    }
    pending.clear();
  }
  void reset() {
    for (int c = 0; c < KC_COUNT; ++c) { ms[c] = 0.0; cnt[c] = 0; }
  }
  ~Tracer() {
    for (const Rec& r : pending)
      if (r.pooled) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

static thread_local Tracer* g_tracer = nullptr;
void trace_begin(int cls, hipStream_t s) { if (g_tracer) g_tracer->begin(cls, s); }
void trace_end(int cls, hipStream_t s) { if (g_tracer) g_tracer->end(cls, s); }

}  // namespace kp

struct kp_plan {
  Geom g;
  PinvOps op;
  int prec = 0;
  int max_batch = 1;
  hipStream_t stream = nullptr;
  int device = 0;
  void* resident = nullptr;
  size_t resident_bytes = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  double* hist = nullptr;       // residual history, pinned host memory mapped to the device
  double* hist_dev = nullptr;   // its device address
  size_t hist_cap = 0;          // doubles
  double* diag = nullptr;       // descriptors of the iterates (KP_FLAG_DIAGNOSTICS), mapped
  double* diag_dev = nullptr;   // like hist: [batch][hs][DIAG_RAW]
  size_t diag_cap = 0;          // doubles
  int diag_batch = 0;           // shape of the last solve's table (0: none)
  int diag_hs = 0;
  RhsState* st_host = nullptr;  // pinned, mapped mirror of the state (written by the device)
  RhsState* st_dev = nullptr;   // its device address
  int expect_iters = 0;         // iterations the last solve needed (first chunk size)
  bool expect_split = false;    // ... and whether it stopped before their last preconditioning
  bool profiling = false;
  Tracer tracer;
  hipStream_t own = nullptr;    // private stream of kp_solve (graph capture needs one)
  hipEvent_t ev_in = nullptr;   // orders kp_solve after earlier work on `stream`
  hipEvent_t ev_done = nullptr; // recorded after each enqueued chunk of a solve
  kp_ticket* busy = nullptr;    // the solve in flight (kp_solve_async), if any
  // Captured chunks of iterations, keyed by everything their kernels capture.
  struct GraphKey {
    int whole;          // 1: start, iterations and exit step; 0: iterations only
    int batch, n, flags, hs;
    double tol;
    const void* u;
    const void* hist;
    const void* diag;   // descriptor table (nullptr without KP_FLAG_DIAGNOSTICS)
    const void* eta;    // when the captured kernels read it, else nullptr
    bool operator==(const GraphKey& o) const {
      return whole == o.whole && batch == o.batch && n == o.n && flags == o.flags &&
             hs == o.hs && tol == o.tol && u == o.u && hist == o.hist && diag == o.diag &&
             eta == o.eta;
    }
  };
  struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    std::vector<Tracer::Rec> trace;   // event pairs recorded by every replay
  };
  std::vector<GraphEntry> graphs;     // most recently used last
  bool graphs_ok = true;              // cleared if capture is unavailable
  const void* last_eta = nullptr;     // buffers of the previous solve: when a solve
  const void* last_u = nullptr;       // repeats them, the whole solve is one graph
  int pc_kind = KP_PRECOND_PINV;      // preconditioner of kp_solve / kp_apply_preconditioner
  int jac_p = 3;                      // Jacobi(p, omega) parameters
  double jac_omega = 1.3;
  double* faces_dev = nullptr;        // boundary data of kp_assemble_rhs / kp_field
  size_t faces_cap = 0;               // doubles
  CertOps cert{};                     // low-mode error certificate (in `resident`)
  bool small_ok = false;              // FP64 2D plan small enough for the one-kernel solve
  SmallOps small{};                   // its full eigenbases (in `resident`)
  struct {                            // arguments of the last one-kernel solve
    const double* eta = nullptr;
    double* u = nullptr;
    int batch = 0, max_iter = 0, flags = 0;
    double tol = 0.0;
  } small_last;
  double* lr_dev = nullptr;           // G_r of the low-rank preconditioner, [ny][nx] (2D)
  int lr_rank = 0;                    // its rank (0: not built)
  struct {                            // continuous batch (the request server)
    bool open = false;
    const double* eta = nullptr;      // max_batch slots of eta and u, caller-owned
    double* u = nullptr;
    double tol = 0.0;
    int flags = 0;
  } slot;
};

namespace {
// Activates the plan's tracer on this thread for the lifetime of the guard.
struct TraceScope {
  Tracer* prev;
  explicit TraceScope(kp_plan* p) : prev(g_tracer) { g_tracer = p->profiling ? &p->tracer : nullptr; }
  ~TraceScope() { g_tracer = prev; }
};
}  // namespace

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

size_t elem_bytes(int prec) {
  return (prec == PREC_F64 || prec_int8(prec)) ? 8 : (prec == PREC_BF16 ? 2 : 4);
}

struct Layout {
  size_t R, P, W, Z, T0, T1, J, C1, C2, C3, part, st, total;
};

Layout layout_for(const kp_plan* p, int batch) {
  Layout L{};
  const size_t N = (size_t)p->g.N * (size_t)batch;
  const int G = vec_blocks(p->g.N, batch);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
  L.R = take(N * 8);
  L.P = take(N * 8);
  L.W = take(N * 8);
  L.Z = take(N * 8);
  L.T0 = take(N * elem_bytes(p->prec));
  L.T1 = take(N * elem_bytes(p->prec));
  L.J = p->pc_kind == KP_PRECOND_JACOBI ? take(N * 8) : 0;   // Jacobi ping-pong buffer
  // low-mode certificate: box coefficients after the x, y (and z) products
  const size_t rows1 = (size_t)(p->g.N / p->g.nx);
  const size_t nzp = p->g.dim == 3 ? (size_t)p->g.nz : 1;
  L.C1 = take((size_t)batch * rows1 * CERT_M * 8);
  L.C2 = take((size_t)batch * nzp * CERT_M * CERT_M * 8);
  L.C3 = take((size_t)batch * CERT_PARTS * 8);
  (void)G;
  L.part = take((size_t)batch * NSLOTS * 8192 * 8);   // GMAX partials per slot
  L.st = take((size_t)batch * sizeof(RhsState));
  L.total = off;
  return L;
}

}  // namespace

// Serialises graph capture against the calls that invalidate a capture in
// progress on another host thread (device and pinned allocations and frees,
// synchronous copies, stream, event and graph creation and destruction).
// Shared with the request server, whose worker threads solve concurrently.
namespace kp {
std::mutex& api_mutex() {
  static std::mutex m;
  return m;
}
}  // namespace kp
using kp::api_mutex;

namespace {

// The HIP call behind the last KP_EHIP (or KP_ENOMEM from an allocation) of
// this host thread, for kp_last_error.
thread_local char t_last_error[256] = "";

bool ok_at(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  snprintf(t_last_error, sizeof t_last_error, "%s: %s (%d)", what, hipGetErrorName(e), (int)e);
  return false;
}
#define ok(e) ok_at((e), #e)

int ensure_workspace(kp_plan* p) {
  if (p->ws) return KP_OK;
  const size_t need = layout_for(p, p->max_batch).total;
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(api_mutex());
    if (!ok(hipMalloc(&ptr, need))) return KP_ENOMEM;
  }
  p->ws = ptr;
  p->ws_bytes = need;
  p->ws_owned = true;
  return KP_OK;
}

// Pinned host memory that the device writes directly (residual history,
// descriptor table), so reading it needs no copy kernel.
int ensure_mapped(double** host, double** dev, size_t* cap, size_t doubles) {
  if (*cap >= doubles) return KP_OK;
  std::lock_guard<std::mutex> lk(api_mutex());
  if (*host) (void)hipHostFree(*host);
  *host = nullptr;
  *dev = nullptr;
  *cap = 0;
  if (!ok(hipHostMalloc((void**)host, doubles * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent)))
    return KP_ENOMEM;
  if (!ok(hipHostGetDevicePointer((void**)dev, *host, 0))) return KP_EHIP;
  *cap = doubles;
  return KP_OK;
}

int ensure_hist(kp_plan* p, size_t doubles) {
  return ensure_mapped(&p->hist, &p->hist_dev, &p->hist_cap, doubles);
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + bytes && y < x + bytes;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Z = M(R).  In a solve (`part` given) the FP64 and int8 split
// pseudoinverse also leaves the partial sums of the CG step after it, <R, Z>
// and ||Z||^2 by Parseval in the eigenbasis, and returns how many there are;
// 0 means the step computes them itself in FP64 from R and Z (other
// preconditioners, the FP32 and BF16 products, and the flexible beta, which
// needs <W, Z>).  Returns Gdot > 0 when the pseudoinverse left the partial sums
// of <R, Z> and ||Z||^2 (spectral, Gdot blocks) -- then Z has zero mean and,
// if `z0` is given, the result goes to z0 instead of Z (the first
// application writes P_0 = Z_0 directly).
// h_fold (the first application of a solve whose eta is R_0, int8 split
// pseudoinverse): the first product also leaves eta's sums in the S_SUM and
// S_SQ slots, and ||eta||^2 is finished from them before the second product
// (in place of a pass over eta before the application).
struct HFold {
  RhsState* st;
  double* hist;
  int hist_stride;
};

int precondition(kp_plan* p, const Layout& L, const double* R, double* Z, int batch, int flags,
                 const RhsState* st, hipStream_t s, double* part = nullptr,
                 double* z0 = nullptr, const HFold* h_fold = nullptr) {
  char* base = (char*)p->ws;
  if (flags & KP_FLAG_NO_PRECOND) {
    launch_copy(p->g, R, Z, st, batch, vec_blocks(p->g.N, batch), s);
    return 0;
  }
  if (p->pc_kind == KP_PRECOND_JACOBI) {
    launch_jacobi(p->g, R, Z, (double*)(base + L.J), p->jac_p, p->jac_omega, st, batch,
                  vec_blocks(p->g.N, batch), s);
    return 0;
  }
  PinvOps op = p->op;
  int Gdot = 0;
  if (p->pc_kind == KP_PRECOND_LOWRANK) {
    op.gtab = p->lr_dev;
  } else if (part && st && !(flags & KP_FLAG_FLEX_BETA) &&
             (p->prec == PREC_F64 || prec_int8(p->prec))) {
    // <R, Z> by Parseval from the coefficients in the eigenbasis, which are
    // FP64-accurate only for the FP64 and the int8 split products; the FP32
    // and BF16 forms take the inner products in FP64 from R and Z in space
    const int b = pinv_ghat_blocks(op);
    if (b <= GMAX) {
      op.rpart = part;
      Gdot = b;
    }
  }
  double* out = (Gdot > 0 && z0) ? z0 : Z;
  if (h_fold && part) {
    op.hpart = part;
    pinv_step(op, 0, R, out, base + L.T0, base + L.T1, batch, st, s);
    op.hpart = nullptr;
    launch_fin_h(p->g, part, h_fold->st, h_fold->hist, h_fold->hist_stride, batch,
                 pinv_first_blocks(op), s);
    for (int q = 1; q < 2 * op.dim; ++q)
      pinv_step(op, q, R, out, base + L.T0, base + L.T1, batch, st, s);
    return Gdot;
  }
  pinv_apply(op, R, out, base + L.T0, base + L.T1, batch, st, s);
  return Gdot;
}

// Checks host boundary data [batch][dim][2] (finite; zero on periodic axes)
// and copies it to the plan's device buffer, ordered on the plan's stream.
int stage_faces(kp_plan* p, const double* faces, int batch, const double** out) {
  const int dim = p->g.dim;
  const size_t n = (size_t)batch * dim * 2;
  for (int b = 0; b < batch; ++b)
    for (int a = 0; a < dim; ++a)
      for (int e = 0; e < 2; ++e) {
        const double v = faces[((size_t)b * dim + a) * 2 + e];
        if (!std::isfinite(v) || (p->g.bc[a] == BC_P && v != 0.0)) return KP_EINVAL;
      }
  if (p->faces_cap < n) {
    std::lock_guard<std::mutex> lk(api_mutex());
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->faces_dev) (void)hipFree(p->faces_dev);
    p->faces_dev = nullptr;
    p->faces_cap = 0;
    if (!ok(hipMalloc((void**)&p->faces_dev, n * sizeof(double)))) return KP_ENOMEM;
    p->faces_cap = n;
  }
  if (!ok(hipMemcpyAsync(p->faces_dev, faces, n * sizeof(double), hipMemcpyHostToDevice,
                         p->stream)) ||
      !ok(hipStreamSynchronize(p->stream)))
    return KP_EHIP;
  *out = p->faces_dev;
  return KP_OK;
}

void clear_graphs(kp_plan* p) {
  std::lock_guard<std::mutex> lk(api_mutex());
  for (auto& e : p->graphs) (void)hipGraphExecDestroy(e.exec);
  p->graphs.clear();
}

}  // namespace

// Device scratch of kp_apply_pinv_noalloc, for callers that cannot allocate:
// the two intermediate grids of the mode products.  Each device the library
// runs on holds its own copy, at its own address, until the process ends.
// In host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[KP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kScratchDevices = 64;
char* g_scratch[kScratchDevices] = {};   // per device: address of its `scratch`

// The current device's copy of `scratch` (dev must be current).
int noalloc_scratch(int dev, char** out) {
  if (dev < 0 || dev >= kScratchDevices) return KP_EINVAL;
  std::lock_guard<std::mutex> lk(api_mutex());
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (!ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)))) return KP_EHIP;
    if (!ptr) return KP_EHIP;
    g_scratch[dev] = (char*)ptr;
  }
  *out = g_scratch[dev];
  return KP_OK;
}

}  // namespace

// A solve in flight: the host side of Algorithm 1's outer loop.  The first
// chunk of iterations (and the exit step) is enqueued at the start; the
// host then reads the per-RHS done flags once the chunk has finished and
// enqueues one more iteration (and the exit step again) while some
// right-hand side still runs.  kp_solve drives it to the end; kp_solve_async
// returns after the start and kp_poll / kp_wait advance it.
struct kp_ticket {
  kp_plan* p = nullptr;
  const double* eta = nullptr;
  double* u = nullptr;
  int batch = 0, max_iter = 0, flags = 0, hs = 0;
  double tol = 0.0;
  kp_result* results = nullptr;
  double* res_hist = nullptr;
  bool diag = false, cert = false, warm = false, small = false;
  int done_iters = 0;
  bool pending_tail = false;   // second part of a split iteration still owed
  bool finished = false;
  int status = KP_OK;
};

namespace {

// Argument checks shared by kp_solve and kp_solve_async; returns the flags
// the solve runs with (or a negative status).
int solve_flags(kp_plan* p, const double* eta, double* u, int batch, double tol, int max_iter,
                int flags) {
  if (!p || !eta || !u || batch < 1 || batch > p->max_batch) return KP_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol) || max_iter < 1 || max_iter > 1000000) return KP_EINVAL;
  if (flags & ~(KP_FLAG_NO_PRECOND | KP_FLAG_FLEX_BETA | KP_FLAG_RESIDUAL_ONLY | KP_FLAG_NO_GRAPH |
                KP_FLAG_DIAGNOSTICS | KP_FLAG_ANORM_STOP | KP_FLAG_WARM_START))
    return KP_EINVAL;
  if (!aligned16(eta) || !aligned16(u)) return KP_EINVAL;
  const size_t vbytes = (size_t)p->g.N * batch * 8;
  if (overlap(eta, u, vbytes)) return KP_EINVAL;
  // With M = I the preconditioned residual is R itself, which is no error
  // estimate: stop on the residual alone.
  if (flags & KP_FLAG_NO_PRECOND) flags |= KP_FLAG_RESIDUAL_ONLY;
  // Jacobi(p, omega) approximates L^{-1} too loosely for M(R) to estimate
  // the error either
  if (p->pc_kind == KP_PRECOND_JACOBI || p->pc_kind == KP_PRECOND_LOWRANK)
    flags |= KP_FLAG_RESIDUAL_ONLY;
  // the low-mode certificate backs the residual test unless the error test
  // is off
  if (!(flags & (KP_FLAG_RESIDUAL_ONLY | KP_FLAG_ANORM_STOP))) flags |= F_CERT;
  return flags;
}

// The launches of one solve on the plan's private stream.
struct SolveRun {
  kp_ticket* t;
  kp_plan* p;
  Layout L;
  char* base;
  double *R, *P, *W, *Z, *part;
  RhsState* st;
  int G;
  hipStream_t s;
  double* diag_dev;
  const double* R0;

  // layout_batch: the batch the workspace is laid out for when it differs
  // from the batch launched over (a continuous batch's first slots)
  explicit SolveRun(kp_ticket* t_, int layout_batch = 0) : t(t_), p(t_->p) {
    L = layout_for(p, layout_batch ? layout_batch : t->batch);
    base = (char*)p->ws;
    R = (double*)(base + L.R);
    P = (double*)(base + L.P);
    W = (double*)(base + L.W);
    Z = (double*)(base + L.Z);
    part = (double*)(base + L.part);
    st = (RhsState*)(base + L.st);
    G = vec_blocks(p->g.N, t->batch);
    s = p->own;
    diag_dev = t->diag ? p->diag_dev : nullptr;
    // Algorithm 1 from U_0 = 0 has R_0 = eta_c: a nonsingular set reads eta
    // itself where R_0 is needed (the first application and the first U/R
    // update, which stores R_1 in R); a warm start stores eta_c - L U_0
    R0 = (p->g.singular || t->warm) ? R : t->eta;
  }
  // ||eta||^2 taken by the first product of the first application: the int8
  // splits read eta itself there (a nonsingular set from U_0 = 0) and apply
  // no input scale, so nothing before that product needs it
  bool fold_h() const {
    if (!prec_int8(p->prec) || p->pc_kind != KP_PRECOND_PINV || p->g.singular || t->warm ||
        t->diag || (t->flags & KP_FLAG_NO_PRECOND))
      return false;
    const int b = pinv_first_blocks(p->op);
    return b > 0 && b <= GMAX;
  }
  // R_0, Z_0 = M(R_0), rho_0, P_0 = Z_0
  void head() {
    const bool fold = fold_h();
    // U_0 = 0 is stored only for the descriptors of iterate 0; R_0 = eta_c
    // only for a singular set started from zero
    launch_init(p->g, t->eta, (p->g.singular && !t->warm) ? R : nullptr,
                (t->diag && !t->warm) ? t->u : nullptr, part, st, p->hist_dev, t->hs, t->batch,
                G, s, 0, fold);
    if (t->warm)
      launch_warm(p->g, t->eta, t->u, R, part, st, p->hist_dev, t->hs, t->batch, t->tol,
                  t->flags, s);
    if (t->diag) launch_diag(p->g, t->eta, t->u, part, st, diag_dev, t->hs, t->batch, s);
    // spectral sums: Z_0 has zero mean, so P_0 = Z_0 is written by the
    // application itself and the P update is skipped
    const HFold hf{st, p->hist_dev, t->hs};
    const int Gdot = precondition(p, L, R0, Z, t->batch, t->flags, st, s, part, P,
                                  fold ? &hf : nullptr);
    launch_after_pinv(p->g, R0, Z, W, P, part, st, t->batch, G, 1, t->tol, t->flags, s, Gdot,
                      Gdot > 0);
  }
  // An iteration in two parts: up to the residual test and certificate,
  // then preconditioning and the updates that depend on it.  with_cert: the
  // low-mode certificate runs after this iteration's residual test (only
  // the last iteration of a chunk, where the solve is expected to stop;
  // earlier ones fall back to the error estimate after the next
  // application, and their launches are saved)
  void iteration_head(bool first_iter, bool with_cert) {
    const bool u0 = first_iter && !t->warm;
    launch_iter_head(p->g, P, W, R, t->u, part, st, p->hist_dev, t->hs, t->batch, G, t->tol,
                     t->flags, s, (u0 && !p->g.singular) ? t->eta : nullptr, u0);
    if (t->diag) launch_diag(p->g, t->eta, t->u, part, st, diag_dev, t->hs, t->batch, s);
    if (t->cert && with_cert)
      launch_cert(p->g, p->cert, R, (double*)(base + L.C1), (double*)(base + L.C2),
                  (double*)(base + L.C3), st, t->batch, t->tol, s);
  }
  void iteration_tail() {
    const int Gdot = precondition(p, L, R, Z, t->batch, t->flags, st, s, part);
    launch_after_pinv(p->g, R, Z, W, P, part, st, t->batch, G, 0, t->tol, t->flags, s, Gdot);
  }
  // n iterations; with `split` the last one stops after its residual test
  // (its second part runs later, only if some right-hand side continues);
  // `from_start`: the first of them is the solve's first iteration
  void iterations(int n, bool split, bool from_start) {
    for (int q = 0; q < n; ++q) {
      iteration_head(from_start && q == 0, q == n - 1);
      if (!(split && q == n - 1)) iteration_tail();
    }
  }
  // exit step: true residual, centering of U, state to the mapped host mirror
  void tail() {
    launch_finish(p->g, t->eta, t->u, part, st, p->st_dev, t->batch, G, s);
  }
  // Finds or captures the graph of `key`; returns its index or -1.
  template <class F>
  int graph_for(const kp_plan::GraphKey& key, F&& body) {
    for (size_t e = 0; e < p->graphs.size(); ++e)
      if (p->graphs[e].key == key) {
        std::rotate(p->graphs.begin() + e, p->graphs.begin() + e + 1, p->graphs.end());
        return (int)p->graphs.size() - 1;
      }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::lock_guard<std::mutex> lk(api_mutex());
    bool okc = ok(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    if (okc) {
      body();
      okc = ok(hipStreamEndCapture(s, &graph)) && graph != nullptr;
    }
    if (okc) okc = ok(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!okc) {
      p->graphs_ok = false;   // capture unavailable: launch directly from now on
      return -1;
    }
    if (p->graphs.size() >= 8) {
      (void)hipGraphExecDestroy(p->graphs.front().exec);
      p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back({key, exec, {}});
    return (int)p->graphs.size() - 1;
  }
};

// Validates, prepares and enqueues the start of a solve: the first chunk of
// iterations (what the previous solve on this plan needed, or a guess per
// precision) and the exit step, as one captured HIP graph where possible
// (cached per plan; when the caller repeats the previous solve's buffers the
// whole solve -- start, chunk and exit step -- is one graph).  Small 2D
// problems with the FP64 pseudoinverse run the whole solve as one kernel.
int solve_start(kp_ticket* t, kp_plan* p, const double* eta, double* u, int batch, double tol,
                int max_iter, int flags, kp_result* results, double* res_hist) {
  flags = solve_flags(p, eta, u, batch, tol, max_iter, flags);
  if (flags < 0) return flags;
  int rc = ensure_workspace(p);
  if (rc != KP_OK) return rc;
  const int hs = max_iter + 1;
  rc = ensure_hist(p, (size_t)batch * hs);
  if (rc != KP_OK) return rc;
  const bool diag = (flags & KP_FLAG_DIAGNOSTICS) != 0;
  p->diag_batch = 0;
  if (diag) {
    rc = ensure_mapped(&p->diag, &p->diag_dev, &p->diag_cap, (size_t)batch * hs * DIAG_RAW);
    if (rc != KP_OK) return rc;
  }
  (void)hipGetLastError();
  t->p = p;
  t->eta = eta;
  t->u = u;
  t->batch = batch;
  t->tol = tol;
  t->max_iter = max_iter;
  t->flags = flags;
  t->hs = hs;
  t->results = results;
  t->res_hist = res_hist;
  t->diag = diag;
  t->cert = (flags & F_CERT) != 0;
  t->warm = (flags & KP_FLAG_WARM_START) != 0;
  // Work runs on the plan's private stream, ordered after earlier work on the
  // caller's stream.
  hipStream_t s = p->own;
  if (!ok(hipEventRecord(p->ev_in, p->stream)) || !ok(hipStreamWaitEvent(s, p->ev_in, 0)))
    return KP_EHIP;

  TraceScope scope(p);
  std::memset(p->hist, 0, (size_t)batch * hs * sizeof(double));   // no kernel writes it now
  if (diag) {
    std::fill(p->diag, p->diag + (size_t)batch * hs * DIAG_RAW,
              std::numeric_limits<double>::quiet_NaN());
    p->diag_batch = batch;
    p->diag_hs = hs;
  }
  SolveRun run(t);
  // Small 2D problems with the FP64 pseudoinverse: the whole solve is one
  // kernel (the same stopping rules, without the low-mode certificate).
  t->small = p->small_ok && p->pc_kind == KP_PRECOND_PINV && !diag &&
             !(flags & (KP_FLAG_NO_PRECOND | KP_FLAG_FLEX_BETA | KP_FLAG_ANORM_STOP |
                        KP_FLAG_WARM_START));
  if (t->small) {
    p->small_last.eta = eta;
    p->small_last.u = u;
    p->small_last.batch = batch;
    p->small_last.max_iter = max_iter;
    p->small_last.flags = flags;
    p->small_last.tol = tol;
    launch_small_solve(p->g, p->small, eta, u, run.st, p->st_dev, p->hist_dev, hs, batch, tol,
                       max_iter, flags, s);
    t->done_iters = max_iter;
  } else {
    const bool use_graphs = p->graphs_ok && !p->profiling && !(flags & KP_FLAG_NO_GRAPH);
    const bool repeat = eta == p->last_eta && u == p->last_u;
    p->last_eta = eta;
    p->last_u = u;
    const int chunk = p->expect_iters > 0
                          ? p->expect_iters
                          : ((flags & KP_FLAG_NO_PRECOND)
                                 ? 8
                                 : ((p->prec == PREC_F64 || prec_int8(p->prec))
                                        ? 1
                                        : (p->prec == PREC_BF16 ? 8 : 2)));
    // a first chunk that ends where the previous solve stopped, before the
    // last preconditioning, launches no kernels for finished right-hand sides
    const int n = std::min(chunk, max_iter);
    const bool split = p->expect_iters > 0 && p->expect_split && n == chunk;
    const int nkey = 2 * n + (split ? 1 : 0);
    bool launched = false;
    if (use_graphs) {
      if (repeat) {
        const kp_plan::GraphKey key{1, batch, nkey, flags, hs, tol, u, p->hist_dev, run.diag_dev,
                                    eta};
        const int gi = run.graph_for(key, [&]() {
          run.head();
          run.iterations(n, split, true);
          run.tail();
        });
        if (gi >= 0) {
          if (!ok(hipGraphLaunch(p->graphs[gi].exec, s))) return KP_EHIP;
          launched = true;
        }
      } else {
        run.head();
        // (the iterations read eta for the descriptors, and as R_0 of a
        // nonsingular set in the first U/R update)
        const bool reads_eta = diag || (!p->g.singular && !t->warm);
        const kp_plan::GraphKey key{0,   batch, nkey,         flags,
                                    hs,  tol,   u,            p->hist_dev,
                                    run.diag_dev, reads_eta ? eta : nullptr};
        const int gi = run.graph_for(key, [&]() { run.iterations(n, split, true); });
        if (gi >= 0) {
          if (!ok(hipGraphLaunch(p->graphs[gi].exec, s))) return KP_EHIP;
        } else {
          run.iterations(n, split, true);
        }
        run.tail();
        launched = true;
      }
    }
    if (!launched) {
      run.head();
      run.iterations(n, split, true);
      run.tail();
    }
    t->pending_tail = split;
    t->done_iters = n;
  }
  if (!ok(hipGetLastError()) || !ok(hipEventRecord(p->ev_done, s))) return KP_EHIP;
  return KP_OK;
}

// Per-RHS statuses and results of a finished solve; the first chunk of the
// next solve on this plan is sized by this one.
void solve_finish(kp_ticket* t) {
  kp_plan* p = t->p;
  const int batch = t->batch;
  if (t->res_hist) std::memcpy(t->res_hist, p->hist, (size_t)batch * t->hs * sizeof(double));
  int worst = KP_OK;
  int max_it = 0;
  for (int b = 0; b < batch; ++b) {
    const RhsState& x = p->st_host[b];
    int stt;
    switch (x.done) {
      case CONVERGED: case ZERO_RHS: stt = KP_OK; break;
      case BREAKDOWN: stt = KP_EBREAKDOWN; break;
      case NONFINITE: stt = KP_ENONFINITE; break;
      default: stt = KP_NOT_CONVERGED; break;
    }
    if (t->results) {
      kp_result& r = t->results[b];
      r.status = stt;
      r.iterations = x.iter;
      r.pinv_applications = x.pinv_count;
      r.reserved = 0;
      r.rel_res = x.rel_res;
      r.true_rel_res = x.true_rel_res;
      r.err_est = x.err_est;
      r.removed_mean = x.mean;
    }
    if (stt < 0 && (worst >= 0 || stt < worst)) worst = stt;
    else if (stt == KP_NOT_CONVERGED && worst == KP_OK) worst = stt;
    if (stt == KP_OK) max_it = std::max(max_it, x.iter);
  }
  if (max_it > 0) {
    p->expect_iters = max_it;
    // split next time if every right-hand side that took max_it iterations
    // stopped before preconditioning in its last one
    bool split = true;
    for (int b = 0; b < batch; ++b) {
      const RhsState& x = p->st_host[b];
      if (x.done == CONVERGED && x.iter == max_it && x.pinv_count > x.iter) split = false;
    }
    p->expect_split = split;
  }
  t->status = worst;
  t->finished = true;
}

// Advances a solve: once its last enqueued chunk has finished (waiting for
// it with `block`, else returning 0 while it runs), either finishes it or
// enqueues one more iteration and the exit step.  Returns 1 when finished.
int solve_advance(kp_ticket* t, bool block) {
  if (t->finished) return 1;
  kp_plan* p = t->p;
  for (;;) {
    if (block) {
      if (!ok(hipEventSynchronize(p->ev_done))) {
        t->status = KP_EHIP;
        t->finished = true;
        return 1;
      }
    } else {
      const hipError_t q = hipEventQuery(p->ev_done);
      if (q == hipErrorNotReady) return 0;
      if (!ok_at(q, "hipEventQuery")) {
        t->status = KP_EHIP;
        t->finished = true;
        return 1;
      }
    }
    if (p->profiling) p->tracer.collect();
    bool all_done = true;
    for (int b = 0; b < t->batch; ++b) all_done = all_done && p->st_host[b].done != RUNNING;
    if (all_done || t->done_iters >= t->max_iter) {
      solve_finish(t);
      return 1;
    }
    TraceScope scope(p);
    SolveRun run(t);
    if (t->pending_tail) run.iteration_tail();
    run.iterations(1, false, false);
    run.tail();
    t->pending_tail = false;
    t->done_iters += 1;
    if (!ok(hipGetLastError()) || !ok(hipEventRecord(p->ev_done, p->own))) {
      t->status = KP_EHIP;
      t->finished = true;
      return 1;
    }
    if (!block) return 0;
  }
}

}  // namespace

// ------------------------------------------------- continuous batches ----
// The request server keeps one batch of max_batch slots running on a plan:
// every slot is a right-hand side at its own stage of Algorithm 1 (or empty).
// A step is the start (R_0, Z_0, rho_0, P_0) for slots that joined since the
// last step, then one or more iterations for the running slots, then the
// exit step (true residual, centring) for slots whose solve ended in it (a
// slot that ends early in a step is skipped by the rest of it).  All of it
// is the same arithmetic per right-hand side as kp_solve's, with the
// low-mode certificate tried in every iteration, so a slot's result does not
// depend on the other slots, on when it joined, on the slot it took or on
// how the iterations were grouped into steps.
namespace kp {

int slots_open(kp_plan* p, const double* eta, double* u, double tol, int flags) {
  if (!p || !eta || !u || !(tol > 0.0) || p->busy) return KP_EINVAL;
  // (small 2D plans run the general kernels here too, not the one-kernel solve)
  if (p->pc_kind != KP_PRECOND_PINV) return KP_EINVAL;
  if (flags & ~(KP_FLAG_NO_PRECOND | KP_FLAG_FLEX_BETA | KP_FLAG_RESIDUAL_ONLY)) return KP_EINVAL;
  int rc = ensure_workspace(p);
  if (rc != KP_OK) return rc;
  if (flags & KP_FLAG_NO_PRECOND) flags |= KP_FLAG_RESIDUAL_ONLY;
  if (!(flags & KP_FLAG_RESIDUAL_ONLY)) flags |= F_CERT;
  p->slot.open = true;
  p->slot.eta = eta;
  p->slot.u = u;
  p->slot.tol = tol;
  p->slot.flags = flags;
  const Layout L = layout_for(p, p->max_batch);
  (void)hipGetLastError();
  launch_slot_set((RhsState*)((char*)p->ws + L.st), p->max_batch, -1, IDLE, p->stream);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

int slots_mark(kp_plan* p, int slot, int code) {
  if (!p || !p->slot.open || slot < 0 || slot >= p->max_batch) return KP_EINVAL;
  const Layout L = layout_for(p, p->max_batch);
  launch_slot_set((RhsState*)((char*)p->ws + L.st), p->max_batch, slot, code, p->stream);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

// Enqueues one step on the plan's private stream after the plan's stream
// (where the slots' right-hand sides were staged and marked), as one
// captured graph where possible.
int slots_step(kp_plan* p, int iters, int nslots) {
  if (!p || !p->slot.open || iters < 1 || iters > 8 || nslots < 0 || nslots > p->max_batch)
    return KP_EINVAL;
  kp_ticket t;
  t.p = p;
  t.eta = p->slot.eta;
  t.u = p->slot.u;
  t.batch = nslots ? nslots : p->max_batch;   // slots past it are left as they are
  t.tol = p->slot.tol;
  t.flags = p->slot.flags;
  t.hs = 1;
  t.cert = (t.flags & F_CERT) != 0;
  SolveRun run(&t, p->max_batch);   // the slots' states sit in the max_batch layout
  run.R0 = run.R;   // every slot's R_0 = eta_c is stored
  auto body = [&]() {
    launch_init(p->g, t.eta, run.R, nullptr, run.part, run.st, nullptr, 0, t.batch, run.G,
                run.s, 1);
    for (int i = 0; i < iters; ++i) {
      launch_iter_head(p->g, run.P, run.W, run.R, t.u, run.part, run.st, nullptr, 0, t.batch,
                       run.G, t.tol, t.flags, run.s, nullptr, false);
      if (t.cert)
        launch_cert(p->g, p->cert, run.R, (double*)(run.base + run.L.C1),
                    (double*)(run.base + run.L.C2), (double*)(run.base + run.L.C3), run.st,
                    t.batch, t.tol, run.s);
      const int Gdot = precondition(p, run.L, run.R, run.Z, t.batch, t.flags, run.st, run.s,
                                    run.part);
      launch_after_pinv(p->g, run.R, run.Z, run.W, run.P, run.part, run.st, t.batch, run.G, 0,
                        t.tol, t.flags, run.s, Gdot, false);
    }
    launch_finish(p->g, t.eta, t.u, run.part, run.st, p->st_dev, t.batch, run.G, run.s, 1);
  };
  (void)hipGetLastError();
  if (!ok(hipEventRecord(p->ev_in, p->stream)) || !ok(hipStreamWaitEvent(run.s, p->ev_in, 0)))
    return KP_EHIP;
  TraceScope scope(p);
  bool launched = false;
  if (p->graphs_ok && !p->profiling) {
    const kp_plan::GraphKey key{2, t.batch, iters, t.flags, 1, t.tol, t.u, nullptr, nullptr,
                                t.eta};
    const int gi = run.graph_for(key, body);
    if (gi >= 0) {
      if (!ok(hipGraphLaunch(p->graphs[gi].exec, run.s))) return KP_EHIP;
      launched = true;
    }
  }
  if (!launched) body();
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

// Waits for the last step; the slots' states (max_batch entries) are then
// in the host mirror.
const RhsState* slots_wait(kp_plan* p) {
  if (!p || !p->slot.open) return nullptr;
  if (!ok(hipStreamSynchronize(p->own))) return nullptr;
  if (p->profiling) p->tracer.collect();
  return p->st_host;
}

void slots_close(kp_plan* p) {
  if (p) p->slot.open = false;
}

}  // namespace kp

extern "C" {

int kp_basis_1d(int n, int bc, double* Q, double* lambda) {
  if (n < 3 || bc < 0 || bc > 4 || !Q || !lambda) return KP_EINVAL;
  return basis_1d(n, bc, Q, lambda) == 0 ? KP_OK : KP_EINVAL;
}

int kp_plan_create(kp_plan** out, int nx, int ny, int nz, const int bc[3], int prec,
                   int max_batch, void* hip_stream) {
  if (!out || !bc) return KP_EINVAL;
  *out = nullptr;
  if (nx < 3 || ny < 3 || !(nz >= 3 || nz == 1)) return KP_EINVAL;
  if (prec < PREC_F64 || prec > PREC_I8X6 || max_batch < 1) return KP_EINVAL;
  const int dim = nz == 1 ? 2 : 3;
  for (int a = 0; a < dim; ++a)
    if (bc[a] < 0 || bc[a] > 4) return KP_EINVAL;
  // the int8 split products digitise 16 values per lane along every axis
  if (prec_int8(prec)) {
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < dim; ++a)
      if (n[a] % 16 != 0 || n[a] > 512) return KP_EINVAL;
  }
  const int64_t N = (int64_t)nx * ny * nz;
  if (N >= ((int64_t)1 << 31)) return KP_EINVAL;
  if (max_batch > 65535) return KP_EINVAL;

  kp_plan* p = new (std::nothrow) kp_plan();
  if (!p) return KP_ENOMEM;
  p->g.nx = nx; p->g.ny = ny; p->g.nz = nz; p->g.dim = dim; p->g.N = N;
  p->g.bc[0] = bc[0]; p->g.bc[1] = bc[1]; p->g.bc[2] = dim == 3 ? bc[2] : KP_BC_D;
  bool singular = true;
  for (int a = 0; a < dim; ++a) singular = singular && (bc[a] == KP_BC_P || bc[a] == KP_BC_N);
  p->g.singular = singular ? 1 : 0;
  if (!zgrid_fits(p->g)) { delete p; return KP_EINVAL; }
  p->prec = prec;
  p->max_batch = max_batch;
  p->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&p->device);

  // Host bases (closed form), packed per axis for the forward (B = V) and the
  // backward (B = V^T) mode products.
  const int n[3] = {nx, ny, nz};
  size_t bytes = 0;
  size_t offF[3] = {0, 0, 0}, offB[3] = {0, 0, 0}, offL[3] = {0, 0, 0};
  size_t offV[3] = {0, 0, 0};
  for (int a = 0; a < dim; ++a) {
    const size_t pb = mp_packed_bytes(n[a], prec);
    offF[a] = bytes; bytes += align_up(pb);
    offB[a] = bytes; bytes += align_up(pb);
    offL[a] = bytes; bytes += align_up((size_t)n[a] * 8);
    offV[a] = bytes; bytes += align_up((size_t)n[a] * CERT_M * 8);
  }
  const size_t offW = bytes;
  bytes += align_up((size_t)CERT_M * CERT_M * CERT_M * 8);
  // full FP64 eigenbases and their transposes for the one-kernel solve of
  // small 2D problems
  const bool small = prec == PREC_F64 && small_solve_fits(p->g);
  size_t offQ[2] = {0, 0}, offQt[2] = {0, 0};
  if (small)
    for (int a = 0; a < 2; ++a) {
      offQ[a] = bytes;
      bytes += align_up((size_t)n[a] * n[a] * 8);
      offQt[a] = bytes;
      bytes += align_up((size_t)n[a] * n[a] * 8);
    }
  std::vector<double> lam_axis[3];
  std::vector<char> host(bytes, 0);
  double lam0[3] = {0.0, 0.0, 0.0}, lam1[3] = {INFINITY, INFINITY, INFINITY};
  for (int a = 0; a < dim; ++a) {
    const int na = n[a];
    std::vector<double> Q((size_t)na * na), Qt((size_t)na * na), lam(na);
    if (basis_1d(na, p->g.bc[a], Q.data(), lam.data()) != 0) { delete p; return KP_EINVAL; }
    for (int r = 0; r < na; ++r)
      for (int c = 0; c < na; ++c) Qt[(size_t)c * na + r] = Q[(size_t)r * na + c];
    mp_pack(Q.data(), na, prec, host.data() + offF[a]);
    mp_pack(Qt.data(), na, prec, host.data() + offB[a]);
    std::memcpy(host.data() + offL[a], lam.data(), (size_t)na * 8);
    if (small) {
      std::memcpy(host.data() + offQ[a], Q.data(), (size_t)na * na * 8);
      std::memcpy(host.data() + offQt[a], Qt.data(), (size_t)na * na * 8);
    }
    // the m_a lowest eigenvectors (columns of Q, eigenvalues ascending)
    const int ma = std::min(na, CERT_M);
    double* Vl = (double*)(host.data() + offV[a]);
    for (int x = 0; x < na; ++x)
      for (int i = 0; i < ma; ++i) Vl[(size_t)x * CERT_M + i] = Q[(size_t)x * na + i];
    lam_axis[a] = lam;
    // smallest eigenvalue of the axis, and its smallest nonzero one
    double m0 = INFINITY, m1 = INFINITY;
    for (double l : lam) {
      m0 = std::min(m0, l);
      if (l > 1e-13) m1 = std::min(m1, l);
    }
    lam0[a] = m0;
    lam1[a] = m1;
  }
  // The eigenvalues of the Kronecker sum are the sums over the axes (eq. 3.3):
  // the smallest is the sum of the smallest; if that is zero (a singular
  // set, each axis having a zero eigenvalue), the smallest nonzero one adds
  // one axis's smallest nonzero eigenvalue to zeros.
  {
    double sum0 = 0.0, best1 = INFINITY;
    for (int a = 0; a < dim; ++a) {
      sum0 += lam0[a];
      best1 = std::min(best1, lam1[a]);
    }
    p->g.lam_min = sum0 > 1e-13 ? sum0 : best1;
  }
  // certificate weights 1/lambda^2 over the box of the m_a lowest modes per
  // axis (0 for the null mode), and theta, the smallest eigenvalue outside
  {
    const int mx = std::min(nx, CERT_M), my = std::min(ny, CERT_M);
    const int mz = dim == 3 ? std::min(nz, CERT_M) : 1;
    double* w = (double*)(host.data() + offW);
    for (int k = 0; k < mz; ++k)
      for (int j = 0; j < my; ++j)
        for (int i = 0; i < mx; ++i) {
          const double l = lam_axis[0][i] + lam_axis[1][j] + (dim == 3 ? lam_axis[2][k] : 0.0);
          w[((size_t)k * CERT_M + j) * CERT_M + i] = l > 1e-13 ? 1.0 / (l * l) : 0.0;
        }
    const int m[3] = {mx, my, mz};
    double theta = INFINITY;
    for (int a = 0; a < dim; ++a) {
      if (m[a] >= n[a]) continue;
      double t = lam_axis[a][m[a]];
      for (int b = 0; b < dim; ++b)
        if (b != a) t += lam_axis[b][0];
      theta = std::min(theta, t);
    }
    p->cert.theta2inv = std::isfinite(theta) ? 1.0 / (theta * theta) : 0.0;
  }
  std::lock_guard<std::mutex> alk(api_mutex());   // held until the plan is complete
  if (!ok(hipMalloc(&p->resident, bytes))) { delete p; return KP_ENOMEM; }
  p->resident_bytes = bytes;
  if (!ok(hipMemcpy(p->resident, host.data(), bytes, hipMemcpyHostToDevice))) {
    (void)hipFree(p->resident);
    delete p;
    return KP_EHIP;
  }
  p->op.dim = dim;
  p->op.prec = prec;
  p->op.N = N;
  // product order: x, y, z forward, x, y, z backward (3D); x, y, x, y (2D)
  for (int q = 0; q < 6; ++q) {
    const int ax = dim == 3 ? q % 3 : q % 2;
    p->op.cfg[q] = (q < 2 * dim) ? mp_default_config(n[ax], prec) : 0;
  }
  for (int a = 0; a < 3; ++a) {
    p->op.n[a] = n[a];
    if (a < dim) {
      p->op.Bf[a] = (char*)p->resident + offF[a];
      p->op.Bb[a] = (char*)p->resident + offB[a];
      p->op.lam[a] = (const double*)((char*)p->resident + offL[a]);
      p->cert.V[a] = (const double*)((char*)p->resident + offV[a]);
    } else {
      p->op.Bf[a] = p->op.Bb[a] = nullptr;
      p->op.lam[a] = nullptr;
    }
  }
  p->cert.w = (const double*)((char*)p->resident + offW);
  if (small) {
    p->small_ok = true;
    p->small.Vx = (const double*)((char*)p->resident + offQ[0]);
    p->small.Vy = (const double*)((char*)p->resident + offQ[1]);
    p->small.Vxt = (const double*)((char*)p->resident + offQt[0]);
    p->small.Vyt = (const double*)((char*)p->resident + offQt[1]);
    p->small.lx = p->op.lam[0];
    p->small.ly = p->op.lam[1];
  }
  if (!ok(hipStreamCreateWithFlags(&p->own, hipStreamNonBlocking)) ||
      !ok(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming)) ||
      !ok(hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming))) {
    if (p->own) (void)hipStreamDestroy(p->own);
    (void)hipFree(p->resident);
    delete p;
    return KP_EHIP;
  }
  if (!ok(hipHostMalloc((void**)&p->st_host, (size_t)max_batch * sizeof(RhsState),
                        hipHostMallocMapped | hipHostMallocCoherent)) ||
      !ok(hipHostGetDevicePointer((void**)&p->st_dev, p->st_host, 0))) {
    if (p->st_host) (void)hipHostFree(p->st_host);
    (void)hipFree(p->resident);
    delete p;
    return KP_ENOMEM;
  }
  *out = p;
  return KP_OK;
}

void kp_plan_destroy(kp_plan* p) {
  if (!p) return;
  if (p->busy) {   // a solve still in flight: finished and released here
    solve_advance(p->busy, true);
    delete p->busy;
    p->busy = nullptr;
  }
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  if (p->own) (void)hipStreamSynchronize(p->own);
  clear_graphs(p);
  std::lock_guard<std::mutex> lk(api_mutex());
  if (p->own) (void)hipStreamDestroy(p->own);
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->ev_done) (void)hipEventDestroy(p->ev_done);
  if (p->ws_owned && p->ws) (void)hipFree(p->ws);
  if (p->hist) (void)hipHostFree(p->hist);
  if (p->diag) (void)hipHostFree(p->diag);
  if (p->resident) (void)hipFree(p->resident);
  if (p->st_host) (void)hipHostFree(p->st_host);
  if (p->faces_dev) (void)hipFree(p->faces_dev);
  if (p->lr_dev) (void)hipFree(p->lr_dev);
  delete p;
}

size_t kp_plan_workspace_bytes(const kp_plan* p, int batch) {
  if (!p || batch < 1) return 0;
  return layout_for(p, batch).total;
}

size_t kp_plan_resident_bytes(const kp_plan* p) { return p ? p->resident_bytes : 0; }

int kp_plan_set_workspace(kp_plan* p, void* dev, size_t bytes) {
  if (!p || !dev || ((uintptr_t)dev & (ALIGN - 1))) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (bytes < layout_for(p, p->max_batch).total) return KP_ENOMEM;
  if (p->ws_owned && p->ws) {
    (void)hipStreamSynchronize(p->stream);
    std::lock_guard<std::mutex> lk(api_mutex());
    (void)hipFree(p->ws);
  }
  p->ws = dev;
  p->ws_bytes = bytes;
  p->ws_owned = false;
  clear_graphs(p);    // captured kernels point into the old workspace
  return KP_OK;
}

int kp_plan_set_stream(kp_plan* p, void* s) {
  if (!p) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  p->stream = (hipStream_t)s;
  return KP_OK;
}

int kp_apply_laplacian(kp_plan* p, const double* P, double* W, int batch) {
  if (!p || !P || !W || batch < 1 || batch > p->max_batch) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (!aligned16(P) || !aligned16(W)) return KP_EINVAL;
  if (overlap(P, W, (size_t)p->g.N * batch * 8)) return KP_EINVAL;
  TraceScope scope(p);
  launch_laplacian(p->g, P, W, batch, vec_blocks(p->g.N, batch), p->stream);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

int kp_apply_pinv(kp_plan* p, const double* R, double* Z, int batch) {
  if (!p || !R || !Z || batch < 1 || batch > p->max_batch) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (!aligned16(R) || !aligned16(Z)) return KP_EINVAL;
  if (overlap(R, Z, (size_t)p->g.N * batch * 8)) return KP_EINVAL;
  int rc = ensure_workspace(p);
  if (rc != KP_OK) return rc;
  const Layout L = layout_for(p, batch);
  char* base = (char*)p->ws;
  TraceScope scope(p);
  pinv_apply(p->op, R, Z, base + L.T0, base + L.T1, batch, nullptr, p->stream);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

int kp_apply_pinv_noalloc(kp_plan* p, const double* R, double* Z, int batch) {
  if (!p || !R || !Z || batch < 1 || batch > p->max_batch) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (!aligned16(R) || !aligned16(Z)) return KP_EINVAL;
  if (overlap(R, Z, (size_t)p->g.N * batch * 8)) return KP_EINVAL;
  // the two intermediate grids of the mode products, back to back
  const size_t half = align_up((size_t)p->g.N * batch * elem_bytes(p->prec));
  if (2 * half > (size_t)KP_NOALLOC_SCRATCH_BYTES) {
    snprintf(t_last_error, sizeof t_last_error,
             "kp_apply_pinv_noalloc: %zu bytes of scratch needed, the static scratch holds %zu",
             2 * half, (size_t)KP_NOALLOC_SCRATCH_BYTES);
    return KP_ENOMEM;
  }
  int dev = -1;
  if (!ok(hipGetDevice(&dev))) return KP_EHIP;
  if (dev != p->device) return KP_EINVAL;
  char* base = nullptr;
  const int rc = noalloc_scratch(dev, &base);
  if (rc != KP_OK) return rc;
  (void)hipGetLastError();
  // no tracer here: its timing events would be created on demand
  pinv_apply(p->op, R, Z, base, base + half, batch, nullptr, p->stream);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

int kp_solve(kp_plan* p, const double* eta, double* u, int batch, double tol, int max_iter,
             int flags, kp_result* results, double* res_hist) {
  if (!p) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  kp_ticket t;
  int rc = solve_start(&t, p, eta, u, batch, tol, max_iter, flags, results, res_hist);
  if (rc != KP_OK) return rc;
  solve_advance(&t, true);
  return t.status;
}

int kp_solve_async(kp_plan* p, const double* eta, double* u, int batch, double tol, int max_iter,
                   int flags, kp_result* results, double* res_hist, kp_ticket** ticket) {
  if (ticket) *ticket = nullptr;
  if (!p || !ticket) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  kp_ticket* t = new (std::nothrow) kp_ticket();
  if (!t) return KP_ENOMEM;
  const int rc = solve_start(t, p, eta, u, batch, tol, max_iter, flags, results, res_hist);
  if (rc != KP_OK) {
    delete t;
    return rc;
  }
  p->busy = t;
  *ticket = t;
  return KP_OK;
}

int kp_poll(kp_ticket* t) {
  if (!t) return KP_EINVAL;
  return solve_advance(t, false);
}

int kp_wait(kp_ticket* t) {
  if (!t) return KP_EINVAL;
  solve_advance(t, true);
  const int rc = t->status;
  if (t->p && t->p->busy == t) t->p->busy = nullptr;
  delete t;
  return rc;
}

int kp_plan_diagnostics(const kp_plan* p, double* out, int batch, int hs, int delay) {
  if (!p || !out || p->diag_batch == 0 || batch != p->diag_batch || hs != p->diag_hs ||
      delay < 1)
    return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (int b = 0; b < batch; ++b) {
    const double* raw = p->diag + (size_t)b * hs * DIAG_RAW;
    const int last = std::min(p->st_host[b].diag_iter, hs - 1);   // rows 0..last recorded
    double kmin = std::numeric_limits<double>::infinity();
    for (int q = 0; q <= last; ++q) kmin = std::min(kmin, raw[q * DIAG_RAW + 1]);
    for (int q = 0; q < hs; ++q) {
      double* o = out + ((size_t)b * hs + q) * KP_DIAG_COLUMNS;
      if (q > last) {
        for (int c = 0; c < KP_DIAG_COLUMNS; ++c) o[c] = nan;
        continue;
      }
      const double* r = raw + q * DIAG_RAW;
      o[0] = r[0];
      o[1] = p->hist[(size_t)b * hs + q];
      o[2] = r[1];
      o[3] = std::sqrt(std::max(r[1] - kmin, 0.0));
      o[4] = r[2];
      o[5] = r[3];
      double acc = 0.0;
      for (int j = q + 1; j <= std::min(q + delay, last); ++j) acc += raw[j * DIAG_RAW + 3];
      o[6] = std::sqrt(std::max(acc, 0.0));
    }
  }
  return KP_OK;
}

int kp_lowrank_table(int n, int bc_n, int q, int bc_q, int rank, double* table) {
  if (n < 3 || q < 3 || bc_n < 0 || bc_n > 4 || bc_q < 0 || bc_q > 4 || !table) return KP_EINVAL;
  if (rank < 1 || rank > std::min(KP_LOWRANK_MAX, std::min(n, q))) return KP_EINVAL;
  std::vector<double> Qn((size_t)n * n), Qq((size_t)q * q), ln(n), lq(q);
  if (basis_1d(n, bc_n, Qn.data(), ln.data()) != 0 || basis_1d(q, bc_q, Qq.data(), lq.data()) != 0)
    return KP_EINVAL;
  return lowrank_table(ln.data(), n, lq.data(), q, rank, table) == 0 ? KP_OK : KP_EINVAL;
}

int kp_plan_set_preconditioner(kp_plan* p, int kind, int steps, double omega) {
  if (!p || (kind != KP_PRECOND_PINV && kind != KP_PRECOND_JACOBI && kind != KP_PRECOND_LOWRANK))
    return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (kind == KP_PRECOND_JACOBI &&
      (steps < 1 || steps > 10000 || !(omega >= 1.0) || !std::isfinite(omega)))
    return KP_EINVAL;
  if (kind == KP_PRECOND_LOWRANK) {
    if (p->g.dim != 2) return KP_EINVAL;   // no 3D analogue (Sec. 4.3.2)
    if (steps < 1 || steps > std::min(KP_LOWRANK_MAX, std::min(p->g.nx, p->g.ny)))
      return KP_EINVAL;
    if (steps != p->lr_rank) {
      const size_t n = (size_t)p->g.nx * p->g.ny;
      std::vector<double> tab(n);
      const int rc = kp_lowrank_table(p->g.nx, p->g.bc[0], p->g.ny, p->g.bc[1], steps, tab.data());
      if (rc != KP_OK) return rc;
      if (p->stream) (void)hipStreamSynchronize(p->stream);
      if (p->own) (void)hipStreamSynchronize(p->own);
      std::lock_guard<std::mutex> lk(api_mutex());
      if (!p->lr_dev && !ok(hipMalloc((void**)&p->lr_dev, n * sizeof(double)))) {
        p->lr_dev = nullptr;
        return KP_ENOMEM;
      }
      if (!ok(hipMemcpy(p->lr_dev, tab.data(), n * sizeof(double), hipMemcpyHostToDevice))) {
        p->lr_rank = 0;
        return KP_EHIP;
      }
      p->lr_rank = steps;
    }
  }
  const int old_kind = p->pc_kind;
  p->pc_kind = kind;
  const size_t need = layout_for(p, p->max_batch).total;
  if (p->ws && p->ws_bytes < need) {
    if (!p->ws_owned) { p->pc_kind = old_kind; return KP_ENOMEM; }   // caller's buffer too small
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->own) (void)hipStreamSynchronize(p->own);
    std::lock_guard<std::mutex> lk(api_mutex());
    (void)hipFree(p->ws);
    p->ws = nullptr;          // reallocated at the next use
    p->ws_bytes = 0;
  }
  if (kind == KP_PRECOND_JACOBI) {
    p->jac_p = steps;
    p->jac_omega = omega;
  }
  clear_graphs(p);
  return KP_OK;
}

int kp_apply_preconditioner(kp_plan* p, const double* R, double* Z, int batch) {
  if (!p || !R || !Z || batch < 1 || batch > p->max_batch) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (!aligned16(R) || !aligned16(Z)) return KP_EINVAL;
  if (overlap(R, Z, (size_t)p->g.N * batch * 8)) return KP_EINVAL;
  int rc = ensure_workspace(p);
  if (rc != KP_OK) return rc;
  const Layout L = layout_for(p, batch);
  TraceScope scope(p);
  (void)hipGetLastError();
  precondition(p, L, R, Z, batch, 0, nullptr, p->stream);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

int kp_assemble_rhs(kp_plan* p, const double* eta, double* rhs, int batch, const double* faces) {
  if (!p || !eta || !rhs || batch < 1 || batch > p->max_batch) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (!aligned16(eta) || !aligned16(rhs)) return KP_EINVAL;
  const size_t vbytes = (size_t)p->g.N * batch * 8;
  if (eta != rhs && overlap(eta, rhs, vbytes)) return KP_EINVAL;
  const double* fdev = nullptr;
  if (faces) {
    const int rc = stage_faces(p, faces, batch, &fdev);
    if (rc != KP_OK) return rc;
  }
  (void)hipGetLastError();
  if (eta != rhs &&
      !ok(hipMemcpyAsync(rhs, eta, vbytes, hipMemcpyDeviceToDevice, p->stream)))
    return KP_EHIP;
  if (fdev) launch_face_updates(p->g, rhs, fdev, batch, p->stream);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

int kp_field(kp_plan* p, const double* u, double* eps, int batch, const double* faces) {
  if (!p || !u || !eps || batch < 1 || batch > p->max_batch) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (!aligned16(u) || !aligned16(eps)) return KP_EINVAL;
  const size_t ub = (size_t)p->g.N * batch * 8;
  const char* a = (const char*)u;
  const char* e = (const char*)eps;
  if (a < e + ub * p->g.dim && e < a + ub) return KP_EINVAL;   // u and eps overlap
  const double* fdev = nullptr;
  if (faces) {
    const int rc = stage_faces(p, faces, batch, &fdev);
    if (rc != KP_OK) return rc;
  }
  (void)hipGetLastError();
  launch_field(p->g, u, eps, fdev, batch, p->stream);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

const char* kp_strerror(int s) {
  switch (s) {
    case KP_OK: return "ok";
    case KP_NOT_CONVERGED: return "not converged within max_iter";
    case KP_EINVAL: return "invalid argument";
    case KP_ENOMEM: return "out of device memory or workspace too small";
    case KP_EHIP: return "HIP runtime error";
    case KP_ENONFINITE: return "non-finite value in right-hand side or iterate";
    case KP_EBREAKDOWN: return "CG breakdown (non-positive curvature or rho)";
    case KP_EBUSY: return "the plan has a solve in flight (kp_solve_async not yet waited for)";
    default: return "unknown status";
  }
}

const char* kp_version(void) { return "kpcg 0.1 (gfx950)"; }

const char* kp_last_error(void) { return t_last_error; }

int kp_plan_autotune(kp_plan* p, int batch, int reps, int* chosen) {
  if (!p || batch < 1 || batch > p->max_batch || reps < 1 || reps > 1000) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  (void)hipGetLastError();
  int rc = ensure_workspace(p);
  if (rc != KP_OK) return rc;
  if (p->own) (void)hipStreamSynchronize(p->own);
  const Layout L = layout_for(p, batch);
  char* base = (char*)p->ws;
  hipStream_t s = p->stream;
  const size_t vb = (size_t)p->g.N * batch * 8;
  const size_t tb = (size_t)p->g.N * batch * elem_bytes(p->prec);
  // defined contents for timing (values do not change the work)
  if (!ok(hipMemsetAsync(base + L.R, 0, vb, s)) || !ok(hipMemsetAsync(base + L.T0, 0, tb, s)) ||
      !ok(hipMemsetAsync(base + L.T1, 0, tb, s)))
    return KP_EHIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!ok(hipEventCreate(&e0)) || !ok(hipEventCreate(&e1))) return KP_EHIP;
  Tracer* saved = g_tracer;
  g_tracer = nullptr;
  const int nprod = 2 * p->g.dim;
  for (int q = 0; q < nprod; ++q) {
    const int ax = q % p->g.dim;
    const int K = p->op.n[ax];
    const int kf = (K + 15) / 16;
    const void* in = q == 0 ? (const void*)(base + L.R) : (const void*)(base + L.T0);
    void* out = q == nprod - 1 ? (void*)(base + L.Z) : (void*)(base + L.T1);
    float best = 1e30f;
    int best_id = p->op.cfg[q];
    for (int id = 0; id < mp_num_configs(); ++id) {
      if (!mp_config_allowed(id, p->prec) || !mp_config_fits(id, K)) continue;
      int wn, wm, wc;
      mp_config(id, &wn, &wm, &wc);
      const int cb = wn * wc;
      if (cb > 2 * kf && cb > 4) continue;          // mostly zero columns
      PinvOps trial = p->op;
      trial.cfg[q] = id;
      pinv_product(trial, q, in, out, batch, s);     // warm-up
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) pinv_product(trial, q, in, out, batch, s);
      (void)hipEventRecord(e1, s);
      if (!ok(hipEventSynchronize(e1))) { g_tracer = saved; return KP_EHIP; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; best_id = id; }
    }
    p->op.cfg[q] = best_id;
    if (chosen) chosen[q] = best_id;
  }
  clear_graphs(p);    // captured kernels carry the old tile choices
  g_tracer = saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ok(hipGetLastError()) ? KP_OK : KP_EHIP;
}

int kp_plan_time_kernel(kp_plan* p, int cls, int batch, int flags, int reps, double* avg_ms) {
  if (!p || !avg_ms || batch < 1 || batch > p->max_batch || reps < 1 || reps > 100000 ||
      (flags & ~KP_FLAG_FLEX_BETA))
    return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  const int dim = p->g.dim;
  int q = -1;
  switch (cls) {
    case KC_MP_X_FWD: q = 0; break;
    case KC_MP_Y_FWD: q = 1; break;
    case KC_MP_Z_FWD: q = dim == 3 ? 2 : -2; break;
    case KC_MP_X_BWD: q = dim; break;
    case KC_MP_Y_BWD: q = dim + 1; break;
    case KC_MP_Z_BWD: q = dim == 3 ? 5 : -2; break;
    case KC_STENCIL: case KC_UPDATE_UR: case KC_DOT_RZ: case KC_UPDATE_P: break;
    case KC_SMALL:
      // the last one-kernel solve again: its input, output and stopping
      // arguments (each launch recomputes the same result)
      if (!p->small_ok || !p->small_last.eta || batch > p->small_last.batch) q = -2;
      break;
    default: q = -2;
  }
  if (q == -2) return KP_EINVAL;
  (void)hipGetLastError();
  int rc = ensure_workspace(p);
  if (rc != KP_OK) return rc;
  if (p->own) (void)hipStreamSynchronize(p->own);
  const Layout L = layout_for(p, batch);
  char* base = (char*)p->ws;
  hipStream_t s = p->stream;
  const int G = vec_blocks(p->g.N, batch);
  const int64_t n = p->g.N * (int64_t)batch;
  double* R = (double*)(base + L.R);
  double* P = (double*)(base + L.P);
  double* W = (double*)(base + L.W);
  double* Z = (double*)(base + L.Z);
  double* part = (double*)(base + L.part);
  RhsState* st = (RhsState*)(base + L.st);
  void* T0 = base + L.T0;
  void* T1 = base + L.T1;
  Tracer* saved = g_tracer;
  g_tracer = nullptr;
  // defined, non-trivial data; every right-hand side running
  launch_fill(R, n, 1, s);
  launch_fill(P, n, 2, s);
  launch_fill(W, n, 3, s);
  launch_fill(Z, n, 4, s);
  launch_timing_states(st, batch, s);
  // a product's input is the previous product's output, as in a solve
  for (int k = 0; k < q; ++k) pinv_step(p->op, k, R, Z, T0, T1, batch, st, s);
  auto once = [&]() {
    if (q >= 0) pinv_step(p->op, q, R, Z, T0, T1, batch, st, s);
    else if (cls == KC_SMALL)
      launch_small_solve(p->g, p->small, p->small_last.eta, p->small_last.u, st, nullptr, nullptr,
                         0, batch, p->small_last.tol, p->small_last.max_iter,
                         p->small_last.flags, s);
    else launch_vector_class(cls, p->g, P, W, R, Z, Z, part, st, batch, G, flags, s);
  };
  once();   // warm-up
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!ok(hipEventCreate(&e0)) || !ok(hipEventCreate(&e1))) {
    g_tracer = saved;
    return KP_EHIP;
  }
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) once();
  (void)hipEventRecord(e1, s);
  rc = ok(hipEventSynchronize(e1)) ? KP_OK : KP_EHIP;
  float ms = 0.f;
  if (rc == KP_OK && !ok(hipEventElapsedTime(&ms, e0, e1))) rc = KP_EHIP;
  g_tracer = saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == KP_OK && !ok(hipGetLastError())) rc = KP_EHIP;
  if (rc == KP_OK) *avg_ms = (double)ms / reps;
  return rc;
}

int kp_plan_get_tuning(const kp_plan* p, int* cfg, int n) {
  if (!p || !cfg || n < 2 * p->g.dim) return KP_EINVAL;
  for (int q = 0; q < 2 * p->g.dim; ++q) cfg[q] = p->op.cfg[q];
  return 2 * p->g.dim;
}

int kp_tile_shape(int id, int prec, int* wn, int* wm, int* wc) {
  if (!wn || !wm || !wc || prec < PREC_F64 || prec > PREC_I8X6) return KP_EINVAL;
  if (!mp_config_allowed(id, prec)) return KP_EINVAL;
  mp_config(id, wn, wm, wc);
  return KP_OK;
}

int kp_plan_set_tuning(kp_plan* p, const int* cfg, int n) {
  if (!p || !cfg || n != 2 * p->g.dim) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  for (int q = 0; q < n; ++q)
    if (!mp_config_allowed(cfg[q], p->prec) || !mp_config_fits(cfg[q], p->op.n[q % p->g.dim]))
      return KP_EINVAL;
  for (int q = 0; q < n; ++q) p->op.cfg[q] = cfg[q];
  clear_graphs(p);
  return KP_OK;
}

int kp_plan_graph_count(const kp_plan* p) {
  if (!p) return KP_EINVAL;
  return p->graphs_ok ? (int)p->graphs.size() : -1;
}

int kp_plan_set_profiling(kp_plan* p, int enable) {
  if (!p) return KP_EINVAL;
  if (p->busy) return KP_EBUSY;
  if (p->profiling != (enable != 0)) clear_graphs(p);   // captured with or without events
  p->profiling = enable != 0;
  return KP_OK;
}

int kp_plan_profile(kp_plan* p, int cls, double* total_ms, int64_t* launches) {
  if (!p || cls < 0 || cls >= KC_COUNT) return KP_EINVAL;
  if (!ok(hipStreamSynchronize(p->stream))) return KP_EHIP;
  p->tracer.collect();
  if (total_ms) *total_ms = p->tracer.ms[cls];
  if (launches) *launches = p->tracer.cnt[cls];
  return KP_OK;
}

int kp_plan_profile_reset(kp_plan* p) {
  if (!p) return KP_EINVAL;
  if (!ok(hipStreamSynchronize(p->stream))) return KP_EHIP;
  p->tracer.collect();
  p->tracer.reset();
  return KP_OK;
}

const char* kp_kernel_class_name(int cls) {
  static const char* names[KC_COUNT] = {
      "stencil_dot", "update_ur", "dot_rz", "update_p", "finalize", "init", "finish",
      "modeprod_z_fwd", "modeprod_y_fwd", "modeprod_x_fwd", "modeprod_x_bwd",
      "modeprod_y_bwd", "modeprod_z_bwd", "copy", "jacobi", "diagnostics", "certificate",
      "small_solve"};
  return (cls >= 0 && cls < KC_COUNT) ? names[cls] : "unknown";
}

}  // extern "C"
