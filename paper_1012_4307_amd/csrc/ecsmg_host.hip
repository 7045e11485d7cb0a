// ecsmg_host.hip -- host side of the C ABI in include/ecsmg.h: problem
// context, ECS contour and grid hierarchy, multigrid cycle orchestration
// (Algorithm 1 of bin Zubair, Reps, Vanroose, Sec. 4.2), and the right-
// preconditioned GMRES / FGMRES / Bi-CGSTAB drivers of Sec. 5.  Every
// arithmetic step on grid vectors runs in the HIP kernels of kernels_mg.hip
// and kernels_blas.hip; the host only sequences launches, sets the problem up
// (contour weights, coarsest dense inverse) and reads one residual estimate per
// iteration to decide convergence.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ecs_krylov.h"
#include "ecsmg.h"

using namespace ecs;
using cd = std::complex<double>;

thread_local KernelEvents ecs::g_kernel_events;

// Device scratch of ecs_solve_static: the Krylov vectors of a solve for
// callers that cannot allocate device memory.  Every GPU the library runs on
// holds its own copy until the process ends.  In host code the array's name
// stands for no device address: kernels and copies take the per-device
// address looked up once (scratch_address) instead.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxLev = 16;
constexpr int kMaxDevices = 64;
// host-pinned scalars per context: readbacks in [0, kPinnedStage), host-to-
// device staging above
constexpr size_t kPinnedBytes = 1024;
constexpr size_t kPinnedStage = 768;

std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch array (the current device), looked up on
// the first call per device; null (and the HIP error in *err) on failure.
char *scratch_address(int device, hipError_t *err) {
  *err = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[device] = reinterpret_cast<char *>(p);
  }
  return g_scratch_ptr[device];
}

struct Side {
  int kind = ECS_BC_DIRICHLET;
  double start = 0, theta = 0;
};

// host copy of one level's contour and second-difference weights
struct HostLevel {
  int n[3] = {1, 1, 1};
  int64_t nn = 0;
  std::vector<cd> z[3], am[3], ap[3], w[3];
};

template <typename R>
struct DevLevel {
  cplx<R> *cm[3] = {nullptr, nullptr, nullptr};  // alpha * a-  (preconditioner operator M)
  cplx<R> *cp[3] = {nullptr, nullptr, nullptr};  // alpha * a+
  R *k2 = nullptr;
  cplx<R> *b = nullptr, *u = nullptr, *t = nullptr;
};

struct Timer {
  std::vector<hipEvent_t> ev;  // start/stop pairs
  size_t used = 0;
  bool on = false;
  int every = 1;               // time one launch in `every` of the class
  int64_t seen = 0;            // launch scopes of the class since enabling
  double bytes = 0;            // algorithmic bytes of the timed launches
};

// timing classes (see ecs_timing_enable in ecsmg.h)
enum { kTSmooth = 0, kTMdot = 1, kTApply = 2, kTCoarse = 3, kTMupdate = 4, kTRestrict = 5, kTProlong = 6,
       kTDown = 7, kTUp = 8, kTEmpty = 9, kTDownP = 10, kTDownS = 11, kTClasses = 12 };

// bump allocator over the caller's workspace (256 B alignment); with a null
// base it only measures
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(char *b) : base(b) {}
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace

struct ecs_ctx {
  int dim = 2;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  hipStream_t stream = nullptr;
  int device = 0;
  Side side[3][2];
  // k^2 as handed over (borrowed), its dtype, and the FP64 array the kernels
  // read: the caller's own array for FP64, else a copy widened at set-up
  const void *k2_user = nullptr;
  int k2_dtype = ECS_F64;
  const double *k2 = nullptr;
  double *k2_wide = nullptr;
  bool have_prec = false;
  ecs_prec_desc prec{};
  int nlev = 0;
  std::vector<HostLevel> hl;
  cd alpha{1, 0}, beta{-1, 0}, c{0, 0};
  double lam0 = 0;

  char *ws = nullptr;
  size_t ws_bytes = 0, hier_bytes = 0;
  bool ready = false;

  // FP64 finest-level weights of A and of the symmetriser W
  cplx<double> *Acm[3] = {}, *Acp[3] = {}, *Wd[3] = {};
  cplx<float> *Acm32[3] = {}, *Acp32[3] = {};  // FP32 copy of A's weights (nested form)
  DevLevel<double> L64[kMaxLev];
  DevLevel<float> L32[kMaxLev];
  cplx<double> *minv64 = nullptr;
  cplx<float> *minv32 = nullptr;
  int *unk = nullptr;
  int nunk = 0;
  cplx<double> *partials = nullptr;
  double *dscal = nullptr;  // misc device scalars (max k^2 ...)
  GmresScalars *gs = nullptr;
  BicgScalars *bs = nullptr, *bs_in = nullptr;
  double *pinned = nullptr;  // host-pinned scalars for readback
  hipEvent_t step_ev = nullptr;  // completion of the batched driver's last step on this context

  Timer timers[kTClasses];
  std::string err;

  // this device's ecs_solve_static scratch (looked up at creation); while
  // no_alloc is set the cycle is launched eagerly (no graph is captured or
  // instantiated) and no timer records
  char *scratch = nullptr;
  bool no_alloc = false;

  // replayable V-cycles: one instantiated graph per (input, output, dtype),
  // captured on a private stream and launched on `stream`
  struct GraphEntry {
    const void *b;
    void *u;
    int real_bytes;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t capture = nullptr;
  int graph_mode = ECS_GRAPHS_AUTO;

  // launch schedule of the fused V(1,1) cycle (autotuned per grid and dtype)
  ecs_tuning tune{4, 8, 513, 33, 129, 1};
  // FP64 Bi-CGSTAB with its p update inside the cycle: which of p / p2 holds
  // the current direction (reset at every restart)
  int bicg_pflip = 0;

  // coarse end of the general cycle in one workgroup (2D): packed weights and
  // inverse diagonals of the levels that may form it (levels sfirst .. coarsest,
  // level l at spko[l] - spko[sfirst]), and the schedules unrolled from
  // Algorithm 1 for the loaded key (tail level, gamma_f, gamma_c, nu1, nu2,
  // smoother); variants: (gf, gc) or (gc, gf), each from zero or from a guess
  cplx<double> *spack64 = nullptr;
  cplx<float> *spack32 = nullptr;
  int sfirst = -1;
  int spko[kMaxLev + 1] = {};
  uint32_t *sprog = nullptr;
  int sprog_len[4] = {};
  int skey[6] = {-2, 0, 0, 0, 0, 0};
  int gt_l = -1;  // first level of the tail in use, -1: none
};

namespace {

int64_t nn_of(const ecs_ctx *C) { return (int64_t)C->n[0] * C->n[1] * C->n[2]; }

ecs_status fail(ecs_ctx *C, ecs_status st, const std::string &msg) {
  if (C) C->err = msg;
  return st;
}

#define HIP_OK(call)                                                                                        \
  do {                                                                                                      \
    hipError_t e_ = (call);                                                                                 \
    if (e_ != hipSuccess) return fail(C, ECS_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_));     \
  } while (0)

// ------------------------------------------------------------ geometry
// Sec. 3.1: nodal contour of one axis, z = x up to a layer start s, rotated
// beyond it: z = s + (x - s) e^{i theta}.
std::vector<cd> contour(int n, double lo, double hi, const Side &slo, const Side &shi) {
  std::vector<cd> z(n);
  const double h = (hi - lo) / (n - 1);
  for (int i = 0; i < n; i++) {
    double x = lo + i * h;
    cd zi(x, 0);
    if (shi.kind == ECS_BC_ECS && x > shi.start) zi = shi.start + (x - shi.start) * std::polar(1.0, shi.theta);
    if (slo.kind == ECS_BC_ECS && x < slo.start) zi = slo.start + (x - slo.start) * std::polar(1.0, slo.theta);
    z[i] = zi;
  }
  return z;
}

// Sec. 3.2: non-uniform 3-point weights from node spacings h_{i-1}, h_i:
//   a-_i = 2/((h_{i-1}+h_i) h_{i-1}),  a+_i = 2/((h_{i-1}+h_i) h_i),
// dual width w_i = (h_{i-1}+h_i)/2; end nodes get a = 0, w = 1.
void weights(const std::vector<cd> &z, std::vector<cd> &am, std::vector<cd> &ap, std::vector<cd> &w) {
  const size_t n = z.size();
  am.assign(n, 0.0);
  ap.assign(n, 0.0);
  w.assign(n, 1.0);
  for (size_t i = 1; i + 1 < n; i++) {
    cd hl = z[i] - z[i - 1], hr = z[i + 1] - z[i];
    cd s = hl + hr;
    am[i] = 2.0 / (s * hl);
    ap[i] = 2.0 / (s * hr);
    w[i] = 0.5 * s;
  }
}

void build_host_levels(ecs_ctx *C) {
  C->hl.assign(C->nlev, HostLevel());
  for (int l = 0; l < C->nlev; l++) {
    HostLevel &L = C->hl[l];
    for (int a = 0; a < 3; a++) {
      if (a >= C->dim) {
        L.n[a] = 1;
        L.z[a].assign(1, 0.0);
        L.am[a].assign(1, 0.0);
        L.ap[a].assign(1, 0.0);
        L.w[a].assign(1, 1.0);
        continue;
      }
      if (l == 0) {
        L.n[a] = C->n[a];
        L.z[a] = contour(C->n[a], C->lo[a], C->hi[a], C->side[a][0], C->side[a][1]);
      } else {
        const HostLevel &F = C->hl[l - 1];
        L.n[a] = (F.n[a] - 1) / 2 + 1;
        L.z[a].resize(L.n[a]);
        for (int i = 0; i < L.n[a]; i++) L.z[a][i] = F.z[a][2 * i];  // exact nesting
      }
      weights(L.z[a], L.am[a], L.ap[a], L.w[a]);
    }
    L.nn = (int64_t)L.n[0] * L.n[1] * L.n[2];
  }
}

// ------------------------------------------------------ workspace plan
size_t plan_layout(ecs_ctx *C, Carver &cv) {
  const bool f32 = C->prec.vcycle_dtype == ECS_F32;
  C->k2_wide = C->k2_dtype == ECS_F32 ? cv.take<double>(C->hl[0].nn) : nullptr;
  for (int a = 0; a < C->dim; a++) {
    C->Acm[a] = cv.take<cplx<double>>(C->hl[0].n[a]);
    C->Acp[a] = cv.take<cplx<double>>(C->hl[0].n[a]);
    C->Wd[a] = cv.take<cplx<double>>(C->hl[0].n[a]);
    if (f32) {
      C->Acm32[a] = cv.take<cplx<float>>(C->hl[0].n[a]);
      C->Acp32[a] = cv.take<cplx<float>>(C->hl[0].n[a]);
    }
  }
  for (int l = 0; l < C->nlev; l++) {
    const HostLevel &L = C->hl[l];
    DevLevel<double> &D = C->L64[l];
    DevLevel<float> &S = C->L32[l];
    for (int a = 0; a < C->dim; a++) {
      D.cm[a] = cv.take<cplx<double>>(L.n[a]);
      D.cp[a] = cv.take<cplx<double>>(L.n[a]);
      if (f32) {
        S.cm[a] = cv.take<cplx<float>>(L.n[a]);
        S.cp[a] = cv.take<cplx<float>>(L.n[a]);
      }
    }
    D.k2 = (l == 0) ? nullptr : cv.take<double>(L.nn);
    if (f32) S.k2 = cv.take<float>(L.nn);
    if (!f32) {
      D.b = (l == 0) ? nullptr : cv.take<cplx<double>>(L.nn);
      D.u = (l == 0) ? nullptr : cv.take<cplx<double>>(L.nn);
      D.t = cv.take<cplx<double>>(L.nn);
    } else {
      S.b = cv.take<cplx<float>>(L.nn);
      S.u = (l == 0) ? nullptr : cv.take<cplx<float>>(L.nn);
      S.t = cv.take<cplx<float>>(L.nn);
    }
  }
  const HostLevel &Lc = C->hl[C->nlev - 1];
  int nunk = 1;
  for (int a = 0; a < C->dim; a++) nunk *= (Lc.n[a] - 2);
  C->nunk = nunk;
  C->minv64 = cv.take<cplx<double>>((size_t)nunk * nunk);
  if (f32) C->minv32 = cv.take<cplx<float>>((size_t)nunk * nunk);
  C->unk = cv.take<int>(nunk);
  C->spack64 = cv.take<cplx<double>>(kSchedPack);
  if (f32) C->spack32 = cv.take<cplx<float>>(kSchedPack);
  C->sprog = cv.take<uint32_t>(4 * kSchedProgCap);
  C->partials = cv.take<cplx<double>>((size_t)kRedBlocks * (2 * kMaxRestart + 2));
  C->dscal = cv.take<double>(kRedBlocks + 8);
  C->gs = cv.take<GmresScalars>(1);
  C->bs = cv.take<BicgScalars>(kMaxRhs);  // one per right-hand side slot of the batched solve
  C->bs_in = cv.take<BicgScalars>(1);
  return cv.off;
}

// Lays out the hierarchy in the workspace.  With a null base only the size
// is measured and the context's device pointers are left untouched.
size_t plan_hierarchy(ecs_ctx *C, char *base) {
  if (!base) {
    ecs_ctx probe;
    probe.dim = C->dim;
    probe.nlev = C->nlev;
    probe.prec = C->prec;
    probe.k2_dtype = C->k2_dtype;
    probe.hl = C->hl;
    Carver cv(nullptr);
    return plan_layout(&probe, cv);
  }
  Carver cv(base);
  return plan_layout(C, cv);
}

// Krylov storage laid out after the hierarchy
struct KrylovBufs {
  cplx<double> *V = nullptr;  // (m+1) x n
  void *Z = nullptr;          // m x n in the cycle dtype (FGMRES)
  cplx<double> *t = nullptr;  // n
  void *tz = nullptr;         // n, cycle dtype
  cplx<double> *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *tt = nullptr;
  void *ph = nullptr, *sh = nullptr;
  cplx<double> *p2 = nullptr;  // FP64 cycle: second p buffer for the update inside the cycle
  // nested Bi-CGSTAB of the FGMRES preconditioner, in the cycle's dtype; fp2:
  // second p buffer (the fused update writes p beside the old one)
  void *fr = nullptr, *frh = nullptr, *fp = nullptr, *fv = nullptr, *fs = nullptr, *ft = nullptr, *fph = nullptr,
       *fsh = nullptr, *fp2 = nullptr;
  // its deferred x update: fph / fsh hold fdefer steps' p^ and s^ (ld apart),
  // fcoef their (alpha, omega)
  int fdefer = 0;
  cplx<double> *fcoef = nullptr;
  cplx<double> *a1 = nullptr, *a2 = nullptr;  // adjoint scaling buffers
  cplx<double> *bz = nullptr;                 // right-hand side with its boundary entries zeroed
  int64_t ld = 0;
  // batched Bi-CGSTAB (plan_batch): slots copies of every vector, rhs_stride(n)
  // apart (r .. sh, bz above, the iterates bx), the FP32 cycle's input per slot
  // and the cycle's level buffers per slot (void: the cycle's dtype)
  int slots = 0;
  cplx<double> *bx = nullptr;
  void *b32 = nullptr;
  void *lb[kMaxLev] = {}, *lt[kMaxLev] = {}, *lu[kMaxLev] = {};
};

// Storage of the batched Bi-CGSTAB for `slots` right-hand sides at once (one
// group of a system's right-hand sides; see batch_solve_impl).
size_t plan_batch(const ecs_ctx *C, int slots, char *base, KrylovBufs *K) {
  Carver cv(base);
  const int64_t n = nn_of(C), sn = rhs_stride(n) * slots;
  const bool f32 = C->prec.vcycle_dtype == ECS_F32;
  const size_t zs = f32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  K->slots = slots;
  K->ld = rhs_stride(n);
  K->bz = cv.take<cplx<double>>(sn);
  K->bx = cv.take<cplx<double>>(sn);
  K->r = cv.take<cplx<double>>(sn);
  K->rh = cv.take<cplx<double>>(sn);
  K->p = cv.take<cplx<double>>(sn);
  K->v = cv.take<cplx<double>>(sn);
  K->s = cv.take<cplx<double>>(sn);
  K->tt = cv.take<cplx<double>>(sn);
  K->ph = cv.take<char>(sn * zs);
  K->sh = cv.take<char>(sn * zs);
  K->b32 = f32 ? cv.take<char>(sn * zs) : nullptr;
  for (int l = 0; l < C->nlev; l++) {
    const int64_t sl = rhs_stride(C->hl[l].nn) * slots;
    K->lt[l] = cv.take<char>(sl * zs);
    K->lb[l] = l == 0 ? nullptr : cv.take<char>(sl * zs);
    K->lu[l] = l == 0 ? nullptr : cv.take<char>(sl * zs);
  }
  return cv.off;
}

// The outer FP64 Bi-CGSTAB forms p and s inside the cycle (bicg_enqueue_step) up to 1025^2 finest
// nodes, where a launch is short enough that the two it saves count: measured
// 2-3% faster at 513^2 and 1025^2.  At 2049^2 the fused FP64 kernels (121
// VGPRs for p against 84 for the plain down kernel) lose occupancy on a level
// that is bandwidth-bound: 1-2% slower for every tile height, so the separate
// update kernels stay there.
constexpr int64_t kFuse64MaxNodes = int64_t(1025) * 1025;

size_t plan_krylov(const ecs_ctx *C, const ecs_solve_desc *d, char *base, KrylovBufs *K) {
  Carver cv(base);
  const int64_t n = nn_of(C);
  const size_t zs = C->prec.vcycle_dtype == ECS_F32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  K->ld = (n + 31) & ~int64_t(31);
  K->a1 = cv.take<cplx<double>>(n);
  K->a2 = cv.take<cplx<double>>(n);
  K->tz = cv.take<char>(n * zs);
  K->bz = cv.take<cplx<double>>(n);
  if (!d) return cv.off;
  if (d->krylov == ECS_KRYLOV_BICGSTAB) {
    K->r = cv.take<cplx<double>>(n);
    K->rh = cv.take<cplx<double>>(n);
    K->p = cv.take<cplx<double>>(n);
    K->v = cv.take<cplx<double>>(n);
    K->s = cv.take<cplx<double>>(n);
    K->tt = cv.take<cplx<double>>(n);
    K->ph = cv.take<char>(n * zs);
    K->sh = cv.take<char>(n * zs);
    // its second p buffer (kFuse64MaxNodes above)
    if (C->prec.vcycle_dtype == ECS_F64 && n <= kFuse64MaxNodes) K->p2 = cv.take<cplx<double>>(n);
  } else {
    const int m = d->restart;
    K->V = cv.take<cplx<double>>((size_t)K->ld * (m + 1));
    K->t = cv.take<cplx<double>>(n);
    if (d->krylov == ECS_KRYLOV_FGMRES) K->Z = cv.take<char>((size_t)K->ld * m * zs);
    if (d->inner > 0) {
      K->fr = cv.take<char>(n * zs);
      K->frh = cv.take<char>(n * zs);
      K->fp = cv.take<char>(n * zs);
      K->fv = cv.take<char>(n * zs);
      K->fs = cv.take<char>(n * zs);
      K->ft = cv.take<char>(n * zs);
      K->fdefer = std::min(d->inner, kDeferSteps);
      K->fph = cv.take<char>((size_t)K->ld * K->fdefer * zs);
      K->fsh = cv.take<char>((size_t)K->ld * K->fdefer * zs);
      K->fcoef = cv.take<cplx<double>>(2 * (size_t)K->fdefer);
      K->fp2 = cv.take<char>(n * zs);
    }
  }
  return cv.off;
}

// ------------------------------------------------------------ timing
struct TimedScope {
  ecs_ctx *C;
  Timer *T;
  size_t slot = SIZE_MAX;
  double bytes = 0;
  TimedScope(ecs_ctx *c, int cls, double b) : C(c), T(&c->timers[cls]) {
    if (!T->on || C->no_alloc) return;
    if (T->seen++ % T->every != 0) return;
    if (T->used + 2 > T->ev.size()) {
      if (T->ev.size() >= 2 * 65536) return;
      size_t old = T->ev.size();
      T->ev.resize(old + 2 * 1024);
      for (size_t q = old; q < T->ev.size(); q++) (void)hipEventCreate(&T->ev[q]);
    }
    slot = T->used;
    T->used += 2;
    bytes = b;
    T->bytes += b;
    // the scope's first kernel launch records into this pair
    g_kernel_events.start = T->ev[slot];
    g_kernel_events.stop = T->ev[slot + 1];
  }
  ~TimedScope() {
    if (slot == SIZE_MAX) return;
    if (g_kernel_events.start == T->ev[slot]) {  // nothing was launched: drop the sample
      g_kernel_events.start = g_kernel_events.stop = nullptr;
      T->used -= 2;
      T->bytes -= bytes;
    }
  }
};

// ------------------------------------------------------- grid views
template <typename R>
cplx<R> tocx(cd v) {
  return mk<R>((R)v.real(), (R)v.imag());
}

template <typename R>
Grid<R> grid_M(const ecs_ctx *C, int l);

template <>
Grid<double> grid_M<double>(const ecs_ctx *C, int l) {
  const HostLevel &L = C->hl[l];
  const DevLevel<double> &D = C->L64[l];
  Grid<double> g;
  g.n0 = L.n[0];
  g.n1 = L.n[1];
  g.n2 = L.n[2];
  g.cm0 = D.cm[0]; g.cp0 = D.cp[0];
  g.cm1 = D.cm[1]; g.cp1 = D.cp[1];
  g.cm2 = D.cm[2]; g.cp2 = D.cp[2];
  g.k2 = l == 0 ? C->k2 : D.k2;
  g.beta = tocx<double>(C->beta);
  g.c = tocx<double>(C->c);
  return g;
}

template <>
Grid<float> grid_M<float>(const ecs_ctx *C, int l) {
  const HostLevel &L = C->hl[l];
  const DevLevel<float> &D = C->L32[l];
  Grid<float> g;
  g.n0 = L.n[0];
  g.n1 = L.n[1];
  g.n2 = L.n[2];
  g.cm0 = D.cm[0]; g.cp0 = D.cp[0];
  g.cm1 = D.cm[1]; g.cp1 = D.cp[1];
  g.cm2 = D.cm[2]; g.cp2 = D.cp[2];
  g.k2 = D.k2;
  g.beta = tocx<float>(C->beta);
  g.c = tocx<float>(C->c);
  return g;
}

// the discrete ECS Helmholtz operator A = Z on the finest grid (FP64)
Grid<double> grid_A(const ecs_ctx *C) {
  Grid<double> g = grid_M<double>(C, 0);
  g.cm0 = C->Acm[0]; g.cp0 = C->Acp[0];
  g.cm1 = C->Acm[1]; g.cp1 = C->Acp[1];
  g.cm2 = C->Acm[2]; g.cp2 = C->Acp[2];
  g.beta = mk<double>(-1, 0);
  g.c = mk<double>(0, 0);
  return g;
}

// A in FP32 (finest grid), for the FP32 inner Krylov iteration
Grid<float> grid_A32(const ecs_ctx *C) {
  Grid<float> g = grid_M<float>(C, 0);
  g.cm0 = C->Acm32[0]; g.cp0 = C->Acp32[0];
  g.cm1 = C->Acm32[1]; g.cp1 = C->Acp32[1];
  g.cm2 = C->Acm32[2]; g.cp2 = C->Acp32[2];
  g.beta = mk<float>(-1, 0);
  g.c = mk<float>(0, 0);
  return g;
}

template <typename R>
DevLevel<R> &dev_level(ecs_ctx *C, int l);
template <>
DevLevel<double> &dev_level<double>(ecs_ctx *C, int l) { return C->L64[l]; }
template <>
DevLevel<float> &dev_level<float>(ecs_ctx *C, int l) { return C->L32[l]; }

template <typename R>
const cplx<R> *minv_of(const ecs_ctx *C);
template <>
const cplx<double> *minv_of<double>(const ecs_ctx *C) { return C->minv64; }
template <>
const cplx<float> *minv_of<float>(const ecs_ctx *C) { return C->minv32; }

// ---------------------------------------------------------- setup
template <typename R>
ecs_status upload_cx(ecs_ctx *C, cplx<R> *dst, const std::vector<cd> &src, cd scale) {
  std::vector<cplx<R>> h(src.size());
  for (size_t i = 0; i < src.size(); i++) h[i] = tocx<R>(scale * src[i]);
  HIP_OK(hipMemcpy(dst, h.data(), h.size() * sizeof(cplx<R>), hipMemcpyHostToDevice));
  return ECS_OK;
}

// Gauss-Jordan inverse with partial pivoting (FP64) of a dense complex matrix
bool invert(std::vector<cd> &a, int n) {
  std::vector<cd> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; i++) inv[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; k++) {
    int pr = k;
    double best = std::abs(a[(size_t)k * n + k]);
    for (int r = k + 1; r < n; r++)
      if (std::abs(a[(size_t)r * n + k]) > best) {
        best = std::abs(a[(size_t)r * n + k]);
        pr = r;
      }
    if (best == 0) return false;
    if (pr != k)
      for (int q = 0; q < n; q++) {
        std::swap(a[(size_t)k * n + q], a[(size_t)pr * n + q]);
        std::swap(inv[(size_t)k * n + q], inv[(size_t)pr * n + q]);
      }
    cd piv = 1.0 / a[(size_t)k * n + k];
    for (int q = 0; q < n; q++) {
      a[(size_t)k * n + q] *= piv;
      inv[(size_t)k * n + q] *= piv;
    }
    for (int r = 0; r < n; r++) {
      if (r == k) continue;
      cd f = a[(size_t)r * n + k];
      if (f == 0.0) continue;
      for (int q = 0; q < n; q++) {
        a[(size_t)r * n + q] -= f * a[(size_t)k * n + q];
        inv[(size_t)r * n + q] -= f * inv[(size_t)k * n + q];
      }
    }
  }
  a.swap(inv);
  return true;
}

ecs_status setup(ecs_ctx *C) {
  const bool f32 = C->prec.vcycle_dtype == ECS_F32;
  hipStream_t s = C->stream;
  const int64_t nn0 = nn_of(C);
  // the kernels read k^2 in FP64: an FP32 field is widened (exactly) once here
  if (C->k2_dtype == ECS_F32) {
    launch_widen_real(reinterpret_cast<const float *>(C->k2_user), C->k2_wide, nn0, s);
    C->k2 = C->k2_wide;
  } else {
    C->k2 = reinterpret_cast<const double *>(C->k2_user);
  }
  // operator scalars of M (Sec. 5)
  const ecs_prec_desc &P = C->prec;
  double lam0 = 0;
  if (P.kind == ECS_PREC_QD) {
    lam0 = std::fabs(P.re_lambda0);
    if (lam0 == 0) {
      launch_max_real(C->k2, nn0, C->dscal, C->dscal + kRedBlocks, s);
      HIP_OK(hipMemcpyAsync(C->pinned, C->dscal + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      lam0 = C->pinned[0];
      if (!(lam0 > 0)) return fail(C, ECS_EINVAL, "QD: max k^2 must be positive for the automatic |Re lambda0|");
    }
  }
  C->lam0 = lam0;
  switch (P.kind) {
    case ECS_PREC_NONE: C->alpha = 1.0; C->beta = -1.0; C->c = 0.0; break;
    case ECS_PREC_LAPLACE: C->alpha = 1.0; C->beta = 0.0; C->c = 0.0; break;
    case ECS_PREC_CSL: C->alpha = 1.0; C->beta = cd(P.beta1, P.beta2); C->c = 0.0; break;
    case ECS_PREC_CSG:  // every weight is homogeneous of degree -2 in the widths
      C->alpha = std::polar(1.0, -2.0 * P.theta_alpha); C->beta = -1.0; C->c = 0.0; break;
    case ECS_PREC_QD: C->alpha = 1.0 / lam0; C->beta = -1.0 / lam0; C->c = cd(1.0, -1.0); break;
    default: return fail(C, ECS_EINVAL, "unknown preconditioner kind");
  }
  // weights
  const HostLevel &F = C->hl[0];
  for (int a = 0; a < C->dim; a++) {
    ecs_status st;
    if ((st = upload_cx<double>(C, C->Acm[a], F.am[a], 1.0)) != ECS_OK) return st;
    if ((st = upload_cx<double>(C, C->Acp[a], F.ap[a], 1.0)) != ECS_OK) return st;
    if ((st = upload_cx<double>(C, C->Wd[a], F.w[a], 1.0)) != ECS_OK) return st;
    if (f32) {
      if ((st = upload_cx<float>(C, C->Acm32[a], F.am[a], 1.0)) != ECS_OK) return st;
      if ((st = upload_cx<float>(C, C->Acp32[a], F.ap[a], 1.0)) != ECS_OK) return st;
    }
  }
  for (int l = 0; l < C->nlev; l++) {
    const HostLevel &L = C->hl[l];
    for (int a = 0; a < C->dim; a++) {
      ecs_status st;
      if ((st = upload_cx<double>(C, C->L64[l].cm[a], L.am[a], C->alpha)) != ECS_OK) return st;
      if ((st = upload_cx<double>(C, C->L64[l].cp[a], L.ap[a], C->alpha)) != ECS_OK) return st;
      if (f32) {
        if ((st = upload_cx<float>(C, C->L32[l].cm[a], L.am[a], C->alpha)) != ECS_OK) return st;
        if ((st = upload_cx<float>(C, C->L32[l].cp[a], L.ap[a], C->alpha)) != ECS_OK) return st;
      }
    }
    // k^2 on level l: injection from the finest grid (rediscretisation, Sec. 4.2)
    if (l > 0) launch_inject_k2<double>(L.n[0], L.n[1], L.n[2], C->k2, F.n[0], F.n[1], C->L64[l].k2, s);
    if (f32) {
      if (l == 0) launch_cast_real(C->k2, C->L32[0].k2, L.nn, s);
      else launch_inject_k2<float>(L.n[0], L.n[1], L.n[2], C->k2, F.n[0], F.n[1], C->L32[l].k2, s);
    }
  }
  // coarsest dense inverse of M
  const int lc = C->nlev - 1;
  const HostLevel &Lc = C->hl[lc];
  std::vector<double> k2c(Lc.nn);
  const double *k2dev = lc == 0 ? C->k2 : C->L64[lc].k2;
  HIP_OK(hipMemcpyAsync(k2c.data(), k2dev, Lc.nn * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  std::vector<int> unk;
  std::vector<int64_t> pos(Lc.nn, -1);
  const int kz0 = C->dim == 3 ? 1 : 0, kz1 = C->dim == 3 ? Lc.n[2] - 1 : 1;
  for (int k = kz0; k < kz1; k++)
    for (int j = 1; j < Lc.n[1] - 1; j++)
      for (int i = 1; i < Lc.n[0] - 1; i++) {
        int64_t p = ((int64_t)k * Lc.n[1] + j) * Lc.n[0] + i;
        pos[p] = (int64_t)unk.size();
        unk.push_back((int)p);
      }
  const int nu = (int)unk.size();
  if (nu != C->nunk) return fail(C, ECS_EINVAL, "internal: coarse unknown count");
  std::vector<cd> M((size_t)nu * nu, 0.0);
  for (int r = 0; r < nu; r++) {
    int64_t p = unk[r];
    int ci[3] = {(int)(p % Lc.n[0]), (int)((p / Lc.n[0]) % Lc.n[1]), (int)(p / ((int64_t)Lc.n[0] * Lc.n[1]))};
    int64_t stride[3] = {1, Lc.n[0], (int64_t)Lc.n[0] * Lc.n[1]};
    cd diag = C->beta * k2c[p] + C->c;
    for (int a = 0; a < C->dim; a++) {
      cd am = C->alpha * Lc.am[a][ci[a]], ap = C->alpha * Lc.ap[a][ci[a]];
      diag += am + ap;
      int64_t qm = pos[p - stride[a]], qp = pos[p + stride[a]];
      if (qm >= 0) M[(size_t)r * nu + qm] -= am;
      if (qp >= 0) M[(size_t)r * nu + qp] -= ap;
    }
    M[(size_t)r * nu + r] += diag;
  }
  if (!invert(M, nu)) return fail(C, ECS_EINVAL, "coarsest preconditioner matrix is singular");
  {
    // the solve kernel reads the inverse column by column (transposed layout)
    std::vector<cd> MT((size_t)nu * nu);
    for (int r = 0; r < nu; r++)
      for (int q = 0; q < nu; q++) MT[(size_t)q * nu + r] = M[(size_t)r * nu + q];
    ecs_status st;
    if ((st = upload_cx<double>(C, C->minv64, MT, 1.0)) != ECS_OK) return st;
    if (f32 && (st = upload_cx<float>(C, C->minv32, MT, 1.0)) != ECS_OK) return st;
  }
  HIP_OK(hipMemcpy(C->unk, unk.data(), nu * sizeof(int), hipMemcpyHostToDevice));
  // pack of the levels that may form the one-workgroup tail of a general cycle
  C->sfirst = -1;
  C->gt_l = -1;
  C->skey[0] = -2;
  if (C->dim == 2 && C->nlev >= 2) {
    auto plen = [&](int l) { return 2 * C->hl[l].n[0] + 2 * C->hl[l].n[1] + (int)C->hl[l].nn; };
    int first = lc;
    int64_t nodes = Lc.nn;
    int len = plen(lc);
    while (first > 0 && C->hl[first - 1].n[0] <= kTailNodes && C->hl[first - 1].n[1] <= kTailNodes &&
           lc - (first - 1) + 1 <= kTailMaxLevels && nodes + C->hl[first - 1].nn <= kTailCap &&
           len + plen(first - 1) <= kSchedPack) {
      first--;
      nodes += C->hl[first].nn;
      len += plen(first);
    }
    if (first < lc) {
      std::vector<cd> pack;
      pack.reserve(len);
      for (int l = first; l <= lc; l++) {
        const HostLevel &L = C->hl[l];
        C->spko[l] = (int)pack.size();
        std::vector<double> k2l(L.nn);
        const double *src = l == 0 ? C->k2 : C->L64[l].k2;
        HIP_OK(hipMemcpyAsync(k2l.data(), src, L.nn * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        for (int a = 0; a < 2; a++) {
          for (int i = 0; i < L.n[a]; i++) pack.push_back(C->alpha * L.am[a][i]);
          for (int i = 0; i < L.n[a]; i++) pack.push_back(C->alpha * L.ap[a][i]);
        }
        for (int j = 0; j < L.n[1]; j++)
          for (int i = 0; i < L.n[0]; i++) {
            const bool in = i >= 1 && i <= L.n[0] - 2 && j >= 1 && j <= L.n[1] - 2;
            const cd dg = C->alpha * (L.am[0][i] + L.ap[0][i] + L.am[1][j] + L.ap[1][j]) +
                          C->beta * k2l[(size_t)j * L.n[0] + i] + C->c;
            pack.push_back(in ? 1.0 / dg : cd(0.0));
          }
      }
      C->spko[lc + 1] = (int)pack.size();
      ecs_status st;
      if ((st = upload_cx<double>(C, C->spack64, pack, 1.0)) != ECS_OK) return st;
      if (f32 && (st = upload_cx<float>(C, C->spack32, pack, 1.0)) != ECS_OK) return st;
      C->sfirst = first;
    }
  }
  // Krylov scalars start cleared
  HIP_OK(hipMemsetAsync(C->gs, 0, sizeof(GmresScalars), s));
  HIP_OK(hipMemsetAsync(C->bs, 0, kMaxRhs * sizeof(BicgScalars), s));
  HIP_OK(hipMemsetAsync(C->bs_in, 0, sizeof(BicgScalars), s));
  HIP_OK(hipStreamSynchronize(s));
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

// ----------------------------------------------------------- multigrid
// smoothing sweeps on level l, u in place (t = level scratch)
template <typename R>
void smooth(ecs_ctx *C, int l, const cplx<R> *b, cplx<R> *u, cplx<R> *t, int nsweeps, bool zero_guess) {
  Grid<R> g = grid_M<R>(C, l);
  const R om = (R)C->prec.omega;
  const int64_t nn = C->hl[l].nn;
  for (int q = 0; q < nsweeps; q++) {
    bool zg = zero_guess && q == 0;
    // algorithmic bytes of one sweep: read u, b, k^2, write u (a zero guess skips u)
    TimedScope ts(C, l == 0 ? kTSmooth : kTCoarse, (double)nn * sizeof(R) * (zg ? 5 : 7));
    if (C->prec.smoother == ECS_SMOOTH_JACOBI) {
      launch_jacobi<R>(g, b, u, t, om, zg, C->stream);
      (void)hipMemcpyAsync(u, t, nn * sizeof(cplx<R>), hipMemcpyDeviceToDevice, C->stream);
    } else {
      launch_rb_colour<R>(g, b, u, om, 0, zg, C->stream);
      launch_rb_colour<R>(g, b, u, om, 1, false, C->stream);
    }
  }
  if (nsweeps == 0 && zero_guess) launch_zero<R>(u, nn, C->stream);
}

template <typename R>
void coarse_solve(ecs_ctx *C, const cplx<R> *b, cplx<R> *x) {
  const HostLevel &L = C->hl[C->nlev - 1];
  launch_coarse_solve<R>(C->nunk, minv_of<R>(C), C->unk, L.n[0], L.n[1], L.n[2], b, x, C->stream);
}

// omega-Jacobi sweeps of Algorithm 1 on level l, alternating out of place
// between the iterate's buffer `cur` and `oth` (no copies); returns the
// buffer that holds the result
template <typename R>
cplx<R> *jacobi_sweeps(ecs_ctx *C, int l, const cplx<R> *b, cplx<R> *cur, cplx<R> *oth, int nsweeps,
                       bool zero_guess) {
  Grid<R> g = grid_M<R>(C, l);
  const int64_t nn = C->hl[l].nn;
  for (int q = 0; q < nsweeps; q++) {
    const bool zg = zero_guess && q == 0;
    TimedScope ts(C, l == 0 ? kTSmooth : kTCoarse, (double)nn * sizeof(R) * (zg ? 5 : 7));
    launch_jacobi<R>(g, b, cur, oth, (R)C->prec.omega, zg, C->stream);
    std::swap(cur, oth);
  }
  if (nsweeps == 0 && zero_guess) launch_zero<R>(cur, nn, C->stream);
  return cur;
}

template <typename R>
const cplx<R> *spack_of(const ecs_ctx *C);
template <>
const cplx<double> *spack_of<double>(const ecs_ctx *C) { return C->spack64; }
template <>
const cplx<float> *spack_of<float>(const ecs_ctx *C) { return C->spack32; }

// Algorithm 1 from tail level l to the coarsest in one launch, following the
// schedule unrolled for (gf, gc) and the guess
template <typename R>
void sched_tail(ecs_ctx *C, int l, const cplx<R> *b, cplx<R> *u, int gf, int gc, bool zero_guess) {
  const ecs_prec_desc &P = C->prec;
  const int lc = C->nlev - 1;
  SchedArgs<R> a{};
  a.nl = lc - l + 1;
  const int base = C->spko[l];
  for (int k = 0; k < a.nl; k++) {
    const HostLevel &L = C->hl[l + k];
    a.n0[k] = L.n[0];
    a.n1[k] = L.n[1];
    a.noff[k + 1] = a.noff[k] + (int)L.nn;
    a.pko[k] = C->spko[l + k] - base;
  }
  a.pko[a.nl] = C->spko[lc + 1] - base;
  a.pack = spack_of<R>(C) + base;
  a.pack_len = a.pko[a.nl];
  a.minvT = minv_of<R>(C);
  a.nunk = C->nunk;
  a.tpr = 64;
  while (a.tpr > 1 && a.tpr * C->nunk > 1024) a.tpr >>= 1;
  a.b_in = b;
  a.u_in = zero_guess ? nullptr : u;
  a.u_out = u;
  const int v = ((gf == P.gamma_f && gc == P.gamma_c) ? 0 : 2) + (zero_guess ? 0 : 1);
  a.prog = C->sprog + (size_t)v * kSchedProgCap;
  a.prog_len = C->sprog_len[v];
  a.omega = (R)P.omega;
  TimedScope ts(C, kTCoarse, 0.0);
  launch_sched_tail<R>(a, C->stream);
}

// Algorithm 1: u <- MG(l, M_l, b, u, nu1, nu2, C, gf, gc).  zero_guess: u == 0
// on entry (u's contents are not read and need not be cleared).  From the
// tail level on (2D, small levels) the rest of the recursion runs in one
// launch; above it each step is a launch, omega-Jacobi alternating between u
// and the level scratch t.
template <typename R>
void mg(ecs_ctx *C, int l, const cplx<R> *b, cplx<R> *u, int gf, int gc, bool zero_guess) {
  const int lc = C->nlev - 1;
  if (l == lc) {
    coarse_solve<R>(C, b, u);
    return;
  }
  if (l == C->gt_l) {
    sched_tail<R>(C, l, b, u, gf, gc, zero_guess);
    return;
  }
  DevLevel<R> &D = dev_level<R>(C, l);
  DevLevel<R> &Dc = dev_level<R>(C, l + 1);
  const bool jac = C->prec.smoother == ECS_SMOOTH_JACOBI;
  cplx<R> *cur = u;
  if (jac) cur = jacobi_sweeps<R>(C, l, b, u, D.t, C->prec.nu1, zero_guess);
  else smooth<R>(C, l, b, u, D.t, C->prec.nu1, zero_guess);
  {
    // read b, u, k^2, write the coarse residual
    const double per = 5.0 + 2.0 / (C->dim == 3 ? 8 : 4);
    TimedScope ts(C, l == 0 ? kTRestrict : kTCoarse, (double)C->hl[l].nn * sizeof(R) * per);
    launch_residual_restrict<R>(grid_M<R>(C, l), grid_M<R>(C, l + 1), b, cur, Dc.b, C->stream);
  }
  if (l + 1 == lc) {
    coarse_solve<R>(C, Dc.b, Dc.u);
  } else {
    for (int i = 1; i <= gc; i++) {
      if (i == 1) mg<R>(C, l + 1, Dc.b, Dc.u, gf, gc, true);
      else mg<R>(C, l + 1, Dc.b, Dc.u, gc, gf, false);
    }
  }
  const int nu2 = C->prec.nu2;
  if (jac && C->dim == 2 && nu2 >= 1 && (cur == u) == ((nu2 & 1) == 0)) {
    // correction fused with the first post-sweep (cur -> its other buffer);
    // the remaining out-of-place sweeps end in u
    cplx<R> *oth = cur == u ? D.t : u;
    {
      // read u, b, k^2, the coarse correction; write the swept iterate
      TimedScope ts(C, l == 0 ? kTProlong : kTCoarse, (double)C->hl[l].nn * sizeof(R) * (7.0 + 2.0 / 4));
      launch_prolong_jacobi<R>(grid_M<R>(C, l), grid_M<R>(C, l + 1), Dc.u, b, cur, oth, (R)C->prec.omega,
                               C->stream);
    }
    jacobi_sweeps<R>(C, l, b, oth, cur, nu2 - 1, false);
    return;
  }
  // the corrected iterate goes where an odd / even number of out-of-place
  // post-sweeps ends in u
  cplx<R> *dst = (jac && (nu2 & 1)) ? D.t : u;
  {
    // read u and the coarse correction, write u
    const double per = 4.0 + 2.0 / (C->dim == 3 ? 8 : 4);
    TimedScope ts(C, l == 0 ? kTProlong : kTCoarse, (double)C->hl[l].nn * sizeof(R) * per);
    launch_prolong_to<R>(grid_M<R>(C, l), grid_M<R>(C, l + 1), Dc.u, cur, dst, C->stream);
  }
  if (jac) jacobi_sweeps<R>(C, l, b, dst, dst == u ? D.t : u, C->prec.nu2, false);
  else smooth<R>(C, l, b, u, D.t, C->prec.nu2, false);
}

// V(1,1) red-black in 2D (the QD set-up of Sec. 4.2) runs on the fused
// kernels: one down and one up kernel per level.
bool fused_vcycle(const ecs_ctx *C) {
  const ecs_prec_desc &P = C->prec;
  return C->dim == 2 && P.smoother == ECS_SMOOTH_RBGS && P.nu1 == 1 && P.nu2 == 1 && P.gamma_f == 1 &&
         P.gamma_c == 1 && C->nlev > 1;
}

// Which kernel runs each level of the fused cycle: levels from lt on run in
// the single-workgroup tail; above it, pair_start[l] marks levels l, l+1 run
// by one two-level kernel; every other level has its own down and up kernel.
struct FusedPlan {
  int lt;
  bool pair_start[kMaxLev + 1];
};

FusedPlan fused_plan(const ecs_ctx *C) {
  const int lc = C->nlev - 1;
  const ecs_tuning &T = C->tune;
  FusedPlan P{};
  // first level handled by the tail: the coarsest levels that are small
  // (FP32 cycles: up to 65 nodes per axis in the wide tail; FP64: up to 33)
  const bool wide = C->prec.vcycle_dtype == ECS_F32;
  const int tn = wide ? T.tail_nodes : std::min(T.tail_nodes, kTailNodes);
  const int64_t cap = wide ? kTailWideCap : kTailCap;
  int lt = lc;
  int64_t tail_nn = C->hl[lc].nn, tail_w = std::max(C->hl[lc].n[0], C->hl[lc].n[1]);
  while (lt > 0 && C->hl[lt - 1].n[0] <= tn && C->hl[lt - 1].n[1] <= tn && lc - (lt - 1) + 1 <= kTailMaxLevels &&
         tail_nn + C->hl[lt - 1].nn <= cap &&
         tail_w + std::max(C->hl[lt - 1].n[0], C->hl[lt - 1].n[1]) <= (wide ? kTailWideWeights : 128)) {
    lt--;
    tail_nn += C->hl[lt].nn;
    tail_w += std::max(C->hl[lt].n[0], C->hl[lt].n[1]);
  }
  P.lt = lt;
  // the levels above the tail with at most pair_grid nodes per axis run two
  // per kernel, pairs counted from the tail up
  int ls = lt;
  while (ls > 0 && C->hl[ls - 1].n[0] <= T.pair_grid && C->hl[ls - 1].n[1] <= T.pair_grid) ls--;
  for (int l = lt - 2; l >= ls; l -= 2) P.pair_start[l] = true;
  return P;
}

// A Bi-CGSTAB (the nested FP32 one, or the outer one with the FP64 cycle) can
// form each cycle's right-hand side (its p and s updates) inside the finest
// level's down kernel when that level has one and the cycle is launched
// eagerly.
bool fused_updates(const ecs_ctx *C) {
  if (!C->tune.fuse_updates || !fused_vcycle(C) || C->graph_mode == ECS_GRAPHS_ALWAYS) return false;
  const FusedPlan P = fused_plan(C);
  return P.lt > 0 && !P.pair_start[0];
}

// Level buffers of the fused cycle: the hierarchy's own (one right-hand
// side), or for the batched solve arrays holding one copy per right-hand side
// slot, rhs_stride(level nodes) elements apart.
template <typename R>
struct CycleBufs {
  cplx<R> *b[kMaxLev] = {}, *t[kMaxLev] = {}, *u[kMaxLev] = {};
};

template <typename R>
CycleBufs<R> hierarchy_bufs(ecs_ctx *C) {
  CycleBufs<R> B;
  for (int l = 0; l < C->nlev; l++) {
    DevLevel<R> &D = dev_level<R>(C, l);
    B.b[l] = D.b;
    B.t[l] = D.t;
    B.u[l] = D.u;
  }
  return B;
}

// src (FP32, finest level by its own down kernel): the right-hand side b0 is
// formed by that kernel from src and stored in b0 == src->out.  cb / rs (the
// batched solve): the cycle of every right-hand side slot in rs at once, b0
// and u0 holding one vector per slot rhs_stride(nodes) apart.
template <typename R>
void vcycle_fused(ecs_ctx *C, const cplx<R> *b0, cplx<R> *u0, const DownSrc<R> *src = nullptr,
                  const CycleBufs<R> *cb = nullptr, const RhsSet &rs = one_rhs()) {
  const int lc = C->nlev - 1;
  const R om = (R)C->prec.omega;
  const ecs_tuning &T = C->tune;
  const FusedPlan plan = fused_plan(C);
  const int lt = plan.lt;
  const bool *pair_start = plan.pair_start;
  const CycleBufs<R> B = cb ? *cb : hierarchy_bufs<R>(C);
  const double nr = rs.count;  // algorithmic bytes scale with the right-hand sides of a launch
  auto small = [&](int l) { return C->hl[l].n[0] <= T.small_grid && C->hl[l].n[1] <= T.small_grid; };
  for (int l = 0; l < lt;) {
    const cplx<R> *b = l == 0 ? b0 : B.b[l];
    if (l == 0 && src) {
      // reads the vectors b is formed from (r, p, v or r, v) and k^2;
      // writes b and the coarse residual
      const bool pm = src->mode == kDownSrcP;
      TimedScope ts(C, pm ? kTDownP : kTDownS, (double)C->hl[0].nn * sizeof(R) * (pm ? 9.5 : 7.5));
      launch_down_rb_src<R>(grid_M<R>(C, 0), grid_M<R>(C, 1), *src, B.b[1], om, small(0) ? 2 : T.down_rows,
                            C->stream);
      l++;
      continue;
    }
    if (pair_start[l]) {
      // reads b, k^2 of both levels; writes u of both, b of level l+1, the
      // residual restricted to level l+2
      TimedScope ts(C, kTCoarse, nr * (C->hl[l].nn + C->hl[l + 1].nn) * sizeof(R) * 5.5);
      launch_down2_rb<R>(grid_M<R>(C, l), grid_M<R>(C, l + 1), grid_M<R>(C, l + 2), b, B.t[l], B.b[l + 1],
                         B.t[l + 1], B.b[l + 2], om, C->stream, rs);
      l += 2;
      continue;
    }
    // reads b, k^2; writes the coarse residual (3.5 reals per node)
    TimedScope ts(C, l == 0 ? kTDown : kTCoarse, nr * C->hl[l].nn * sizeof(R) * 3.5);
    launch_down_rb<R>(grid_M<R>(C, l), grid_M<R>(C, l + 1), b, B.b[l + 1], om, small(l) ? 2 : T.down_rows,
                      C->stream, rs);
    l++;
  }
  if (lt == lc) {
    // no small levels above the coarsest: dense solve only
    const cplx<R> *b = lc == 0 ? b0 : B.b[lc];
    cplx<R> *u = lc == 0 ? u0 : B.u[lc];
    TimedScope ts(C, kTCoarse, 0.0);
    const HostLevel &L = C->hl[lc];
    launch_coarse_solve<R>(C->nunk, minv_of<R>(C), C->unk, L.n[0], L.n[1], L.n[2], b, u, C->stream, rs);
  } else {
    TailArgs<R> a{};
    a.nl = lc - lt + 1;
    a.noff[0] = a.woff[0] = a.poff[0] = 0;
    for (int k = 0; k < a.nl; k++) {
      const int l = lt + k;
      a.g[k] = grid_M<R>(C, l);
      a.noff[k + 1] = a.noff[k] + (int)C->hl[l].nn;
      a.poff[k + 1] = a.poff[k] + ((int)C->hl[l].nn + 63) / 64 * 64;
      a.woff[k + 1] = a.woff[k] + (int)std::max(C->hl[l].n[0], C->hl[l].n[1]);
    }
    a.b0 = lt == 0 ? b0 : B.b[lt];
    a.u0 = lt == 0 ? u0 : B.u[lt];
    a.minvT = minv_of<R>(C);
    a.nunk = C->nunk;
    a.tpr = 64;
    while (a.tpr > 1 && a.tpr * C->nunk > 1024) a.tpr >>= 1;
    a.omega = om;
    TimedScope ts(C, kTCoarse, 0.0);
    launch_tail<R>(a, C->stream, rs);
  }
  for (int l = lt - 1; l >= 0;) {
    if (l >= 1 && pair_start[l - 1]) {
      // levels l - 1 and l: reads u, b, k^2 of both and the correction from
      // level l + 1; writes u of level l - 1
      const int lf = l - 1;
      const cplx<R> *b = lf == 0 ? b0 : B.b[lf];
      cplx<R> *out = lf == 0 ? u0 : B.u[lf];
      TimedScope ts(C, kTCoarse, nr * (C->hl[lf].nn + C->hl[lf + 1].nn) * sizeof(R) * 7.5);
      launch_up2_rb<R>(grid_M<R>(C, lf), grid_M<R>(C, lf + 1), grid_M<R>(C, lf + 2), b, B.t[lf], B.b[lf + 1],
                       B.t[lf + 1], B.u[lf + 2], out, om, C->stream, rs);
      l -= 2;
      continue;
    }
    const cplx<R> *b = l == 0 ? b0 : B.b[l];
    cplx<R> *out = l == 0 ? u0 : B.u[l];
    // reads the coarse correction, b, k^2; writes u (5.5 reals per node)
    TimedScope ts(C, l == 0 ? kTUp : kTCoarse, nr * C->hl[l].nn * sizeof(R) * 5.5);
    launch_up_rb<R>(grid_M<R>(C, l), grid_M<R>(C, l + 1), b, B.u[l + 1], out, om, small(l) ? 4 : T.up_rows,
                    C->stream, rs);
    l--;
  }
}

void drop_graphs(ecs_ctx *C) {
  for (auto &g : C->graphs) (void)hipGraphExecDestroy(g.exec);
  C->graphs.clear();
}

// launches of one general cycle (capped): cycles with very many coarse
// visits (large gamma over many levels) are not captured
int64_t cycle_launches(const ecs_ctx *C, int l, int gf, int gc, int64_t cap) {
  const int lc = C->nlev - 1;
  if (l == lc || l == C->gt_l) return 1;
  int64_t n = C->prec.nu1 + C->prec.nu2 + 2;
  if (l + 1 == lc) return n + 1;
  for (int i = 1; i <= gc && n < cap; i++)
    n += i == 1 ? cycle_launches(C, l + 1, gf, gc, cap) : cycle_launches(C, l + 1, gc, gf, cap);
  return n;
}

// A general cycle is several launches per level, most of them a few
// microseconds of work on the coarse levels, so host launch overhead would
// dominate: the whole cycle is captured once per (input, output) pair and
// replayed as one graph launch.  The fused cycle is about two launches per
// level; there the device-side completion of a graph launch (about 12 us
// before the next kernel on the stream) costs more than the host launches it
// saves, so the automatic mode launches it eagerly.  Per-kernel timing needs
// eager launches, so graphs are bypassed while any cycle timer is on.
// Returns false when the caller should launch the cycle eagerly.
template <typename R>
bool vcycle_graph(ecs_ctx *C, const cplx<R> *b0, cplx<R> *u0) {
  for (int k : {kTSmooth, kTCoarse, kTRestrict, kTProlong, kTDown, kTUp, kTDownP, kTDownS})
    if (C->timers[k].on) return false;
  if (C->graph_mode == ECS_GRAPHS_NEVER || C->no_alloc) return false;
  if (fused_vcycle(C)) {
    if (C->graph_mode == ECS_GRAPHS_AUTO) return false;
  } else if (cycle_launches(C, 0, C->prec.gamma_f, C->prec.gamma_c, 4096) >= 4096) {
    return false;
  }
  for (auto &g : C->graphs)
    if (g.b == b0 && g.u == u0 && g.real_bytes == (int)sizeof(R))
      return hipGraphLaunch(g.exec, C->stream) == hipSuccess;
  if (!C->capture && hipStreamCreateWithFlags(&C->capture, hipStreamNonBlocking) != hipSuccess) {
    C->capture = nullptr;
    return false;
  }
  if (C->graphs.size() >= 256) drop_graphs(C);
  if (hipStreamBeginCapture(C->capture, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
  hipStream_t user = C->stream;
  C->stream = C->capture;
  if (fused_vcycle(C)) vcycle_fused<R>(C, b0, u0);
  else mg<R>(C, 0, b0, u0, C->prec.gamma_f, C->prec.gamma_c, true);
  C->stream = user;
  hipGraph_t graph = nullptr;
  if (hipStreamEndCapture(C->capture, &graph) != hipSuccess || !graph) return false;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return false;
  C->graphs.push_back({b0, u0, (int)sizeof(R), exec});
  return hipGraphLaunch(exec, C->stream) == hipSuccess;
}

// Unrolls Algorithm 1 from tail level k (0 = the tail's first level) into the
// operations of k_sched_tail, tracking which of the two LDS buffers of each
// level holds its iterate (omega-Jacobi alternates; red-black stays in place).
struct SchedGen {
  const ecs_prec_desc *P;
  int nl;
  int cur[kTailMaxLevels] = {};
  std::vector<uint32_t> ops;
  bool overflow = false;

  void emit(uint32_t code, int k, bool zg, int f0, int f1) {
    if (ops.size() >= (size_t)kSchedProgCap) {
      overflow = true;
      return;
    }
    ops.push_back(code | (uint32_t)k << 4 | (uint32_t)zg << 8 | (uint32_t)f0 << 9 | (uint32_t)f1 << 10);
  }
  void smooth(int k, int nsweeps, bool zero_guess) {
    for (int q = 0; q < nsweeps; q++) {
      const bool zg = zero_guess && q == 0;
      if (P->smoother == ECS_SMOOTH_JACOBI) {
        emit(kSchedJacobi, k, zg, cur[k], cur[k] ^ 1);
        cur[k] ^= 1;
      } else {
        emit(kSchedRB, k, zg, cur[k], 0);
        emit(kSchedRB, k, false, cur[k], 1);
      }
    }
    if (nsweeps == 0 && zero_guess) emit(kSchedZero, k, false, cur[k], 0);
  }
  void cycle(int k, int gf, int gc, bool zero_guess) {
    const int last = nl - 1;
    if (overflow) return;
    if (k == last) {
      emit(kSchedCoarse, k, false, cur[k], 0);
      return;
    }
    smooth(k, P->nu1, zero_guess);
    emit(kSchedResid, k, false, cur[k], 0);
    if (k + 1 == last) {
      emit(kSchedCoarse, k + 1, false, cur[k + 1], 0);
    } else {
      for (int i = 1; i <= gc && !overflow; i++) {
        if (i == 1) cycle(k + 1, gf, gc, true);
        else cycle(k + 1, gc, gf, false);
      }
    }
    emit(kSchedProlong, k, false, cur[k], cur[k + 1]);
    smooth(k, P->nu2, false);
  }
};

// Loads the schedules of the general cycle's tail for the current set-up
// (outside any capture: it may copy to the device and drops the graphs that
// replay older schedules).
void ensure_sched(ecs_ctx *C) {
  const ecs_prec_desc &P = C->prec;
  const int lc = C->nlev - 1;
  int lt = -1;
  if (C->sfirst >= 0) {
    lt = lc;
    const int tn = std::min(C->tune.tail_nodes, kTailNodes);  // the schedule tail holds up to 33^2 levels
    while (lt - 1 >= C->sfirst && C->hl[lt - 1].n[0] <= tn && C->hl[lt - 1].n[1] <= tn)
      lt--;
    if (lt == lc) lt = -1;
  }
  const int key[6] = {lt, P.gamma_f, P.gamma_c, P.nu1, P.nu2, P.smoother};
  if (std::memcmp(key, C->skey, sizeof key) == 0) return;
  std::memcpy(C->skey, key, sizeof key);
  C->gt_l = -1;
  drop_graphs(C);
  if (lt < 0) return;
  std::vector<uint32_t> progs[4];
  for (int v = 0; v < 4; v++) {
    SchedGen G;
    G.P = &P;
    G.nl = lc - lt + 1;
    const bool swap = v >= 2;
    G.cycle(0, swap ? P.gamma_c : P.gamma_f, swap ? P.gamma_f : P.gamma_c, (v & 1) == 0);
    G.emit(kSchedEnd, 0, false, G.cur[0], 0);
    if (G.overflow) return;  // too long: the per-level launches stay in use
    progs[v].swap(G.ops);
  }
  for (int v = 0; v < 4; v++) {
    if (hipMemcpyAsync(C->sprog + (size_t)v * kSchedProgCap, progs[v].data(), progs[v].size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, C->stream) != hipSuccess)
      return;
    C->sprog_len[v] = (int)progs[v].size();
  }
  if (hipStreamSynchronize(C->stream) != hipSuccess) return;
  C->gt_l = lt;
}

// z = M^{-1} v approximately: one cycle from zero on the finest level
template <typename R>
void vcycle(ecs_ctx *C, const cplx<R> *b0, cplx<R> *u0) {
  if (C->nlev == 1) {
    coarse_solve<R>(C, b0, u0);
    return;
  }
  if (!fused_vcycle(C)) ensure_sched(C);
  if (vcycle_graph<R>(C, b0, u0)) return;
  if (fused_vcycle(C)) vcycle_fused<R>(C, b0, u0);
  else mg<R>(C, 0, b0, u0, C->prec.gamma_f, C->prec.gamma_c, true);
}

// preconditioner application from an FP64 vector into the cycle's dtype
template <typename RZ>
void precond(ecs_ctx *C, const cplx<double> *v, cplx<RZ> *z);
template <>
void precond<double>(ecs_ctx *C, const cplx<double> *v, cplx<double> *z) {
  if (C->prec.kind == ECS_PREC_NONE) {
    (void)hipMemcpyAsync(z, v, nn_of(C) * sizeof(cplx<double>), hipMemcpyDeviceToDevice, C->stream);
    return;
  }
  vcycle<double>(C, v, z);
}
template <>
void precond<float>(ecs_ctx *C, const cplx<double> *v, cplx<float> *z) {
  cplx<float> *b0 = C->L32[0].b;
  launch_cast<double, float>(v, b0, nn_of(C), C->stream);
  vcycle<float>(C, b0, z);
}

// ----------------------------------------------------------- Krylov
// copy `bytes` (<= 64) from device memory into the pinned buffer and wait
bool read_bytes(ecs_ctx *C, const void *dev, size_t bytes) {
  if (hipMemcpyAsync(C->pinned, dev, bytes, hipMemcpyDeviceToHost, C->stream) != hipSuccess) return false;
  return hipStreamSynchronize(C->stream) == hipSuccess;
}

double read_scalar(ecs_ctx *C, const double *dev) {
  if (hipMemcpyAsync(C->pinned, dev, sizeof(double), hipMemcpyDeviceToHost, C->stream) != hipSuccess) return NAN;
  if (hipStreamSynchronize(C->stream) != hipSuccess) return NAN;
  return C->pinned[0];
}

template <typename R>
Grid<R> grid_A_of(const ecs_ctx *C);
template <>
Grid<double> grid_A_of<double>(const ecs_ctx *C) { return grid_A(C); }
template <>
Grid<float> grid_A_of<float>(const ecs_ctx *C) { return grid_A32(C); }

// Bi-CGSTAB in the cycle's dtype around the cycle, `iters` iterations from
// x = 0, all on the device: the nested preconditioner of FGMRES (complex FP32
// in the mixed form; FP64 gives the same algorithm at full precision)
template <typename R>
void inner_bicgstab(ecs_ctx *C, const KrylovBufs &K, const cplx<double> *v, cplx<R> *x, int iters) {
  const int64_t n = nn_of(C);
  hipStream_t s = C->stream;
  BicgScalars *S = C->bs_in;
  cplx<R> *fr = reinterpret_cast<cplx<R> *>(K.fr), *frh = reinterpret_cast<cplx<R> *>(K.frh);
  cplx<R> *fv = reinterpret_cast<cplx<R> *>(K.fv), *fs = reinterpret_cast<cplx<R> *>(K.fs);
  cplx<R> *ft = reinterpret_cast<cplx<R> *>(K.ft);
  cplx<R> *const ph0 = reinterpret_cast<cplx<R> *>(K.fph), *const sh0 = reinterpret_cast<cplx<R> *>(K.fsh);
  if constexpr (sizeof(R) == 4) launch_cast<double, float>(v, fr, n, s);
  else (void)hipMemcpyAsync(fr, v, n * sizeof(cplx<R>), hipMemcpyDeviceToDevice, s);
  (void)hipMemcpyAsync(frh, fr, n * sizeof(cplx<R>), hipMemcpyDeviceToDevice, s);
  launch_zero<R>(x, n, s);
  launch_zero<R>(reinterpret_cast<cplx<R> *>(K.fp), n, s);
  launch_zero<R>(fv, n, s);
  launch_pairdot<R>(fr, fr, nullptr, nullptr, 1, n, C->partials, S, kBicgInit, s);
  const Grid<R> gA = grid_A_of<R>(C);
  // fused (FP32): the finest down kernel forms p (into the other p buffer:
  // blocks read the old p around their tiles) and s; the same values either way
  const bool fuse = sizeof(R) == 4 && fused_updates(C);
  cplx<R> *p_old = reinterpret_cast<cplx<R> *>(K.fp), *p_new = reinterpret_cast<cplx<R> *>(K.fp2);
  // x = sum of alpha_i p^_i + omega_i s^_i: each step keeps its p^, s^ and
  // scalars, and x is updated once per K.fdefer steps (the same values as
  // a one-step update, in half its traffic per step)
  for (int it = 0; it < iters; it++) {
    const int slot = it % K.fdefer;
    cplx<R> *fph = ph0 + (int64_t)slot * K.ld, *fsh = sh0 + (int64_t)slot * K.ld;
    if (fuse) {
      const DownSrc<R> sp{kDownSrcP, fr, p_old, fv, p_new, S};
      vcycle_fused<R>(C, p_new, fph, &sp);
      std::swap(p_old, p_new);
    } else {
      launch_bicg_p<R>(p_old, fr, fv, n, S, s);
      vcycle<R>(C, p_old, fph);
    }
    launch_apply_dot<R, R>(gA, fph, fv, frh, kBicgAlpha, C->partials, S, s);
    if (fuse) {
      const DownSrc<R> ss{kDownSrcS, fr, nullptr, fv, fs, S};
      vcycle_fused<R>(C, fs, fsh, &ss);
    } else {
      launch_bicg_s<R>(fs, fr, fv, n, S, s);
      vcycle<R>(C, fs, fsh);
    }
    launch_apply_dot<R, R>(gA, fsh, ft, fs, kBicgOmega, C->partials, S, s);
    launch_bicg_r<R>(fr, fs, ft, frh, n, C->partials, S, K.fcoef + 2 * slot, s);
    if (slot == K.fdefer - 1 || it == iters - 1) launch_bicg_xdefer<R>(x, ph0, sh0, K.ld, slot + 1, K.fcoef, n, s);
  }
}

// Arnoldi step j (Sec. 5's GMRES): h = V_{0..j}^H w, w -= V h, ||w||^2 into
// S->nrm2, classical Gram-Schmidt with the multi-dot and multi-update kernels.
// A second pass h2 = V^H w, w -= V h2, H(:, j) += h2 restores the
// orthogonality that one classical pass loses under cancellation: always
// (ECS_ORTH_CGS2), never (ECS_ORTH_CGS1), or when ||w'|| < ||w|| / sqrt(2)
// after the first pass (ECS_ORTH_CGS2_SELECTIVE, decided on the device: the
// gated kernels of the second pass exit at once otherwise).  w is the basis
// column V_{j+1}, so one more multi-dot column gives ||w||^2.
// ECS_ORTH_DCGS2 delays the second pass by one step (Gram-Schmidt with
// delayed reorthogonalisation): v_j enters step j after one pass and its
// normalisation, and its second pass shares the multi-dot and the update pass
// with w's first, so the two passes cost what one does.  The corrections
// H(0..j-1, j-1) += h_{j,j-1} s and h_{j,j-1} *= nu of the column already
// rotated are left out; they are of the size of the first pass's rounding
// error (|s| = O(eps ||w|| / ||w'||)), so the least-squares problem and its
// residual estimate change only at that level (the stopping test and every
// restart use the true residual).  z_j = M^{-1} v_j is taken before v_j's
// second pass: FGMRES accepts any z_j, and for GMRES the mismatch is of the
// same size.
void orthogonalise(ecs_ctx *C, cplx<double> *V, int64_t ld, int j, cplx<double> *w, int64_t n,
                   cplx<double> *partials, GmresScalars *S, int m, int orth, hipStream_t s) {
  cplx<double> *h = S->H + (int64_t)j * (m + 1);
  if (orth == ECS_ORTH_DCGS2) {
    cplx<double> *vj = V + (int64_t)j * ld;
    {
      TimedScope ts(C, kTMdot, (double)n * 16 * (j + 2));  // read v_0..v_{j-1}, v_j, w
      launch_mdot2_partial(V, ld, j, vj, w, n, partials, s);
    }
    launch_reduce_cols(partials, n, 2 * j + 2, S->d2, s);
    {
      TimedScope ts(C, kTMupdate, (double)n * 16 * (j + (j > 0 ? 4 : 3)));  // read v_0..v_j, w; write v_j, w
      launch_mupdate2_partial(V, ld, j, S->d2, vj, w, n, partials, h, s);
    }
    launch_reduce_cols(partials, n, 1, &S->nrm2, s);
    return;
  }
  const bool sel = orth == ECS_ORTH_CGS2_SELECTIVE;
  const int nc = j + 1 + (sel ? 1 : 0);
  {
    TimedScope ts(C, kTMdot, (double)n * 16 * (nc + 1));  // read v_0..v_j (and w as a column) and w
    launch_mdot_partial<double, double>(V, ld, nc, w, n, partials, s);
  }
  launch_reduce_cols(partials, n, nc, h, s);
  {
    TimedScope ts(C, kTMupdate, (double)n * 16 * (j + 3));  // read v_0..v_j, w; write w
    launch_mupdate_partial(V, ld, j + 1, h, w, n, partials, s);
  }
  launch_reduce_cols(partials, n, 1, &S->nrm2, s);
  if (orth == ECS_ORTH_CGS1) return;
  const int *gate = nullptr;
  if (sel) {
    launch_reorth_gate(S, j, m, 0.5, s);
    gate = &S->reorth;
  }
  launch_mdot_partial<double, double>(V, ld, j + 1, w, n, partials, s, gate);
  launch_reduce_cols(partials, n, j + 1, S->h2, s, gate);
  launch_mupdate_partial(V, ld, j + 1, S->h2, w, n, partials, s, gate);
  launch_reduce_cols(partials, n, 1, &S->nrm2, s, gate);
  launch_add_h2(S, j, m, s, gate);
}

// second Gram-Schmidt passes of a solve: counted on the device when selective
// (read through the context's pinned buffer on its stream); with the delayed
// pass every step but the first of a cycle reorthogonalises its basis vector
int64_t reorth_passes(ecs_ctx *C, GmresScalars *S, int orth, int64_t iterations, int64_t later_steps) {
  if (orth == ECS_ORTH_CGS1) return 0;
  if (orth == ECS_ORTH_CGS2) return iterations;
  if (orth == ECS_ORTH_DCGS2) return later_steps;
  int cnt = -1;
  if (read_bytes(C, &S->reorth_count, sizeof(int))) std::memcpy(&cnt, C->pinned, sizeof(int));
  return cnt;
}

template <typename RZ>
ecs_status gmres(ecs_ctx *C, const ecs_solve_desc *d, const KrylovBufs &K, const cplx<double> *b, cplx<double> *x,
                 ecs_stats *st) {
  const int64_t n = nn_of(C);
  const int m = d->restart;
  const bool flexible = d->krylov == ECS_KRYLOV_FGMRES;
  hipStream_t s = C->stream;
  GmresScalars *S = C->gs;
  const int64_t ld = K.ld;
  cplx<RZ> *Z = reinterpret_cast<cplx<RZ> *>(K.Z);
  cplx<RZ> *tz = reinterpret_cast<cplx<RZ> *>(K.tz);
  const cplx<double> one = mk<double>(1, 0);
  HIP_OK(hipMemcpyAsync(&S->one, &one, sizeof(one), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemsetAsync(&S->reorth_count, 0, sizeof(int), s));
  launch_nrm2sq<double>(b, n, C->partials, &S->nrm2, s);
  const double bn2 = read_scalar(C, &S->nrm2.re);
  const double bnorm = std::sqrt(bn2);
  if (!(bnorm == bnorm) || std::isinf(bnorm)) return fail(C, ECS_EBREAKDOWN, "right-hand side contains NaN/Inf");
  if (bnorm == 0) {
    launch_zero<double>(x, n, s);
    st->rel_residual = 0;
    return ECS_OK;
  }
  HIP_OK(hipMemcpyAsync(&S->bnorm, &bnorm, sizeof(double), hipMemcpyHostToDevice, s));
  if (d->inner > 0) {  // the inner iteration has no stopping test: unit reference norm
    const double unit = 1.0;
    HIP_OK(hipMemcpyAsync(&C->bs_in->bnorm, &unit, sizeof(double), hipMemcpyHostToDevice, s));
    // bad and breakdowns (adjacent): inner runs cut short are counted as each
    // new run starts
    HIP_OK(hipMemsetAsync(&C->bs_in->bad, 0, 2 * sizeof(int), s));
  }
  if (!d->x_is_guess) launch_zero<double>(x, n, s);
  int it = 0;
  int64_t later_steps = 0;
  ecs_status status = ECS_NOT_CONVERGED;
  for (;;) {
    {
      TimedScope ts(C, kTApply, (double)n * 56);
      launch_residual<double>(grid_A(C), b, x, K.V, s);
    }
    launch_nrm2sq<double>(K.V, n, C->partials, &S->nrm2, s);
    launch_gmres_start(S, m, s);
    launch_scale_dev(K.V, n, &S->inv, s);
    double rt = read_scalar(C, &S->resid_true);
    st->rel_residual = rt;
    if (!(rt == rt) || std::isinf(rt)) {
      status = fail(C, ECS_EBREAKDOWN, "GMRES: residual is NaN/Inf");
      break;
    }
    if (rt <= d->rtol) { status = ECS_OK; break; }
    if (it >= d->maxit) { status = ECS_NOT_CONVERGED; break; }
    int k = 0;
    bool bad = false;
    for (int j = 0; j < m && it < d->maxit; j++) {
      cplx<double> *vj = K.V + (int64_t)j * ld;
      cplx<double> *w = K.V + (int64_t)(j + 1) * ld;
      cplx<RZ> *zj = flexible ? Z + (int64_t)j * ld : tz;
      if (d->inner > 0) inner_bicgstab<RZ>(C, K, vj, zj, d->inner);
      else precond<RZ>(C, vj, zj);
      st->vcycles += d->inner > 0 ? 2 * d->inner : 1;
      st->inner_iterations += d->inner;
      {
        TimedScope ts(C, kTApply, (double)n * (2 * sizeof(RZ) + 24));
        launch_apply<double, RZ, double>(grid_A(C), zj, w, s);
      }
      orthogonalise(C, K.V, ld, j, w, n, C->partials, S, m, d->orth, s);
      later_steps += j > 0;
      launch_gmres_givens(S, j, m, s);
      launch_scale_dev(w, n, &S->inv, s);
      it++;
      k = j + 1;
      // est, resid_true, bad, happy are contiguous: one readback per iteration
      if (!read_bytes(C, &S->est, 2 * sizeof(double) + 2 * sizeof(int))) { bad = true; break; }
      double est;
      int happy;
      std::memcpy(&est, C->pinned, sizeof(double));
      std::memcpy(&happy, reinterpret_cast<char *>(C->pinned) + 2 * sizeof(double) + sizeof(int), sizeof(int));
      if (d->history && it - 1 < d->history_len) d->history[it - 1] = est;
      if (!(est == est) || std::isinf(est)) { bad = true; break; }
      if (est <= d->rtol || happy) break;
    }
    if (bad) {
      status = fail(C, ECS_EBREAKDOWN, "GMRES: Givens residual estimate is NaN/Inf");
      break;
    }
    launch_gmres_backsolve(S, k, m, s);
    if (flexible) {
      launch_lincomb<RZ>(Z, ld, k, S->y, x, n, s);
    } else {
      launch_zero<double>(K.t, n, s);
      launch_lincomb<double>(K.V, ld, k, S->y, K.t, n, s);
      precond<RZ>(C, K.t, tz);
      st->vcycles++;
      launch_lincomb<RZ>(tz, ld, 1, &S->one, x, n, s);
    }
    st->restarts++;
  }
  st->iterations = it;
  st->reorthogonalisations = reorth_passes(C, S, d->orth, it, later_steps);
  if (d->inner > 0) {
    // the runs counted at their successors' starts, and the last run's flag
    int v[2] = {0, -1};
    if (read_bytes(C, &C->bs_in->bad, 2 * sizeof(int))) std::memcpy(v, C->pinned, sizeof v);
    st->inner_breakdowns = v[1] < 0 ? -1 : v[0] + v[1];
  }
  HIP_OK(hipGetLastError());
  return status;
}

ecs_status check_ready(ecs_ctx *C) {
  if (!C) return ECS_EINVAL;
  if (!C->ready) return fail(C, ECS_ESTATE, "call ecs_set_workspace after ecs_set_k2 and ecs_set_precond");
  return ECS_OK;
}

// Bi-CGSTAB building blocks (right-preconditioned, van der Vorst; Sec. 5),
// shared by the single solve and the batched driver.  Every scalar stays in
// device memory (C->bs); the host only reads {est, bad} after each step.

// r = b - A x, the restart scalars (est = ||r|| / ||b||, rho = ||r||^2,
// beta = 0), r^ = r, p = v = 0
void bicg_enqueue_restart(ecs_ctx *C, const KrylovBufs &K, const cplx<double> *b, const cplx<double> *x) {
  const int64_t n = nn_of(C);
  hipStream_t s = C->stream;
  {
    TimedScope ts(C, kTApply, (double)n * 56);
    launch_residual<double>(grid_A(C), b, x, K.r, s);
  }
  launch_pairdot<double>(K.r, K.r, nullptr, nullptr, 1, n, C->partials, C->bs, kBicgInit, s);
  (void)hipMemcpyAsync(K.rh, K.r, n * sizeof(cplx<double>), hipMemcpyDeviceToDevice, s);
  launch_zero<double>(K.p, n, s);
  launch_zero<double>(K.v, n, s);
  C->bicg_pflip = 0;
}

// one iteration: p = r + beta (p - omega v); ph = M^{-1} p; v = A ph -> alpha;
// s = r - alpha v; sh = M^{-1} s; t = A sh -> omega; x += alpha ph + omega sh;
// r = s - omega t -> est and the next beta.  With the FP64 cycle the p and s
// updates can run inside the finest down kernel (as in the nested FP32
// Bi-CGSTAB): the same values, two launches and two vector passes fewer; p
// then alternates between two buffers (blocks read the old p around their
// tiles while others write the new one).
template <typename RZ>
void bicg_enqueue_step(ecs_ctx *C, const KrylovBufs &K, cplx<double> *x) {
  const int64_t n = nn_of(C);
  hipStream_t s = C->stream;
  BicgScalars *S = C->bs;
  cplx<RZ> *ph = reinterpret_cast<cplx<RZ> *>(K.ph);
  cplx<RZ> *sh = reinterpret_cast<cplx<RZ> *>(K.sh);
  bool fuse = false;
  if constexpr (sizeof(RZ) == 8) fuse = K.p2 && fused_updates(C);
  if (fuse) {
    if constexpr (sizeof(RZ) == 8) {
      cplx<double> *p_old = C->bicg_pflip ? K.p2 : K.p, *p_new = C->bicg_pflip ? K.p : K.p2;
      const DownSrc<double> sp{kDownSrcP, K.r, p_old, K.v, p_new, S};
      vcycle_fused<double>(C, p_new, ph, &sp);
      C->bicg_pflip ^= 1;
    }
  } else {
    launch_bicg_p<double>(K.p, K.r, K.v, n, S, s);
    precond<RZ>(C, K.p, ph);
  }
  {
    TimedScope ts(C, kTApply, (double)n * (2 * sizeof(RZ) + 40));
    launch_apply_dot<double, RZ>(grid_A(C), ph, K.v, K.rh, kBicgAlpha, C->partials, S, s);
  }
  if (fuse) {
    if constexpr (sizeof(RZ) == 8) {
      const DownSrc<double> ss{kDownSrcS, K.r, nullptr, K.v, K.s, S};
      vcycle_fused<double>(C, K.s, sh, &ss);
    }
  } else {
    launch_bicg_s<double>(K.s, K.r, K.v, n, S, s);
    precond<RZ>(C, K.s, sh);
  }
  {
    TimedScope ts(C, kTApply, (double)n * (2 * sizeof(RZ) + 40));
    launch_apply_dot<double, RZ>(grid_A(C), sh, K.tt, K.s, kBicgOmega, C->partials, S, s);
  }
  launch_bicg_xr<double, RZ>(x, ph, sh, K.r, K.s, K.tt, K.rh, n, C->partials, S, s);
}

// {est, bad} of the Bi-CGSTAB scalars into the pinned buffer (async)
void bicg_enqueue_readback(ecs_ctx *C) {
  (void)hipMemcpyAsync(C->pinned, &C->bs->est, sizeof(double) + sizeof(int), hipMemcpyDeviceToHost, C->stream);
}
void bicg_take_readback(const ecs_ctx *C, double *est, int *bad) {
  std::memcpy(est, C->pinned, sizeof(double));
  std::memcpy(bad, reinterpret_cast<const char *>(C->pinned) + sizeof(double), sizeof(int));
}

template <typename RZ>
ecs_status bicgstab(ecs_ctx *C, const ecs_solve_desc *d, const KrylovBufs &K, const cplx<double> *b, cplx<double> *x,
                    ecs_stats *st) {
  const int64_t n = nn_of(C);
  hipStream_t s = C->stream;
  BicgScalars *S = C->bs;
  launch_nrm2sq<double>(b, n, C->partials, &C->gs->nrm2, s);
  const double bnorm = std::sqrt(read_scalar(C, &C->gs->nrm2.re));
  if (!(bnorm == bnorm) || std::isinf(bnorm)) return fail(C, ECS_EBREAKDOWN, "right-hand side contains NaN/Inf");
  if (bnorm == 0) {
    launch_zero<double>(x, n, s);
    st->rel_residual = 0;
    return ECS_OK;
  }
  HIP_OK(hipMemcpyAsync(&S->bnorm, &bnorm, sizeof(double), hipMemcpyHostToDevice, s));
  if (!d->x_is_guess) launch_zero<double>(x, n, s);
  int it = 0, stalls = 0;
  double last_restart = INFINITY;
  ecs_status status = ECS_NOT_CONVERGED;
  for (;;) {
    bicg_enqueue_restart(C, K, b, x);
    double rt = read_scalar(C, &S->est);
    st->rel_residual = rt;
    if (!(rt == rt) || std::isinf(rt)) {
      status = fail(C, ECS_EBREAKDOWN, "Bi-CGSTAB: residual is NaN/Inf");
      break;
    }
    if (rt <= d->rtol) { status = ECS_OK; break; }
    if (it >= d->maxit) { status = ECS_NOT_CONVERGED; break; }
    if (rt >= last_restart) {
      if (++stalls >= 3) {  // the true residual stalled (rounding floor): best iterate, not converged
        status = fail(C, ECS_NOT_CONVERGED, "Bi-CGSTAB: true residual stalled over three restarts");
        break;
      }
    }
    last_restart = rt;
    while (it < d->maxit) {
      bicg_enqueue_step<RZ>(C, K, x);
      bicg_enqueue_readback(C);
      st->vcycles += 2;
      it++;
      if (hipStreamSynchronize(s) != hipSuccess) break;
      double est;
      int bad;
      bicg_take_readback(C, &est, &bad);
      if (d->history && it - 1 < d->history_len) d->history[it - 1] = est;
      if (bad) break;  // restart from the current iterate
      if (est <= d->rtol) break;
    }
    st->restarts++;
  }
  st->iterations = it;
  HIP_OK(hipGetLastError());
  return status;
}

// ------------------------------------------------------------- batched
// Many independent systems (Sec. 2's blocks), every right-hand side solved by
// Bi-CGSTAB.  Each system takes its right-hand sides in groups of up to
// kMaxRhs (one group when the fused 2D V(1,1) red-black cycle runs: every
// kernel of an iteration then serves the whole group in one launch, a slot
// per right-hand side; one right-hand side per group otherwise).  A system
// advances in rounds on its own stream: a round enqueues the restarts (true
// residual) of the slots that need one, one batched iteration of the slots
// that iterate, and the readback of every slot's scalars; an event per
// context marks the round's end, and the host polls the events, so systems of
// different sizes progress independently.  Per slot the arithmetic is that of
// the single solve, kernel for kernel, so results equal single solves.
static_assert(kMaxRhs * sizeof(BicgScalars) <= kPinnedStage, "slot scalars fit the pinned readback area");

struct BatchSlot {
  int phase = 0;  // 1 verify (true residual, restart), 2 iterate, 3 finished
  int it = 0, stalls = 0, restarts = 0;
  double last_restart = INFINITY, rt = 0;
};

struct BatchItem {
  ecs_ctx *C = nullptr;
  const ecs_solve_desc *d = nullptr;  // this system's Krylov settings
  KrylovBufs K;
  const cplx<double> *b0 = nullptr;   // the caller's right-hand sides and solutions
  cplx<double> *x0 = nullptr;
  int nrhs = 0, group = 1;            // right-hand sides; slots per group
  int first = 0, count = 0;           // the current group: right-hand sides [first, first + count)
  bool started = false;               // the group's norms are in
  bool done = false;
  BatchSlot slot[kMaxRhs];
  RhsSet ver{}, itr{};                // slots restarted / iterated in the round in flight
  ecs_stats agg{};
  ecs_status worst = ECS_OK;
};

void batch_note(BatchItem &I, ecs_status st) {
  if (st != ECS_OK && (I.worst == ECS_OK || st < 0)) I.worst = st;
}

void batch_finish_slot(BatchItem &I, int q, ecs_status st) {
  BatchSlot &S = I.slot[q];
  I.agg.iterations += S.it;
  I.agg.restarts += S.restarts;
  I.agg.rel_residual = std::max(I.agg.rel_residual, S.rt);
  batch_note(I, st);
  S.phase = 3;
}

// a slot's vector of the batched layout
template <typename T>
T *slot_of(void *base, const KrylovBufs &K, int q) {
  return reinterpret_cast<T *>(base) + (int64_t)q * K.ld;
}

template <typename RZ>
CycleBufs<RZ> batch_bufs(ecs_ctx *C, const KrylovBufs &K) {
  CycleBufs<RZ> B;
  for (int l = 0; l < C->nlev; l++) {
    B.b[l] = reinterpret_cast<cplx<RZ> *>(K.lb[l]);
    B.t[l] = reinterpret_cast<cplx<RZ> *>(K.lt[l]);
    B.u[l] = reinterpret_cast<cplx<RZ> *>(K.lu[l]);
  }
  return B;
}

// z = M^{-1} v for every slot in rs (FP64 in, cycle dtype out)
template <typename RZ>
void batch_precond(ecs_ctx *C, const KrylovBufs &K, const cplx<double> *v, cplx<RZ> *z, const RhsSet &rs) {
  const int64_t n = nn_of(C);
  if (!fused_vcycle(C)) {  // one slot, slot 0: the single solve's cycle
    precond<RZ>(C, v, z);
    return;
  }
  const CycleBufs<RZ> B = batch_bufs<RZ>(C, K);
  if constexpr (sizeof(RZ) == 4) {
    cplx<float> *b = reinterpret_cast<cplx<float> *>(K.b32);
    launch_cast<double, float>(v, b, n, C->stream, rs);
    vcycle_fused<float>(C, b, z, nullptr, &B, rs);
  } else {
    vcycle_fused<double>(C, v, z, nullptr, &B, rs);
  }
}

// one Bi-CGSTAB iteration of every slot in rs (bicg_enqueue_step per slot)
template <typename RZ>
void batch_step(ecs_ctx *C, const KrylovBufs &K, const RhsSet &rs) {
  const int64_t n = nn_of(C);
  hipStream_t s = C->stream;
  BicgScalars *S = C->bs;
  cplx<RZ> *ph = reinterpret_cast<cplx<RZ> *>(K.ph);
  cplx<RZ> *sh = reinterpret_cast<cplx<RZ> *>(K.sh);
  launch_bicg_p<double>(K.p, K.r, K.v, n, S, s, rs);
  batch_precond<RZ>(C, K, K.p, ph, rs);
  launch_apply_dot<double, RZ>(grid_A(C), ph, K.v, K.rh, kBicgAlpha, C->partials, S, s, rs);
  launch_bicg_s<double>(K.s, K.r, K.v, n, S, s, rs);
  batch_precond<RZ>(C, K, K.s, sh, rs);
  launch_apply_dot<double, RZ>(grid_A(C), sh, K.tt, K.s, kBicgOmega, C->partials, S, s, rs);
  launch_bicg_xr<double, RZ>(K.bx, ph, sh, K.r, K.s, K.tt, K.rh, n, C->partials, S, s, rs);
}

// restart of slot q: r = b - A x, (r, r) -> the restart scalars, r^ = r, p = v = 0
void batch_restart(ecs_ctx *C, const KrylovBufs &K, int q) {
  const int64_t n = nn_of(C);
  hipStream_t s = C->stream;
  cplx<double> *r = slot_of<cplx<double>>(K.r, K, q);
  launch_residual<double>(grid_A(C), slot_of<cplx<double>>(K.bz, K, q), slot_of<cplx<double>>(K.bx, K, q), r, s);
  launch_pairdot<double>(r, r, nullptr, nullptr, 1, n, C->partials + (int64_t)q * kRhsPartials, C->bs + q, kBicgInit,
                         s);
  (void)hipMemcpyAsync(slot_of<cplx<double>>(K.rh, K, q), r, n * sizeof(cplx<double>), hipMemcpyDeviceToDevice, s);
  launch_zero<double>(slot_of<cplx<double>>(K.p, K, q), n, s);
  launch_zero<double>(slot_of<cplx<double>>(K.v, K, q), n, s);
}

// Enqueues the system's next round, ending in a readback into the pinned
// buffer: a new group's right-hand side norms, or every slot's scalars.
void batch_enqueue(BatchItem &I) {
  ecs_ctx *C = I.C;
  const ecs_solve_desc *d = I.d;
  const int64_t nn = nn_of(C);
  const HostLevel &F = C->hl[0];
  hipStream_t s = C->stream;
  if (!I.started) {
    for (int q = 0; q < I.count; q++) {
      const int64_t r = I.first + q;
      cplx<double> *bz = slot_of<cplx<double>>(I.K.bz, I.K, q), *x = slot_of<cplx<double>>(I.K.bx, I.K, q);
      launch_mask_boundary(F.n[0], F.n[1], F.n[2], I.b0 + r * nn, bz, s);
      if (d->x_is_guess) launch_mask_boundary(F.n[0], F.n[1], F.n[2], I.x0 + r * nn, x, s);
      else launch_zero<double>(x, nn, s);
      launch_nrm2sq<double>(bz, nn, C->partials, &C->gs->g[q], s);
    }
    (void)hipMemcpyAsync(C->pinned, C->gs->g, I.count * sizeof(cplx<double>), hipMemcpyDeviceToHost, s);
    return;
  }
  I.ver.count = I.itr.count = 0;
  for (int q = 0; q < I.count; q++) {
    if (I.slot[q].phase == 1) I.ver.slot[I.ver.count++] = q;
    else if (I.slot[q].phase == 2) I.itr.slot[I.itr.count++] = q;
  }
  for (int k = 0; k < I.ver.count; k++) batch_restart(C, I.K, I.ver.slot[k]);
  if (I.itr.count > 0) {
    if (C->prec.vcycle_dtype == ECS_F32) batch_step<float>(C, I.K, I.itr);
    else batch_step<double>(C, I.K, I.itr);
  }
  (void)hipMemcpyAsync(C->pinned, C->bs, I.count * sizeof(BicgScalars), hipMemcpyDeviceToHost, s);
}

void batch_next_group(BatchItem &I) {
  I.first += I.count;
  I.count = std::min(I.group, I.nrhs - I.first);
  I.started = false;
  for (int q = 0; q < kMaxRhs; q++) I.slot[q] = BatchSlot();
  if (I.count <= 0) I.done = true;
}

// Consumes the round's readback and moves every slot on.
void batch_process(BatchItem &I) {
  ecs_ctx *C = I.C;
  const ecs_solve_desc *d = I.d;
  const int64_t nn = nn_of(C);
  if (!I.started) {
    double *stage = reinterpret_cast<double *>(reinterpret_cast<char *>(C->pinned) + kPinnedStage);
    for (int q = 0; q < I.count; q++) {
      cplx<double> g;
      std::memcpy(&g, reinterpret_cast<const char *>(C->pinned) + q * sizeof(cplx<double>), sizeof g);
      const double bn = std::sqrt(g.re);
      if (!(bn == bn) || std::isinf(bn)) {
        batch_finish_slot(I, q, ECS_EBREAKDOWN);
      } else if (bn == 0) {
        launch_zero<double>(slot_of<cplx<double>>(I.K.bx, I.K, q), nn, C->stream);  // A x = 0 -> x = 0
        I.slot[q].rt = 0;
        batch_finish_slot(I, q, ECS_OK);
      } else {
        // the staging area is not written again before this copy has run
        stage[q] = bn;
        (void)hipMemcpyAsync(&C->bs[q].bnorm, &stage[q], sizeof(double), hipMemcpyHostToDevice, C->stream);
        I.slot[q].phase = 1;
      }
    }
    I.started = true;
  } else {
    auto scal = [&](int q, double *est, int *bad) {
      const char *p = reinterpret_cast<const char *>(C->pinned) + q * sizeof(BicgScalars);
      std::memcpy(est, p + offsetof(BicgScalars, est), sizeof(double));
      std::memcpy(bad, p + offsetof(BicgScalars, bad), sizeof(int));
    };
    for (int k = 0; k < I.ver.count; k++) {
      const int q = I.ver.slot[k];
      BatchSlot &S = I.slot[q];
      double est;
      int bad;
      scal(q, &est, &bad);
      S.rt = est;
      if (!(est == est) || std::isinf(est)) {
        batch_finish_slot(I, q, ECS_EBREAKDOWN);
      } else if (est <= d->rtol) {
        batch_finish_slot(I, q, ECS_OK);
      } else if (S.it >= d->maxit) {
        batch_finish_slot(I, q, ECS_NOT_CONVERGED);
      } else if (est >= S.last_restart && ++S.stalls >= 3) {
        batch_finish_slot(I, q, ECS_NOT_CONVERGED);
      } else {
        if (S.last_restart < INFINITY) S.restarts++;
        S.last_restart = est;
        S.phase = 2;
      }
    }
    for (int k = 0; k < I.itr.count; k++) {
      const int q = I.itr.slot[k];
      BatchSlot &S = I.slot[q];
      double est;
      int bad;
      scal(q, &est, &bad);
      S.it++;
      I.agg.vcycles += 2;
      if (bad || est <= d->rtol || S.it >= d->maxit) S.phase = 1;
    }
  }
  bool all = true;
  for (int q = 0; q < I.count; q++) all = all && I.slot[q].phase == 3;
  if (!all) return;
  // the group is finished: its iterates go to the caller's solutions
  for (int q = 0; q < I.count; q++)
    (void)hipMemcpyAsync(I.x0 + (int64_t)(I.first + q) * nn, slot_of<cplx<double>>(I.K.bx, I.K, q),
                         nn * sizeof(cplx<double>), hipMemcpyDeviceToDevice, C->stream);
  batch_next_group(I);
}

ecs_status batch_solve_impl(int n, ecs_ctx *const *ctxs, const ecs_solve_desc *const *descs, const void *const *b,
                            void *const *x, const int *nrhs, ecs_stats *stats) {
  std::vector<BatchItem> items(n);
  for (int q = 0; q < n; q++) {
    ecs_ctx *C = ctxs[q];
    ecs_status st = check_ready(C);
    if (st != ECS_OK) return st;
    const ecs_solve_desc *d = descs[q];
    if (!d) return fail(C, ECS_EINVAL, "null solve descriptor");
    if (d->krylov != ECS_KRYLOV_BICGSTAB) return fail(C, ECS_EINVAL, "the batched solve uses Bi-CGSTAB");
    if (!(d->rtol > 0) || d->maxit < 0) return fail(C, ECS_EINVAL, "rtol must be > 0, maxit >= 0");
    if (nrhs[q] > 0 && (!b[q] || !x[q])) return fail(C, ECS_EINVAL, "null right-hand side or solution pointer");
    for (int p = 0; p < q; p++)
      if (ctxs[p] == C) return fail(C, ECS_EINVAL, "a context appears twice in the batch");
    if (nrhs[q] < 0) return fail(C, ECS_EINVAL, "negative right-hand side count");
    BatchItem &I = items[q];
    // right-hand sides at once: up to kMaxRhs (or the desc's nrhs) with the fused cycle
    const int cap = d->nrhs > 0 ? std::min(d->nrhs, kMaxRhs) : kMaxRhs;
    I.group = fused_vcycle(C) ? std::max(1, std::min(nrhs[q], cap)) : 1;
    const size_t need = C->hier_bytes + plan_batch(C, I.group, nullptr, &I.K);
    if (need > C->ws_bytes)
      return fail(C, ECS_ENOMEM, "workspace too small for the batched solve (size it with nrhs = " +
                                     std::to_string(I.group) + " right-hand sides at once)");
    if (!C->step_ev && hipEventCreateWithFlags(&C->step_ev, hipEventDisableTiming) != hipSuccess) {
      C->step_ev = nullptr;
      return fail(C, ECS_EDEVICE, "event creation failed");
    }
    plan_batch(C, I.group, C->ws + C->hier_bytes, &I.K);
    I.C = C;
    I.d = d;
    I.b0 = reinterpret_cast<const cplx<double> *>(b[q]);
    I.x0 = reinterpret_cast<cplx<double> *>(x[q]);
    I.nrhs = nrhs[q];
    I.first = 0;
    I.count = std::min(I.group, I.nrhs);
    I.done = I.nrhs == 0;
  }
  int active = 0;
  for (auto &I : items) {
    if (I.done) continue;
    batch_enqueue(I);
    if (hipEventRecord(I.C->step_ev, I.C->stream) != hipSuccess) return ECS_EDEVICE;
    active++;
  }
  while (active > 0) {
    for (auto &I : items) {
      if (I.done) continue;
      const hipError_t e = hipEventQuery(I.C->step_ev);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return fail(I.C, ECS_EDEVICE, std::string("batched solve: ") + hipGetErrorString(e));
      batch_process(I);
      if (I.done) {
        active--;
        continue;
      }
      batch_enqueue(I);
      if (hipEventRecord(I.C->step_ev, I.C->stream) != hipSuccess) return ECS_EDEVICE;
    }
  }
  for (auto &I : items)
    if (I.C && hipStreamSynchronize(I.C->stream) != hipSuccess) return ECS_EDEVICE;
  ecs_status worst = ECS_OK;
  for (int q = 0; q < n; q++) {
    items[q].agg.status = items[q].worst;
    if (stats) stats[q] = items[q].agg;
    if (items[q].worst != ECS_OK && (worst == ECS_OK || items[q].worst < 0)) worst = items[q].worst;
  }
  return worst;
}

// ------------------------------------------------------- coupled blocks
// Storage of the outer FGMRES of a coupled block system (caller's workspace):
// the stacked right-hand side with boundary entries zeroed, the Arnoldi basis,
// the preconditioned directions, the outer scalars and reduction partials.
struct CoupledBufs {
  cplx<double> *bz = nullptr, *V = nullptr, *Z = nullptr, *partials = nullptr;
  GmresScalars *S = nullptr;
  int64_t ld = 0;
};

size_t plan_coupled(int nb, int64_t nn, int m, char *base, CoupledBufs *B) {
  Carver cv(base);
  const int64_t N = nb * nn;
  B->ld = (N + 31) & ~int64_t(31);
  B->bz = cv.take<cplx<double>>(N);
  B->V = cv.take<cplx<double>>((size_t)(m + 1) * B->ld);
  B->Z = cv.take<cplx<double>>((size_t)m * B->ld);
  B->S = cv.take<GmresScalars>(1);
  B->partials = cv.take<cplx<double>>((size_t)kRedBlocks * (2 * kMaxRestart + 2));
  return cv.off;
}

// y = A x for the stacked vector: A_ii x_i per block, then the coupling
// -k2c_ij x_j; with b, y = b - A x
void coupled_apply(int nb, ecs_ctx *const *ctx, const double *k2c, const cplx<double> *x, cplx<double> *y,
                   const cplx<double> *b, hipStream_t s) {
  const int64_t nn = nn_of(ctx[0]);
  for (int i = 0; i < nb; i++) launch_apply<double, double, double>(grid_A(ctx[i]), x + i * nn, y + i * nn, s);
  if (k2c || b) launch_couple(k2c ? nb : 1, k2c ? nn : nb * nn, k2c, x, y, b, s);
}

ecs_status coupled_check(int nb, ecs_ctx *const *ctx, const ecs_solve_desc *outer, const ecs_solve_desc *inner) {
  if (nb < 1 || nb > kMaxBlocks || !ctx || !outer)
    return fail(ctx && nb >= 1 ? ctx[0] : nullptr, ECS_EINVAL,
                "coupled solve: nb = " + std::to_string(nb) + " blocks (1 to " + std::to_string(kMaxBlocks) +
                    ") and an outer descriptor are required");
  for (int i = 0; i < nb; i++) {
    if (!ctx[i]) return ECS_EINVAL;
    ecs_status st = check_ready(ctx[i]);
    if (st != ECS_OK) return st;
    if (ctx[i]->dim != ctx[0]->dim || ctx[i]->device != ctx[0]->device)
      return fail(ctx[0], ECS_EINVAL, "coupled blocks must share the dimension and the device");
    for (int a = 0; a < 3; a++)
      if (ctx[i]->n[a] != ctx[0]->n[a]) return fail(ctx[0], ECS_EINVAL, "coupled blocks must share the grid");
  }
  if (outer->krylov != ECS_KRYLOV_FGMRES) return fail(ctx[0], ECS_EINVAL, "the outer method is FGMRES");
  if (outer->restart < 1 || outer->restart > kMaxRestart) return fail(ctx[0], ECS_EINVAL, "restart must be in [1, 64]");
  if (!(outer->rtol > 0) || outer->maxit < 0) return fail(ctx[0], ECS_EINVAL, "rtol must be > 0 and maxit >= 0");
  if (outer->orth < ECS_ORTH_DCGS2 || outer->orth > ECS_ORTH_CGS2_SELECTIVE)
    return fail(ctx[0], ECS_EINVAL, "unknown orthogonalisation");
  if (inner && (inner->krylov != ECS_KRYLOV_BICGSTAB || !(inner->rtol > 0) || inner->maxit < 1))
    return fail(ctx[0], ECS_EINVAL, "the block solves use Bi-CGSTAB with rtol > 0, maxit >= 1");
  return ECS_OK;
}

// Right-preconditioned FGMRES(m) over the stacked vector; the preconditioner
// solves every diagonal block with its own context, all blocks at once through
// the batched Bi-CGSTAB driver (inner == NULL: one multigrid cycle per block).
ecs_status coupled_fgmres(int nb, ecs_ctx *const *ctx, const double *k2c, const ecs_solve_desc *d,
                          const ecs_solve_desc *inner, const CoupledBufs &B, const cplx<double> *b, cplx<double> *x,
                          ecs_stats *st) {
  ecs_ctx *C = ctx[0];
  const int64_t nn = nn_of(C), N = nb * nn;
  const int m = d->restart;
  hipStream_t s = C->stream;
  GmresScalars *S = B.S;
  const int64_t ld = B.ld;
  const HostLevel &F = C->hl[0];
  for (int i = 0; i < nb; i++) launch_mask_boundary(F.n[0], F.n[1], F.n[2], b + i * nn, B.bz + i * nn, s);
  launch_nrm2sq<double>(B.bz, N, B.partials, &S->nrm2, s);
  const double bnorm = std::sqrt(read_scalar(C, &S->nrm2.re));
  if (!(bnorm == bnorm) || std::isinf(bnorm)) return fail(C, ECS_EBREAKDOWN, "right-hand side contains NaN/Inf");
  if (!d->x_is_guess) launch_zero<double>(x, N, s);
  if (bnorm == 0) {
    launch_zero<double>(x, N, s);
    st->rel_residual = 0;
    HIP_OK(hipStreamSynchronize(s));
    return ECS_OK;
  }
  HIP_OK(hipMemcpyAsync(&S->bnorm, &bnorm, sizeof(double), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemsetAsync(&S->reorth_count, 0, sizeof(int), s));
  std::vector<ecs_stats> bst(nb);
  std::vector<const void *> bp(nb);
  std::vector<void *> xp(nb);
  std::vector<int> ones(nb, 1);
  std::vector<const ecs_solve_desc *> inner_descs(nb, inner);
  int it = 0;
  int64_t later_steps = 0;
  ecs_status status = ECS_NOT_CONVERGED;
  for (;;) {
    coupled_apply(nb, ctx, k2c, x, B.V, B.bz, s);  // r = b - A x
    launch_nrm2sq<double>(B.V, N, B.partials, &S->nrm2, s);
    launch_gmres_start(S, m, s);
    launch_scale_dev(B.V, N, &S->inv, s);
    const double rt = read_scalar(C, &S->resid_true);
    st->rel_residual = rt;
    if (!(rt == rt) || std::isinf(rt)) { status = fail(C, ECS_EBREAKDOWN, "coupled FGMRES: residual is NaN/Inf"); break; }
    if (rt <= d->rtol) { status = ECS_OK; break; }
    if (it >= d->maxit) { status = ECS_NOT_CONVERGED; break; }
    int k = 0;
    bool bad = false;
    for (int j = 0; j < m && it < d->maxit; j++) {
      cplx<double> *vj = B.V + (int64_t)j * ld, *w = B.V + (int64_t)(j + 1) * ld, *zj = B.Z + (int64_t)j * ld;
      // z_j = blockdiag(A_ii)^{-1} v_j, approximately
      if (inner) {
        for (int i = 0; i < nb; i++) {
          bp[i] = vj + i * nn;
          xp[i] = zj + i * nn;
        }
        HIP_OK(hipStreamSynchronize(s));
        const ecs_status ist =
            batch_solve_impl(nb, ctx, inner_descs.data(), bp.data(), xp.data(), ones.data(), bst.data());
        if (ist < 0) { status = ist; bad = true; break; }
        for (int i = 0; i < nb; i++) {
          st->vcycles += bst[i].vcycles;
          st->inner_iterations += bst[i].iterations;
          if (ctx[i]->stream != s) HIP_OK(hipStreamSynchronize(ctx[i]->stream));
        }
      } else {
        HIP_OK(hipStreamSynchronize(s));
        for (int i = 0; i < nb; i++) {
          ecs_ctx *Ci = ctx[i];
          if (Ci->prec.vcycle_dtype == ECS_F64) {
            vcycle<double>(Ci, vj + i * nn, zj + i * nn);
          } else {
            KrylovBufs K;  // the block's own cycle-dtype scratch
            plan_krylov(Ci, nullptr, Ci->ws + Ci->hier_bytes, &K);
            cplx<float> *tz = reinterpret_cast<cplx<float> *>(K.tz);
            precond<float>(Ci, vj + i * nn, tz);
            launch_cast<float, double>(tz, zj + i * nn, nn, Ci->stream);
          }
        }
        for (int i = 0; i < nb; i++)
          if (ctx[i]->stream != s) HIP_OK(hipStreamSynchronize(ctx[i]->stream));
        st->vcycles += nb;
      }
      coupled_apply(nb, ctx, k2c, zj, w, nullptr, s);
      orthogonalise(C, B.V, ld, j, w, N, B.partials, S, m, d->orth, s);
      later_steps += j > 0;
      launch_gmres_givens(S, j, m, s);
      launch_scale_dev(w, N, &S->inv, s);
      it++;
      k = j + 1;
      if (!read_bytes(C, &S->est, 2 * sizeof(double) + 2 * sizeof(int))) { bad = true; break; }
      double est;
      int happy;
      std::memcpy(&est, C->pinned, sizeof(double));
      std::memcpy(&happy, reinterpret_cast<char *>(C->pinned) + 2 * sizeof(double) + sizeof(int), sizeof(int));
      if (d->history && it - 1 < d->history_len) d->history[it - 1] = est;
      if (!(est == est) || std::isinf(est)) { bad = true; break; }
      if (est <= d->rtol || happy) break;
    }
    if (bad) {
      if (status >= 0) status = fail(C, ECS_EBREAKDOWN, "coupled FGMRES: breakdown");
      break;
    }
    launch_gmres_backsolve(S, k, m, s);
    launch_lincomb<double>(B.Z, ld, k, S->y, x, N, s);
    st->restarts++;
  }
  st->iterations = it;
  st->reorthogonalisations = reorth_passes(C, S, d->orth, it, later_steps);
  HIP_OK(hipStreamSynchronize(s));
  HIP_OK(hipGetLastError());
  return status;
}

// Krylov storage of one solve: after the hierarchy in the caller's workspace,
// or (kscratch) in this device's static scratch array.
ecs_status plan_solve_storage(ecs_ctx *C, const ecs_solve_desc *d, char *kscratch, KrylovBufs *K) {
  const size_t kb = plan_krylov(C, d, nullptr, K);
  if (kscratch) {
    if (kb > kScratchBytes)
      return fail(C, ECS_ENOMEM, "solve needs " + std::to_string(kb >> 20) + " MiB of Krylov storage; the static "
                                 "scratch holds " + std::to_string(kScratchBytes >> 20) + " MiB");
    plan_krylov(C, d, kscratch, K);
    return ECS_OK;
  }
  if (C->hier_bytes + kb > C->ws_bytes) return fail(C, ECS_ENOMEM, "workspace too small for this solve");
  plan_krylov(C, d, C->ws + C->hier_bytes, K);
  return ECS_OK;
}

ecs_status solve_impl(ecs_ctx *C, const ecs_solve_desc *d, const cplx<double> *b, cplx<double> *x, ecs_stats *st,
                      char *kscratch = nullptr) {
  if (d->restart < 1 || d->restart > kMaxRestart) return fail(C, ECS_EINVAL, "restart must be in [1, 64]");
  if (!(d->rtol > 0) || d->maxit < 0) return fail(C, ECS_EINVAL, "rtol must be > 0 and maxit >= 0");
  if (d->krylov < 0 || d->krylov > 2) return fail(C, ECS_EINVAL, "unknown Krylov method");
  if (d->orth < ECS_ORTH_DCGS2 || d->orth > ECS_ORTH_CGS2_SELECTIVE)
    return fail(C, ECS_EINVAL, "unknown orthogonalisation");
  if (d->inner > 0 && d->krylov != ECS_KRYLOV_FGMRES) return fail(C, ECS_EINVAL, "inner iterations need FGMRES");
  if (d->inner > 0 && C->prec.kind == ECS_PREC_NONE) return fail(C, ECS_EINVAL, "inner iterations need a cycle");
  if (C->prec.kind == ECS_PREC_NONE && C->prec.vcycle_dtype == ECS_F32)
    return fail(C, ECS_EINVAL, "no preconditioner: use vcycle_dtype F64");
  KrylovBufs K;
  ecs_status pst = plan_solve_storage(C, d, kscratch, &K);
  if (pst != ECS_OK) return pst;
  const bool f32 = C->prec.vcycle_dtype == ECS_F32;
  // boundary entries of b are ignored and those of a guess x are reset
  const HostLevel &F = C->hl[0];
  launch_mask_boundary(F.n[0], F.n[1], F.n[2], b, K.bz, C->stream);
  if (d->x_is_guess) launch_mask_boundary(F.n[0], F.n[1], F.n[2], x, x, C->stream);
  b = K.bz;
  if (d->krylov == ECS_KRYLOV_BICGSTAB)
    return f32 ? bicgstab<float>(C, d, K, b, x, st) : bicgstab<double>(C, d, K, b, x, st);
  return f32 ? gmres<float>(C, d, K, b, x, st) : gmres<double>(C, d, K, b, x, st);
}

}  // namespace

// ======================================================================= ABI

extern "C" {

ecs_status ecs_create(ecs_ctx **out, int dim, const int64_t *nodes, const double *lo, const double *hi,
                      void *stream) {
  if (!out || !nodes || !lo || !hi || (dim != 2 && dim != 3)) return ECS_EINVAL;
  *out = nullptr;
  for (int a = 0; a < dim; a++) {
    if (nodes[a] < 3 || nodes[a] > (1 << 20) || !(hi[a] > lo[a])) return ECS_EINVAL;
  }
  int64_t total = 1;
  for (int a = 0; a < dim; a++) total *= nodes[a];
  if (total > (int64_t)1 << 31) return ECS_EINVAL;
  ecs_ctx *C = new ecs_ctx();
  C->dim = dim;
  for (int a = 0; a < dim; a++) {
    C->n[a] = (int)nodes[a];
    C->lo[a] = lo[a];
    C->hi[a] = hi[a];
  }
  C->stream = reinterpret_cast<hipStream_t>(stream);
  if (hipGetDevice(&C->device) != hipSuccess ||
      hipHostMalloc((void **)&C->pinned, kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
    delete C;
    return ECS_EDEVICE;
  }
  // the library's set-up call on this device: look up its static scratch
  // (with the device current) so that ecs_solve_static never has to
  hipError_t se;
  C->scratch = scratch_address(C->device, &se);
  if (!C->scratch) {
    (void)hipHostFree(C->pinned);
    delete C;
    return ECS_EDEVICE;
  }
  *out = C;
  return ECS_OK;
}

ecs_status ecs_set_ecs(ecs_ctx *C, int axis, int side, int kind, double start, double theta) {
  if (!C) return ECS_EINVAL;
  if (axis < 0 || axis >= C->dim || side < 0 || side > 1) return fail(C, ECS_EINVAL, "bad axis or side");
  if (kind == ECS_BC_ECS) {
    if (!(theta > 0 && theta < M_PI / 2)) return fail(C, ECS_EINVAL, "theta must lie in (0, pi/2)");
    if (!(start > C->lo[axis] && start < C->hi[axis])) return fail(C, ECS_EINVAL, "layer start outside the box");
  } else if (kind != ECS_BC_DIRICHLET) {
    return fail(C, ECS_EINVAL, "bad boundary kind");
  }
  C->side[axis][side].kind = kind;
  C->side[axis][side].start = start;
  C->side[axis][side].theta = theta;
  C->ready = false;
  return ECS_OK;
}

ecs_status ecs_set_k2(ecs_ctx *C, const void *k2_dev, int real_dtype) {
  if (!C) return ECS_EINVAL;
  if (!k2_dev) return fail(C, ECS_EINVAL, "k2 is null");
  if (real_dtype != ECS_F64 && real_dtype != ECS_F32) return fail(C, ECS_EINVAL, "k2 dtype must be F64 or F32");
  C->k2_user = k2_dev;
  C->k2_dtype = real_dtype;
  C->k2 = nullptr;
  C->ready = false;
  return ECS_OK;
}

ecs_status ecs_set_precond(ecs_ctx *C, const ecs_prec_desc *d) {
  if (!C || !d) return ECS_EINVAL;
  if (d->kind < ECS_PREC_NONE || d->kind > ECS_PREC_QD) return fail(C, ECS_EINVAL, "unknown preconditioner kind");
  if (d->smoother != ECS_SMOOTH_JACOBI && d->smoother != ECS_SMOOTH_RBGS) return fail(C, ECS_EINVAL, "bad smoother");
  if (!(d->omega > 0 && d->omega < 2)) return fail(C, ECS_EINVAL, "omega must lie in (0, 2)");
  if (d->nu1 < 0 || d->nu2 < 0 || d->nu1 + d->nu2 < 1 || d->nu1 > 8 || d->nu2 > 8)
    return fail(C, ECS_EINVAL, "bad sweep counts");
  if (d->gamma_f < 1 || d->gamma_c < 1 || d->gamma_f > 4 || d->gamma_c > 8)
    return fail(C, ECS_EINVAL, "bad cycle indices");
  if (d->vcycle_dtype != ECS_F64 && d->vcycle_dtype != ECS_F32) return fail(C, ECS_EINVAL, "bad cycle dtype");
  if (d->coarsest_nodes < 3) return fail(C, ECS_EINVAL, "coarsest grid needs >= 3 nodes per axis");
  // levels: every axis must reach coarsest_nodes by exact halving
  int nlev = -1;
  for (int a = 0; a < C->dim; a++) {
    int n = C->n[a], lev = 1;
    while (n > d->coarsest_nodes && (n - 1) % 2 == 0) {
      n = (n - 1) / 2 + 1;
      lev++;
    }
    if (n != d->coarsest_nodes) return fail(C, ECS_EINVAL, "nodes-1 must be (coarsest_nodes-1) * 2^k on every axis");
    if (nlev >= 0 && lev != nlev) return fail(C, ECS_EINVAL, "all axes must have the same number of levels");
    nlev = lev;
  }
  if (nlev > kMaxLev) return fail(C, ECS_EINVAL, "too many levels");
  int nunk = 1;
  for (int a = 0; a < C->dim; a++) nunk *= d->coarsest_nodes - 2;
  if (nunk > 2048) return fail(C, ECS_EINVAL, "coarsest grid too large for the dense solve (> 2048 unknowns)");
  C->prec = *d;
  C->nlev = nlev;
  C->have_prec = true;
  C->ready = false;
  return ECS_OK;
}

ecs_status ecs_workspace_size(ecs_ctx *C, const ecs_solve_desc *d, size_t *bytes) {
  if (!C || !bytes) return ECS_EINVAL;
  if (!C->have_prec) return fail(C, ECS_ESTATE, "set the preconditioner first");
  if (d && (d->restart < 1 || d->restart > kMaxRestart)) return fail(C, ECS_EINVAL, "restart must be in [1, 64]");
  if (d && (d->nrhs < 0 || d->nrhs > kMaxRhs)) return fail(C, ECS_EINVAL, "nrhs must be in [0, 8]");
  build_host_levels(C);
  KrylovBufs K, KB;
  size_t kb = plan_krylov(C, d, nullptr, &K);
  if (d && d->krylov == ECS_KRYLOV_BICGSTAB && d->nrhs > 0) kb = std::max(kb, plan_batch(C, d->nrhs, nullptr, &KB));
  *bytes = plan_hierarchy(C, nullptr) + 256 + kb + 256;
  return ECS_OK;
}

ecs_status ecs_set_workspace(ecs_ctx *C, void *dev, size_t bytes) {
  if (!C) return ECS_EINVAL;
  if (!C->have_prec || !C->k2_user) return fail(C, ECS_ESTATE, "set k2 and the preconditioner first");
  if (!dev || ((uintptr_t)dev % 256) != 0) return fail(C, ECS_EINVAL, "workspace must be 256-byte aligned");
  build_host_levels(C);
  size_t hb = plan_hierarchy(C, nullptr);
  hb = (hb + 255) & ~size_t(255);
  KrylovBufs K;
  if (hb + plan_krylov(C, nullptr, nullptr, &K) > bytes) return fail(C, ECS_ENOMEM, "workspace too small");
  drop_graphs(C);
  C->ws = reinterpret_cast<char *>(dev);
  C->ws_bytes = bytes;
  C->hier_bytes = hb;
  plan_hierarchy(C, C->ws);
  C->ready = false;
  ecs_status st = setup(C);
  if (st != ECS_OK) return st;
  C->ready = true;
  return ECS_OK;
}

ecs_status ecs_solve(ecs_ctx *C, const ecs_solve_desc *d, const void *b, void *x, ecs_stats *stats) {
  ecs_status st = check_ready(C);
  if (st != ECS_OK) return st;
  if (!d || !b || !x) return fail(C, ECS_EINVAL, "null argument");
  ecs_stats local{};
  auto t0 = std::chrono::steady_clock::now();
  st = solve_impl(C, d, reinterpret_cast<const cplx<double> *>(b), reinterpret_cast<cplx<double> *>(x), &local);
  local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  local.status = st;
  if (stats) *stats = local;
  return st;
}

ecs_status ecs_solve_static(ecs_ctx *C, const ecs_solve_desc *d, const void *b, void *x, ecs_stats *stats) {
  ecs_status st = check_ready(C);
  if (st != ECS_OK) return st;
  if (!d || !b || !x) return fail(C, ECS_EINVAL, "null argument");
  if (!C->scratch) return fail(C, ECS_ESTATE, "no static scratch on this device");
  ecs_stats local{};
  auto t0 = std::chrono::steady_clock::now();
  C->no_alloc = true;
  st = solve_impl(C, d, reinterpret_cast<const cplx<double> *>(b), reinterpret_cast<cplx<double> *>(x), &local,
                  C->scratch);
  C->no_alloc = false;
  local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  local.status = st;
  if (stats) *stats = local;
  return st;
}

ecs_status ecs_solve_adjoint(ecs_ctx *C, const ecs_solve_desc *d, const void *g, void *lam, ecs_stats *stats) {
  ecs_status st = check_ready(C);
  if (st != ECS_OK) return st;
  if (!d || !g || !lam) return fail(C, ECS_EINVAL, "null argument");
  KrylovBufs K;
  size_t need = C->hier_bytes + plan_krylov(C, d, nullptr, &K);
  if (need > C->ws_bytes) return fail(C, ECS_ENOMEM, "workspace too small for this solve");
  plan_krylov(C, d, C->ws + C->hier_bytes, &K);
  const HostLevel &F = C->hl[0];
  const int64_t n = nn_of(C);
  auto t0 = std::chrono::steady_clock::now();
  // A^T = W A W^{-1}:  A^T lam = g  <=>  A (W^{-1} lam) = W^{-1} g
  launch_scale_w(F.n[0], F.n[1], F.n[2], C->Wd[0], C->Wd[1], C->Wd[2], reinterpret_cast<const cplx<double> *>(g),
                 K.a1, true, C->stream);
  ecs_solve_desc d2 = *d;
  cplx<double> *y = K.a2;
  if (d->x_is_guess)
    launch_scale_w(F.n[0], F.n[1], F.n[2], C->Wd[0], C->Wd[1], C->Wd[2], reinterpret_cast<cplx<double> *>(lam), y,
                   true, C->stream);
  ecs_stats local{};
  st = solve_impl(C, &d2, K.a1, y, &local);
  launch_scale_w(F.n[0], F.n[1], F.n[2], C->Wd[0], C->Wd[1], C->Wd[2], y, reinterpret_cast<cplx<double> *>(lam), false,
                 C->stream);
  (void)n;
  local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  local.status = st;
  if (stats) *stats = local;
  return st;
}

ecs_status ecs_grad_k2(ecs_ctx *C, const void *lam, const void *u, double *grad) {
  if (!C) return ECS_EINVAL;
  if (!lam || !u || !grad) return fail(C, ECS_EINVAL, "null argument");
  launch_grad_k2(reinterpret_cast<const cplx<double> *>(lam), reinterpret_cast<const cplx<double> *>(u), grad,
                 nn_of(C), C->stream);
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

ecs_status ecs_apply(ecs_ctx *C, int op, const void *x, void *y) {
  ecs_status st = check_ready(C);
  if (st != ECS_OK) return st;
  if (!x || !y) return fail(C, ECS_EINVAL, "null argument");
  const cplx<double> *xi = reinterpret_cast<const cplx<double> *>(x);
  cplx<double> *yo = reinterpret_cast<cplx<double> *>(y);
  const HostLevel &F = C->hl[0];
  if (op == ECS_OP_A) {
    launch_apply<double, double, double>(grid_A(C), xi, yo, C->stream);
  } else if (op == ECS_OP_M) {
    launch_apply<double, double, double>(grid_M<double>(C, 0), xi, yo, C->stream);
  } else if (op == ECS_OP_AT) {
    KrylovBufs K;
    plan_krylov(C, nullptr, C->ws + C->hier_bytes, &K);
    launch_scale_w(F.n[0], F.n[1], F.n[2], C->Wd[0], C->Wd[1], C->Wd[2], xi, K.a1, true, C->stream);
    launch_apply<double, double, double>(grid_A(C), K.a1, K.a2, C->stream);
    launch_scale_w(F.n[0], F.n[1], F.n[2], C->Wd[0], C->Wd[1], C->Wd[2], K.a2, yo, false, C->stream);
  } else {
    return fail(C, ECS_EINVAL, "unknown operator");
  }
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

ecs_status ecs_vcycle(ecs_ctx *C, const void *v, void *z) {
  ecs_status st = check_ready(C);
  if (st != ECS_OK) return st;
  if (!v || !z) return fail(C, ECS_EINVAL, "null argument");
  if (C->prec.kind == ECS_PREC_NONE) return fail(C, ECS_EINVAL, "no preconditioner configured");
  const cplx<double> *vi = reinterpret_cast<const cplx<double> *>(v);
  cplx<double> *zo = reinterpret_cast<cplx<double> *>(z);
  if (C->prec.vcycle_dtype == ECS_F64) {
    vcycle<double>(C, vi, zo);
  } else {
    KrylovBufs K;
    plan_krylov(C, nullptr, C->ws + C->hier_bytes, &K);
    cplx<float> *zf = reinterpret_cast<cplx<float> *>(K.tz);
    precond<float>(C, vi, zf);
    launch_cast<float, double>(zf, zo, nn_of(C), C->stream);
  }
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

ecs_status ecs_vcycle_native(ecs_ctx *C, const void *v, void *z) {
  ecs_status st = check_ready(C);
  if (st != ECS_OK) return st;
  if (!v || !z) return fail(C, ECS_EINVAL, "null argument");
  if (C->prec.kind == ECS_PREC_NONE) return fail(C, ECS_EINVAL, "no preconditioner configured");
  if (C->prec.vcycle_dtype == ECS_F64)
    vcycle<double>(C, reinterpret_cast<const cplx<double> *>(v), reinterpret_cast<cplx<double> *>(z));
  else
    vcycle<float>(C, reinterpret_cast<const cplx<float> *>(v), reinterpret_cast<cplx<float> *>(z));
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

// Stand-alone multigrid on the preconditioner (Sec. 5): x <- x + MG(b - M x)
ecs_status ecs_mg_solve(ecs_ctx *C, const void *b_dev, void *x_dev, double rtol, int maxcycles, int x_is_guess,
                        double *history, int history_len, ecs_stats *stats) {
  ecs_status st = check_ready(C);
  if (st != ECS_OK) return st;
  if (!b_dev || !x_dev) return fail(C, ECS_EINVAL, "null argument");
  if (C->prec.kind == ECS_PREC_NONE) return fail(C, ECS_EINVAL, "no preconditioner configured");
  if (!(rtol >= 0) || maxcycles < 0 || (history_len > 0 && !history)) return fail(C, ECS_EINVAL, "bad argument");
  auto t0 = std::chrono::steady_clock::now();
  const cplx<double> *b = reinterpret_cast<const cplx<double> *>(b_dev);
  cplx<double> *x = reinterpret_cast<cplx<double> *>(x_dev);
  const int64_t n = nn_of(C);
  const HostLevel &F = C->hl[0];
  hipStream_t s = C->stream;
  KrylovBufs K;
  plan_krylov(C, nullptr, C->ws + C->hier_bytes, &K);
  cplx<double> *r = K.a1;
  GmresScalars *S = C->gs;
  const cplx<double> one = mk<double>(1, 0);
  HIP_OK(hipMemcpyAsync(&S->one, &one, sizeof(one), hipMemcpyHostToDevice, s));
  // ||b|| over interior nodes
  launch_mask_boundary(F.n[0], F.n[1], F.n[2], b, K.bz, s);
  launch_nrm2sq<double>(K.bz, n, C->partials, &S->nrm2, s);
  const double bnorm = std::sqrt(read_scalar(C, &S->nrm2.re));
  if (!(bnorm == bnorm) || std::isinf(bnorm)) return fail(C, ECS_EBREAKDOWN, "right-hand side contains NaN/Inf");
  if (!x_is_guess) launch_zero<double>(x, n, s);
  const Grid<double> gM = grid_M<double>(C, 0);
  ecs_stats local{};
  int m = 0;
  double rel = 0;
  ecs_status out = ECS_NOT_CONVERGED;
  for (;; m++) {
    launch_residual<double>(gM, b, x, r, s);
    launch_nrm2sq<double>(r, n, C->partials, &S->nrm2, s);
    const double rn = std::sqrt(read_scalar(C, &S->nrm2.re));
    rel = bnorm > 0 ? rn / bnorm : 0.0;
    if (m < history_len) history[m] = rel;
    if (!(rel == rel) || std::isinf(rel)) {
      out = ECS_EBREAKDOWN;
      break;
    }
    if (rel <= rtol) {
      out = ECS_OK;
      break;
    }
    if (m == maxcycles) break;
    if (C->prec.vcycle_dtype == ECS_F64) {
      cplx<double> *z = K.a2;
      vcycle<double>(C, r, z);
      launch_lincomb<double>(z, n, 1, &S->one, x, n, s);
    } else {
      cplx<float> *z = reinterpret_cast<cplx<float> *>(K.tz);
      precond<float>(C, r, z);
      launch_lincomb<float>(z, n, 1, &S->one, x, n, s);
    }
  }
  HIP_OK(hipStreamSynchronize(s));
  HIP_OK(hipGetLastError());
  local.iterations = m;
  local.vcycles = m;
  local.rel_residual = rel;
  local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  local.status = out;
  if (stats) *stats = local;
  if (out == ECS_EBREAKDOWN) return fail(C, out, "stand-alone multigrid produced NaN/Inf");
  return out;
}

#define LEVEL_CHECK(l)                                                                                    \
  do {                                                                                                    \
    ecs_status st_ = check_ready(C);                                                                      \
    if (st_ != ECS_OK) return st_;                                                                        \
    if ((l) < 0 || (l) >= C->nlev) return fail(C, ECS_EINVAL, "level out of range");                    \
  } while (0)

ecs_status ecs_smooth(ecs_ctx *C, int level, const void *b, void *u, int nsweeps) {
  LEVEL_CHECK(level);
  if (!b || !u || nsweeps < 0) return fail(C, ECS_EINVAL, "bad argument");
  if (C->prec.vcycle_dtype == ECS_F64)
    smooth<double>(C, level, reinterpret_cast<const cplx<double> *>(b), reinterpret_cast<cplx<double> *>(u),
                   C->L64[level].t, nsweeps, false);
  else
    smooth<float>(C, level, reinterpret_cast<const cplx<float> *>(b), reinterpret_cast<cplx<float> *>(u),
                  C->L32[level].t, nsweeps, false);
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

ecs_status ecs_residual_restrict(ecs_ctx *C, int level, const void *b, const void *u, void *rc) {
  LEVEL_CHECK(level);
  if (level + 1 >= C->nlev) return fail(C, ECS_EINVAL, "no coarser level");
  if (!b || !u || !rc) return fail(C, ECS_EINVAL, "null argument");
  if (C->prec.vcycle_dtype == ECS_F64)
    launch_residual_restrict<double>(grid_M<double>(C, level), grid_M<double>(C, level + 1),
                                     reinterpret_cast<const cplx<double> *>(b),
                                     reinterpret_cast<const cplx<double> *>(u), reinterpret_cast<cplx<double> *>(rc),
                                     C->stream);
  else
    launch_residual_restrict<float>(grid_M<float>(C, level), grid_M<float>(C, level + 1),
                                    reinterpret_cast<const cplx<float> *>(b), reinterpret_cast<const cplx<float> *>(u),
                                    reinterpret_cast<cplx<float> *>(rc), C->stream);
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

ecs_status ecs_prolong_correct(ecs_ctx *C, int level, const void *ec, void *u) {
  LEVEL_CHECK(level);
  if (level + 1 >= C->nlev) return fail(C, ECS_EINVAL, "no coarser level");
  if (!ec || !u) return fail(C, ECS_EINVAL, "null argument");
  if (C->prec.vcycle_dtype == ECS_F64)
    launch_prolong_add<double>(grid_M<double>(C, level), grid_M<double>(C, level + 1),
                               reinterpret_cast<const cplx<double> *>(ec), reinterpret_cast<cplx<double> *>(u),
                               C->stream);
  else
    launch_prolong_add<float>(grid_M<float>(C, level), grid_M<float>(C, level + 1),
                              reinterpret_cast<const cplx<float> *>(ec), reinterpret_cast<cplx<float> *>(u), C->stream);
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

ecs_status ecs_coarse_solve(ecs_ctx *C, const void *b, void *x) {
  ecs_status st = check_ready(C);
  if (st != ECS_OK) return st;
  if (!b || !x) return fail(C, ECS_EINVAL, "null argument");
  if (C->prec.vcycle_dtype == ECS_F64)
    coarse_solve<double>(C, reinterpret_cast<const cplx<double> *>(b), reinterpret_cast<cplx<double> *>(x));
  else
    coarse_solve<float>(C, reinterpret_cast<const cplx<float> *>(b), reinterpret_cast<cplx<float> *>(x));
  HIP_OK(hipGetLastError());
  return ECS_OK;
}

ecs_status ecs_level_info(ecs_ctx *C, int level, int *nlevels, int64_t *nodes) {
  if (!C) return ECS_EINVAL;
  if (!C->have_prec) return fail(C, ECS_ESTATE, "set the preconditioner first");
  if (nlevels) *nlevels = C->nlev;
  if (nodes) {
    if (level < 0 || level >= C->nlev) return fail(C, ECS_EINVAL, "level out of range");
    int n[3] = {C->n[0], C->n[1], C->n[2]};
    for (int l = 0; l < level; l++)
      for (int a = 0; a < C->dim; a++) n[a] = (n[a] - 1) / 2 + 1;
    for (int a = 0; a < 3; a++) nodes[a] = a < C->dim ? n[a] : 1;
  }
  return ECS_OK;
}

ecs_status ecs_timing_enable(ecs_ctx *C, int kclass, int enable) {
  if (!C || kclass < 0 || kclass >= kTClasses || enable < 0) return ECS_EINVAL;
  Timer &T = C->timers[kclass];
  T.on = enable != 0;
  T.every = enable > 1 ? enable : 1;
  T.seen = 0;
  return ECS_OK;
}

ecs_status ecs_timing_calibrate(ecs_ctx *C, int launches) {
  if (!C || launches < 1 || launches > 65536) return ECS_EINVAL;
  Timer &T = C->timers[kTEmpty];
  const bool was = T.on;
  T.on = true;
  for (int q = 0; q < launches; q++) {
    TimedScope ts(C, kTEmpty, 0.0);
    launch_empty(C->stream);
  }
  T.on = was;
  return hipGetLastError() == hipSuccess ? ECS_OK : fail(C, ECS_EDEVICE, "empty kernel launch failed");
}

ecs_status ecs_timing_read(ecs_ctx *C, int kclass, int64_t *launches, double *total_ms, double *algo_bytes) {
  if (!C || kclass < 0 || kclass >= kTClasses) return ECS_EINVAL;
  Timer &T = C->timers[kclass];
  HIP_OK(hipStreamSynchronize(C->stream));
  double tot = 0;
  for (size_t q = 0; q + 1 < T.used; q += 2) {
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, T.ev[q], T.ev[q + 1]));
    tot += ms;
  }
  if (launches) *launches = (int64_t)(T.used / 2);
  if (total_ms) *total_ms = tot;
  if (algo_bytes) *algo_bytes = T.bytes;
  T.used = 0;
  T.bytes = 0;
  return ECS_OK;
}

ecs_status ecs_batch_solve(int n, ecs_ctx *const *ctxs, const ecs_solve_desc *const *desc, const void *const *b,
                           void *const *x, const int *nrhs, ecs_stats *stats) {
  if (n < 0 || (n > 0 && (!ctxs || !desc || !b || !x || !nrhs))) return ECS_EINVAL;
  if (n == 0) return ECS_OK;
  for (int q = 0; q < n; q++)
    if (!ctxs[q]) return ECS_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  ecs_status st = batch_solve_impl(n, ctxs, desc, b, x, nrhs, stats);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    for (int q = 0; q < n; q++) stats[q].seconds = secs;
  return st;
}

ecs_status ecs_coupled_workspace_size(int nb, ecs_ctx *const *ctx, const ecs_solve_desc *outer, size_t *bytes) {
  if (!bytes) return ECS_EINVAL;
  ecs_status st = coupled_check(nb, ctx, outer, nullptr);
  if (st != ECS_OK) return st;
  CoupledBufs B;
  *bytes = plan_coupled(nb, nn_of(ctx[0]), outer->restart, nullptr, &B) + 256;
  return ECS_OK;
}

ecs_status ecs_coupled_solve(int nb, ecs_ctx *const *ctx, const double *k2c, const ecs_solve_desc *outer,
                             const ecs_solve_desc *inner, void *workspace, size_t ws_bytes, const void *b, void *x,
                             ecs_stats *stats) {
  ecs_status st = coupled_check(nb, ctx, outer, inner);
  if (st != ECS_OK) return st;
  if (!b || !x || !workspace) return fail(ctx[0], ECS_EINVAL, "null argument");
  if (((uintptr_t)workspace % 256) != 0) return fail(ctx[0], ECS_EINVAL, "workspace must be 256-byte aligned");
  CoupledBufs B;
  if (plan_coupled(nb, nn_of(ctx[0]), outer->restart, nullptr, &B) > ws_bytes)
    return fail(ctx[0], ECS_ENOMEM, "workspace too small for the coupled solve");
  plan_coupled(nb, nn_of(ctx[0]), outer->restart, reinterpret_cast<char *>(workspace), &B);
  if (!inner)
    for (int i = 0; i < nb; i++)
      if (ctx[i]->prec.kind == ECS_PREC_NONE) return fail(ctx[0], ECS_EINVAL, "block without a preconditioner");
  ecs_solve_desc in{};
  if (inner) {  // block solves start from zero and keep no history
    in = *inner;
    in.x_is_guess = 0;
    in.history = nullptr;
    in.history_len = 0;
  }
  ecs_stats local{};
  auto t0 = std::chrono::steady_clock::now();
  st = coupled_fgmres(nb, ctx, k2c, outer, inner ? &in : nullptr, B, reinterpret_cast<const cplx<double> *>(b),
                      reinterpret_cast<cplx<double> *>(x), &local);
  local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  local.status = st;
  if (stats) *stats = local;
  return st;
}

ecs_status ecs_set_tuning(ecs_ctx *C, const ecs_tuning *t) {
  if (!C || !t) return ECS_EINVAL;
  const bool f32 = C->have_prec && C->prec.vcycle_dtype == ECS_F32;
  const bool down_ok = (t->down_rows >= 2 && t->down_rows <= 6) || t->down_rows == 8 || (t->down_rows == 16 && f32);
  const bool up_ok = t->up_rows == 4 || t->up_rows == 8 || t->up_rows == 10 || t->up_rows == 12 || t->up_rows == 16 ||
                     t->up_rows == 32;
  if (!down_ok || !up_ok) return fail(C, ECS_EINVAL, "unsupported tile height");
  if (t->tail_nodes < 3 || t->tail_nodes > kTailWideNodes)
    return fail(C, ECS_EINVAL, "tail_nodes must be in [3, 65]");
  if (t->small_grid < 3) return fail(C, ECS_EINVAL, "small_grid must be >= 3");
  if (t->pair_grid < 0) return fail(C, ECS_EINVAL, "pair_grid must be >= 0");
  if (t->fuse_updates != 0 && t->fuse_updates != 1) return fail(C, ECS_EINVAL, "fuse_updates must be 0 or 1");
  C->tune = *t;
  drop_graphs(C);
  return ECS_OK;
}

ecs_status ecs_get_tuning(ecs_ctx *C, ecs_tuning *t) {
  if (!C || !t) return ECS_EINVAL;
  *t = C->tune;
  return ECS_OK;
}

ecs_status ecs_set_graphs(ecs_ctx *C, int mode) {
  if (!C || mode < ECS_GRAPHS_NEVER || mode > ECS_GRAPHS_AUTO) return ECS_EINVAL;
  C->graph_mode = mode;
  if (mode == ECS_GRAPHS_NEVER) drop_graphs(C);
  return ECS_OK;
}

ecs_status ecs_copy_probe(const void *src, void *dst, size_t bytes, void *stream) {
  if (!src || !dst) return ECS_EINVAL;
  launch_copy_bytes(src, dst, bytes, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? ECS_OK : ECS_EDEVICE;
}

const char *ecs_last_error(const ecs_ctx *C) { return C ? C->err.c_str() : "null context"; }

void ecs_destroy(ecs_ctx *C) {
  if (!C) return;
  drop_graphs(C);
  if (C->capture) (void)hipStreamDestroy(C->capture);
  for (auto &T : C->timers)
    for (auto &e : T.ev) (void)hipEventDestroy(e);
  if (C->pinned) (void)hipHostFree(C->pinned);
  if (C->step_ev) (void)hipEventDestroy(C->step_ev);
  delete C;
}

}  // extern "C"
