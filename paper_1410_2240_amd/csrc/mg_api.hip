// C ABI and host driver of the multigrid pressure solve (declared in include/mg.h).
//
// The host side plans the hierarchy, carves the caller's workspace, queues kernels
// on the caller's stream and reads back one scalar (the residual norm) per cycle.
// It never allocates device memory; the only host allocation besides the context
// object is a small pinned buffer for those read-backs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "mg.h"
#include "mg_kernels.h"
#include "mg_plan.h"

namespace mg {
void symmetric_pinv(int n, std::vector<double>& a, double rtol, std::vector<double>& pinv);
bool graph_pinv(int n, const std::vector<double>& a, const std::vector<int>& component, double rtol,
                std::vector<double>& pinv);
}

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

#define MG_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) return fail(MG_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define MG_TRY(call)          \
  do {                        \
    int rc_ = (call);         \
    if (rc_ != MG_OK) return rc_; \
  } while (0)

constexpr double kPinvRtol = 1e-12;
constexpr double kBreakdownGrowth = 1e3;
// ||P f|| below this fraction of ||f|| is rounding left by the mean removal
constexpr double kZeroRhs = 64.0 * 2.220446049250313e-16;

// device scalar slots
enum {
  S_FMEAN = 0, S_FNORM2 = 1, S_RNORM2 = 2, S_PMEAN = 3, S_DW = 4, S_DR = 5, S_ZW = 6, S_ALPHA = 7, S_ALPHA_PREV = 8,
  S_COUNT = 9
};

struct Level {
  int n = 0, q = 0;
  double h = 0;
  double *bx = nullptr, *by = nullptr, *bz = nullptr, *f = nullptr, *e = nullptr, *t = nullptr;
  double* rt = nullptr;   // finest grid of a hierarchy built from rho: the density form
  float* rt32 = nullptr;  // the same in FP32 (mixed contexts, grids swept in one pass)
  uint8_t* mask = nullptr;
  float *bx32 = nullptr, *by32 = nullptr, *bz32 = nullptr, *f32 = nullptr, *e32 = nullptr, *t32 = nullptr;
};

template <typename T>
struct View {
  T *bx, *by, *bz, *f, *e, *t;
  const T* rt;   // finest grid of a hierarchy built from rho: the density form, else null
};

}  // namespace

struct mg_ctx {
  mg::Plan plan;
  int flags = 0;
  int L = 0;
  Level lv[mg::kMaxLevels];
  hipStream_t stream = nullptr;
  unsigned char* ws = nullptr;
  double* pinv = nullptr;
  double* partials = nullptr;
  double* scal = nullptr;
  long long* counters = nullptr;
  double *kr = nullptr, *kz = nullptr, *kd = nullptr, *kd2 = nullptr, *kw = nullptr;   // flexible-CG vectors
  double* kr2 = nullptr;   // a second residual (absent unless the plan holds one)
  double* kd3 = nullptr;   // a third direction (likewise)
  double* host = nullptr;   // pinned, S_COUNT doubles
  hipEvent_t read_done = nullptr;   // the last read-back of scalars has landed in host
  long long active = 0, dropped = 0;
  // Concurrent right-hand sides (mg_add_lanes): each lane is a context of its own that
  // shares this one's coefficients, masks and pseudo-inverse and owns its scratch, a
  // stream the library created, a read-back buffer and events.
  std::vector<mg_ctx*> lanes;
  bool own_stream = false;              // a lane: `stream` was created by the library
  hipEvent_t order_event = nullptr;     // joins this context's stream with the caller's
  int device = 0;                       // a lane: the device its stream belongs to

  View<double> v64(int l) const {
    const Level& a = lv[l];
    return {a.bx, a.by, a.bz, a.f, a.e, a.t, a.rt};
  }
  View<float> v32(int l) const {
    const Level& a = lv[l];
    return {a.bx32, a.by32, a.bz32, a.f32, a.e32, a.t32, a.rt32};
  }
  template <typename T>
  View<T> view(int l) const;
};

template <>
View<double> mg_ctx::view<double>(int l) const { return v64(l); }
template <>
View<float> mg_ctx::view<float>(int l) const { return v32(l); }

namespace {

template <typename T>
T* at(unsigned char* ws, size_t off) {
  return off == mg::kAbsent ? nullptr : reinterpret_cast<T*>(ws + off);
}

long long cells(const Level& a) { return static_cast<long long>(a.n) * a.n * a.n; }

// ---------------------------------------------------------------- V-cycle (T = double/float)

// `sweeps` red-black sweeps of A p = f on level l.  Grids of 64^3 and up use the one-pass
// fused sweep (32^3 and 64^3 grids with face arrays the block-per-workgroup sweep), which
// alternates p with the level's second buffer; an odd count ends with a copy back.
// Smaller grids use two in-place half-sweeps per sweep.  zero_in: p is known to
// be zero, so the first one-pass sweep does not read it (p's memory may then hold
// anything; half-sweep grids still need it zeroed).  first_done: the first sweep
// (p -> second buffer) has already been queued (see first_sweep), so start from its output.
// Grids whose sweeps run two to a pass: the density form (the finest grid of a context
// set up from rho, in its FP64 cycles and in a mixed context's FP32 cycles), 256^3 and up.
template <typename T>
bool two_sweep_grid(const mg_ctx* c, int l) {
  return c->view<T>(l).rt != nullptr && mg::fused2_supported(c->lv[l].q);
}

// What an FP64 two-sweep pass of flexible CG also does (launch_rbgs_fused2), and where
// the number of its partial sums goes.
struct ZwSums {
  mg::Fused2Extra x;
  int* nblocks;
};

template <typename T>
hipError_t launch_two_sweeps(const mg_ctx* c, int l, const T* pin, T* pout, const T* f, const double* fshift, int order,
                             bool zero_in, const ZwSums* zw = nullptr) {
  const Level& a = c->lv[l];
  return mg::launch_rbgs_fused2(pin, pout, f, c->view<T>(l).rt, a.q, a.h, order, fshift, zero_in ? 1 : 0, c->stream,
                                zw ? &zw->x : nullptr, zw ? zw->nblocks : nullptr);
}

template <typename T>
int smooth(mg_ctx* c, int l, T* p, const T* f, const double* fshift, int sweeps, int order, bool zero_in = false,
           bool first_done = false) {
  const Level& a = c->lv[l];
  const View<T> v = c->view<T>(l);
  const bool box = !v.rt && mg::box_sweep_supported(a.q);   // 32^3 and 64^3 from face arrays
  if (mg::fused_sweep_supported(a.q) || box) {
    T* src = first_done ? v.t : p;
    T* dst = first_done ? p : v.t;
    const bool two = two_sweep_grid<T>(c, l);
    int s = first_done ? (two ? 2 : 1) : 0;   // first_sweep queued one pass
    if (two) {   // pairs of sweeps in one pass each
      for (; s + 2 <= sweeps; s += 2) {
        MG_HIP(launch_two_sweeps<T>(c, l, src, dst, f, fshift, order, zero_in && s == 0));
        T* tmp = src;
        src = dst;
        dst = tmp;
      }
    }
    for (; s < sweeps; ++s) {
      if (box)
        MG_HIP(mg::launch_rbgs_box<T>(src, dst, f, v.bx, v.by, v.bz, a.q, a.h, order, fshift, zero_in && s == 0,
                                      c->stream));
      else
        MG_HIP(mg::launch_rbgs_fused<T>(src, dst, f, v.bx, v.by, v.bz, v.rt, a.q, a.h, order, fshift,
                                        zero_in && s == 0, c->stream));
      T* tmp = src;
      src = dst;
      dst = tmp;
    }
    if (src != p) MG_HIP(hipMemcpyAsync(p, src, sizeof(T) * cells(a), hipMemcpyDeviceToDevice, c->stream));
    return MG_OK;
  }
  for (int s = 0; s < sweeps; ++s) {
    for (int half = 0; half < 2; ++half) {
      const int colour = (order == MG_PRE) ? half : 1 - half;   // red = 0 first when pre-smoothing
      MG_HIP(mg::launch_rbgs_half<T>(p, f, v.bx, v.by, v.bz, a.q, a.h, colour, fshift, c->stream));
    }
  }
  return MG_OK;
}

template <typename T>
int residual_restrict(mg_ctx* c, int l, const T* p, const T* f, const double* fshift, T* fc, T* ec) {
  const Level& a = c->lv[l];
  const View<T> v = c->view<T>(l);
  if (mg::march_supported(a.q)) {
    MG_HIP(mg::launch_residual_restrict_march<T>(p, f, v.bx, v.by, v.bz, v.rt, a.q, a.h, fshift, fc, ec, c->stream));
    return MG_OK;
  }
  MG_HIP(mg::launch_residual_restrict<T>(p, f, v.bx, v.by, v.bz, v.rt, a.q, a.h, fshift, fc, ec, c->stream));
  return MG_OK;
}

// The first pre-smoothing sweep of a finest-grid cycle on a one-pass-swept grid: it
// writes only the grid's second buffer (p is read, or not at all with zero_in), so it can
// be queued before the host has read the convergence check, and the cycle then starts
// from its output (vcycle with first_done); if the check ends the solve, it is discarded.
// On a grid that sweeps two to a pass the whole pre-smoothing (both sweeps) is queued.
template <typename T>
int first_sweep(mg_ctx* c, T* p, const T* f, const double* fshift, bool zero_in) {
  const Level& a = c->lv[0];
  const View<T> v = c->view<T>(0);
  if (two_sweep_grid<T>(c, 0)) {
    MG_HIP(launch_two_sweeps<T>(c, 0, p, v.t, f, fshift, MG_PRE, zero_in));
    return MG_OK;
  }
  MG_HIP(mg::launch_rbgs_fused<T>(p, v.t, f, v.bx, v.by, v.bz, v.rt, a.q, a.h, MG_PRE, fshift, zero_in, c->stream));
  return MG_OK;
}

// zero_in: p enters as zero (a correction), see smooth(); first_done: see first_sweep();
// zw: only on a two-sweep grid, where the last pass also sums p . zw->w (flexible CG's z.w)
template <typename T>
int vcycle(mg_ctx* c, int l, T* p, const T* f, const double* fshift, bool zero_in = false, bool first_done = false,
           const ZwSums* zw = nullptr) {
  if (c->lv[l].n <= mg::kCoarseCycleMaxN) {
    // grids of 16^3 and below: the rest of the cycle in one single-workgroup launch
    mg::CoarseCycle<T> a{};
    a.nlev = c->L - l;
    for (int k = 0; k < a.nlev; ++k) {
      const Level& lv = c->lv[l + k];
      const View<T> v = c->view<T>(l + k);
      a.q[k] = lv.q;
      a.bx[k] = v.bx;
      a.by[k] = v.by;
      a.bz[k] = v.bz;
      a.mask[k] = lv.mask;
      a.f[k] = k == 0 ? const_cast<T*>(f) : v.f;
      a.e[k] = k == 0 ? p : v.e;
      a.h2[k] = static_cast<T>(lv.h * lv.h);
      a.inv_h2[k] = static_cast<T>(1.0 / (lv.h * lv.h));
    }
    a.pinv = c->pinv;
    a.fshift = fshift;
    MG_HIP(mg::launch_coarse_cycle<T>(a, c->stream));
    return MG_OK;
  }
  const View<T> next = c->view<T>(l + 1);
  if (two_sweep_grid<T>(c, l)) {
    // pre-smoothing p -> t in one pass (or already queued by first_sweep), restriction and
    // prolongation on t, post-smoothing t -> p in one pass: no copies
    T* t = c->view<T>(l).t;
    if (!first_done) MG_HIP(launch_two_sweeps<T>(c, l, p, t, f, fshift, MG_PRE, zero_in));
    MG_TRY(residual_restrict<T>(c, l, t, f, fshift, next.f, next.e));
    MG_TRY(vcycle<T>(c, l + 1, next.e, next.f, nullptr, true));
    MG_HIP(mg::launch_prolong_add<T>(next.e, t, c->lv[l].mask, c->lv[l].q, c->stream));
    MG_HIP(launch_two_sweeps<T>(c, l, t, p, f, fshift, MG_POST, false, zw));
    return MG_OK;
  }
  if (zw) return fail(MG_EINVAL, "z.w sums asked of a grid that does not sweep two to a pass");
  const Level& a = c->lv[l];
  const View<T> v = c->view<T>(l);
  if (!v.rt && mg::box_sweep_supported(a.q)) {
    // 32^3 and 64^3 from face arrays, four launches: pre-smoothing p -> t -> p, the second
    // sweep also restricting its residual; post-smoothing from p plus the prolongated
    // correction -> t -> p
    if (!first_done)
      MG_HIP(mg::launch_rbgs_box<T>(p, v.t, f, v.bx, v.by, v.bz, a.q, a.h, MG_PRE, fshift, zero_in, c->stream));
    MG_HIP(mg::launch_rbgs_box_restrict<T>(v.t, p, f, v.bx, v.by, v.bz, a.q, a.h, MG_PRE, fshift, next.f, next.e,
                                           c->stream));
    MG_TRY(vcycle<T>(c, l + 1, next.e, next.f, nullptr, true));
    MG_HIP(mg::launch_rbgs_box_prolong<T>(p, v.t, f, v.bx, v.by, v.bz, a.q, a.h, MG_POST, fshift, next.e, a.mask,
                                          c->stream));
    MG_HIP(mg::launch_rbgs_box<T>(v.t, p, f, v.bx, v.by, v.bz, a.q, a.h, MG_POST, fshift, 0, c->stream));
    return MG_OK;
  }
  MG_TRY(smooth<T>(c, l, p, f, fshift, 2, MG_PRE, zero_in, first_done));
  MG_TRY(residual_restrict<T>(c, l, p, f, fshift, next.f, next.e));
  MG_TRY(vcycle<T>(c, l + 1, next.e, next.f, nullptr, true));   // restriction zeroed next.e
  MG_HIP(mg::launch_prolong_add<T>(next.e, p, c->lv[l].mask, c->lv[l].q, c->stream));
  MG_TRY(smooth<T>(c, l, p, f, fshift, 2, MG_POST));
  return MG_OK;
}

// ---------------------------------------------------------------- reductions

int reduce(mg_ctx* c, int nparts, double scale, int slot) {
  MG_HIP(mg::launch_reduce_final(c->partials, nparts, scale, c->scal + slot, c->stream));
  return MG_OK;
}

// Read-backs in two halves: work queued between them runs while the host waits.
int issue_scalars(mg_ctx* c, int count) {
  MG_HIP(hipMemcpyAsync(c->host, c->scal, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  MG_HIP(hipEventRecord(c->read_done, c->stream));
  return MG_OK;
}

int wait_scalars(mg_ctx* c, double* out, int count) {
  MG_HIP(hipEventSynchronize(c->read_done));
  std::memcpy(out, c->host, sizeof(double) * count);
  return MG_OK;
}

int read_scalars(mg_ctx* c, double* out, int count) {
  MG_TRY(issue_scalars(c, count));
  return wait_scalars(c, out, count);
}

// ||r||^2 of the finest residual into scal[S_RNORM2]; optional FP32 copy of r (with
// e32 = 0) and FP64 copy (with z64 = 0)
int residual_norm(mg_ctx* c, const double* p, const double* f, const double* fshift, float* r32, float* e32,
                  double* r64 = nullptr, double* z64 = nullptr) {
  const Level& a = c->lv[0];
  int nb = 0;
  if (mg::march_supported(a.q))
    MG_HIP(mg::launch_residual_norm_march(p, f, a.bx, a.by, a.bz, a.rt, a.q, a.h, fshift, r32, e32, r64, z64,
                                          c->partials, &nb, c->stream));
  else
    MG_HIP(mg::launch_residual_norm(p, f, a.bx, a.by, a.bz, a.rt, a.q, a.h, fshift, r32, e32, r64, z64, c->partials,
                                    &nb, c->stream));
  return reduce(c, nb, 1.0, S_RNORM2);
}

double* part(mg_ctx* c, int set) { return c->partials + static_cast<size_t>(set) * mg::kNumPartials; }

int reduce_set(mg_ctx* c, int set, int nparts, int slot) {
  MG_HIP(mg::launch_reduce_final(part(c, set), nparts, 1.0, c->scal + slot, c->stream));
  return MG_OK;
}

int check_prec(mg_ctx* c, int prec) {
  if (prec != MG_PREC_F64 && prec != MG_PREC_F32) return fail(MG_EINVAL, "prec must be MG_PREC_F64 or MG_PREC_F32");
  if (prec == MG_PREC_F32 && !(c->flags & MG_MIXED))
    return fail(MG_EINVAL, "FP32 arrays exist only in contexts set up with MG_MIXED");
  return MG_OK;
}

// One right-hand side.  hist has room for max_cycles + 1 entries.
int solve_one(mg_ctx* c, const double* f, double* p, double tol, int max_cycles, double* hist, int* n_hist,
              double* removed_mean, double* final_relres, int* cycles) {
  const Level& a = c->lv[0];
  const double* fshift = c->scal + S_FMEAN;
  int nb = 0;
  // P f: fluid mean of f (applied on the fly by every finest-grid kernel) and ||P f||
  MG_HIP(mg::launch_masked_sum(f, a.mask, a.q, 0, nullptr, c->partials, &nb, c->stream));
  MG_TRY(reduce(c, nb, 1.0 / static_cast<double>(c->active), S_FMEAN));
  MG_HIP(mg::launch_masked_sum(f, a.mask, a.q, 1, fshift, c->partials, &nb, c->stream));
  MG_TRY(reduce(c, nb, 1.0, S_FNORM2));
  MG_HIP(mg::launch_gauge(p, a.mask, a.q, nullptr, c->stream));   // initial guess: 0 in the body
  const bool mixed = (c->flags & MG_MIXED) != 0;
  // the residual pass also leaves the FP32 copy of r that the next FP32 cycle solves for
  float* r32 = mixed ? a.f32 : nullptr;
  float* e32 = mixed ? a.e32 : nullptr;
  // corrections enter their cycle as zero; a one-pass-swept finest grid does not read
  // them, so the passes before the cycle need not clear them
  const bool zin = mg::fused_sweep_supported(a.q);
  float* e32_zero = zin ? nullptr : e32;
  MG_TRY(residual_norm(c, p, f, fshift, r32, e32_zero));
  // The next cycle's first finest-grid sweep is queued before each convergence check is
  // read back (first_sweep), so the GPU does not idle while the host decides.
  const bool spec = mg::fused_sweep_supported(a.q) && a.n > mg::kCoarseCycleMaxN;
  const bool krylov = (c->flags & MG_KRYLOV) != 0;
  auto cycle_first_sweep = [&]() -> int {
    if (mixed) return first_sweep<float>(c, e32, r32, nullptr, true);
    return first_sweep<double>(c, p, f, fshift, false);
  };
  bool ahead = false;   // the next cycle's first sweep is queued
  double s[3];
  MG_TRY(issue_scalars(c, 3));
  if (spec && !krylov && max_cycles > 0) {
    MG_TRY(cycle_first_sweep());
    ahead = true;
  }
  MG_TRY(wait_scalars(c, s, 3));
  *removed_mean = s[S_FMEAN];
  const double nf = std::sqrt(s[S_FNORM2]);
  // ||f|| over the fluid cells from ||P f||^2 + (fluid cells) x mean^2, without a pass
  const double nf_all = std::sqrt(s[S_FNORM2] + static_cast<double>(c->active) * s[S_FMEAN] * s[S_FMEAN]);
  int nh = 0;
  *cycles = 0;
  if (!(nf > kZeroRhs * nf_all)) {   // P f = 0 to rounding (f = 0, f constant): p = 0
    MG_HIP(hipMemsetAsync(p, 0, sizeof(double) * cells(a), c->stream));
    if (hist) hist[0] = 0.0;
    *n_hist = 1;
    *final_relres = 0.0;
    return std::isfinite(nf) ? MG_OK : fail(MG_EBREAKDOWN, "right-hand side is not finite");
  }
  double r = std::sqrt(s[S_RNORM2]) / nf;
  const double r0 = r;
  if (hist) hist[nh] = r;
  ++nh;
  int status = MG_OK;
  if (c->flags & MG_KRYLOV) {
    // flexible CG: r, z, two directions and w in the workspace; z = V(r) in FP64, or V32
    // on float(r).  One step: r -= alpha w (alpha = d.r / d.w); the convergence check;
    // z = V(r); z.w; then one pass forms the new direction d' = z + beta d (beta =
    // -z.w / d.w) in the other direction buffer, w = A d', d'.w and d'.r, and the update
    // p += alpha d deferred from the step before (the last one is applied on exit).
    double *kr = c->kr, *kz = c->kz, *kw = c->kw;
    // p's update every second step where the workspace holds a third direction: the
    // step that skips it leaves its direction in place for the next one (three buffers
    // in turn instead of two)
    const bool defer = c->kd3 != nullptr && mg::fcgx_defer_supported(a.rt, a.q);
    double* dirs[3] = {c->kd, c->kd2, c->kd3};
    int cur = 0;   // dirs[cur] holds the current direction
    auto next_dir = [&](int i) { return defer ? (i + 1) % 3 : 1 - i; };
    int nx = 0;    // direction passes after the first
    const int q = a.q;
    const float* z32 = mixed ? e32 : nullptr;
    const double* z64 = mixed ? nullptr : kz;
    auto precondition = [&](bool first_done) -> int {
      if (mixed) return vcycle<float>(c, 0, e32, r32, nullptr, true, first_done);
      return vcycle<double>(c, 0, kz, kr, nullptr, true, first_done);
    };
    // FP64 preconditioning on a two-sweep finest grid: z.w comes out of its last pass,
    // and, where the workspace holds a second residual, the residual update out of its first
    const bool zw_fused = !mixed && two_sweep_grid<double>(c, 0) && a.n > mg::kCoarseCycleMaxN;
    const bool ru_fused = zw_fused && c->kr2 != nullptr;
    double* kr_other = c->kr2;
    auto precondition_first_sweep = [&]() -> int {
      if (mixed) return first_sweep<float>(c, e32, r32, nullptr, true);
      return first_sweep<double>(c, kz, kr, nullptr, true);
    };
    // the new direction from z and the current one, with w = A d' and the two sums into
    // partial sets 0 and 1; first: d' = z, no update of p
    auto direction = [&](bool first) -> int {
      const double* s_zw = first ? nullptr : c->scal + S_ZW;
      const double* s_dw = first ? nullptr : c->scal + S_DW;
      double* dnew = dirs[next_dir(cur)];
      int nb = 0;
      if (mg::march_supported(q)) {
        mg::FcgxDefer df;
        const bool use_df = defer && !first;
        if (use_df) {
          ++nx;
          if (nx & 1) {   // this step's update of p waits for the next one
            df.skip = true;
            df.s_alpha_save = c->scal + S_ALPHA_PREV;
          } else {        // the one the step before left, then this one
            df.d_prev = dirs[(cur + 2) % 3];
            df.s_alpha_prev = c->scal + S_ALPHA_PREV;
          }
        }
        MG_HIP(mg::launch_fcg_x_march(z64, z32, dirs[cur], dnew, p, s_zw, s_dw, c->scal + S_ALPHA, kr, a.bx, a.by,
                                      a.bz, a.rt, q, a.h, kw, part(c, 0), part(c, 1), &nb, c->stream,
                                      use_df ? &df : nullptr));
      } else {
        MG_HIP(mg::launch_fcg_dir(z64, z32, dirs[cur], dnew, first ? nullptr : p, s_zw, s_dw, c->scal + S_ALPHA, q,
                                  c->stream));
        MG_HIP(mg::launch_fcg_aw(dnew, kr, a.bx, a.by, a.bz, a.rt, q, a.h, kw, part(c, 0), part(c, 1), &nb,
                                 c->stream));
      }
      cur = next_dir(cur);
      MG_TRY(reduce_set(c, 0, nb, S_DW));
      MG_TRY(reduce_set(c, 1, nb, S_DR));
      return MG_OK;
    };
    double* kz_zero = (mixed || zin) ? nullptr : kz;
    if (std::isfinite(r) && r > tol && max_cycles > 0) {
      // the first residual pass also wrote r (and zeroed the preconditioner output)
      MG_TRY(residual_norm(c, p, f, fshift, r32, e32_zero, kr, kz_zero));
      MG_TRY(precondition(false));
      MG_TRY(direction(true));
    }
    while (std::isfinite(r) && r > tol && *cycles < max_cycles) {
      int nb = 0;
      if (ru_fused) {
        // the preconditioner's first pass (z = 0 in, the finest grid's second buffer out)
        // also forms r - alpha w, into the other residual buffer, and its norm
        ZwSums ru{{}, &nb};
        ru.x.w = kw;
        ru.x.partials = part(c, 2);
        ru.x.rnew = kr_other;
        ru.x.s_dr = c->scal + S_DR;
        ru.x.s_dw = c->scal + S_DW;
        ru.x.s_alpha = c->scal + S_ALPHA;
        MG_HIP(launch_two_sweeps<double>(c, 0, kz, a.t, kr, nullptr, MG_PRE, true, &ru));
        std::swap(kr, kr_other);
      } else {
        MG_HIP(mg::launch_fcg_rupdate(kr, kw, c->scal + S_DR, c->scal + S_DW, c->scal + S_ALPHA, q, kz_zero,
                                      mixed ? r32 : nullptr, mixed ? e32_zero : nullptr, part(c, 2), &nb, c->stream));
      }
      MG_TRY(reduce_set(c, 2, nb, S_RNORM2));
      ++*cycles;
      double sn[8];
      MG_TRY(issue_scalars(c, 8));
      ahead = spec && *cycles < max_cycles && !ru_fused;
      if (ahead) MG_TRY(precondition_first_sweep());
      MG_TRY(wait_scalars(c, sn, 8));
      r = std::sqrt(sn[S_RNORM2]) / nf;
      if (hist) hist[nh] = r;
      ++nh;
      const bool broke = !std::isfinite(r) || !(sn[S_DW] < 0.0) || r > kBreakdownGrowth * std::fmax(r0, 1.0);
      if (broke || r <= tol || *cycles >= max_cycles) {
        // p += alpha d of this step, which the next direction pass would have applied
        // (after the update the last direction pass left, if it left one)
        if (defer && (nx & 1))
          MG_HIP(mg::launch_fcg_padd2(p, dirs[(cur + 2) % 3], c->scal + S_ALPHA_PREV, dirs[cur], c->scal + S_ALPHA, q,
                                      c->stream));
        else
          MG_HIP(mg::launch_fcg_padd(p, dirs[cur], c->scal + S_ALPHA, q, c->stream));
        if (broke)
          status = fail(MG_EBREAKDOWN, "flexible CG breakdown after %d steps (residual %g, d.Ad %g)", *cycles, r,
                        sn[S_DW]);
        break;
      }
      if (zw_fused) {   // z.w from the preconditioner's last pass
        ZwSums zw{{}, &nb};
        zw.x.w = kw;
        zw.x.partials = part(c, 3);
        MG_TRY(vcycle<double>(c, 0, kz, kr, nullptr, true, ahead || ru_fused, &zw));
      } else {
        MG_TRY(precondition(ahead));
        MG_HIP(mg::launch_fcg_zw(z64, z32, kw, q, part(c, 3), &nb, c->stream));
      }
      MG_TRY(reduce_set(c, 3, nb, S_ZW));
      MG_TRY(direction(false));
    }
  }
  // Mixed refinement on a density-form finest grid: the FP64 update p + e and the next
  // residual in one pass, p alternating with the finest grid's second FP64 buffer (free
  // while the cycles run in FP32); the last iterate is copied back into p below.  Only
  // where the pass need not also clear e32 (one-pass-swept grids), since it reads e32.
  const bool fuse_update = mixed && a.rt && mg::march_supported(a.q) && e32_zero == nullptr;
  double* cur = p;
  while (!(c->flags & MG_KRYLOV) && std::isfinite(r) && r > tol && *cycles < max_cycles) {
    if (mixed) {
      // FP32 V-cycle for the correction from the FP32 copy of the FP64 residual, FP64 update
      MG_TRY(vcycle<float>(c, 0, e32, r32, nullptr, true, ahead));
      if (fuse_update) {
        double* next = cur == p ? a.t : p;
        int nbu = 0;
        MG_HIP(mg::launch_residual_norm_update_march(cur, e32, next, f, a.rt, a.q, a.h, fshift, r32, e32_zero,
                                                     c->partials, &nbu, c->stream));
        MG_TRY(reduce(c, nbu, 1.0, S_RNORM2));
        cur = next;
      } else {
        MG_HIP(mg::launch_update_p(p, e32, a.mask, a.q, c->stream));
        MG_TRY(residual_norm(c, p, f, fshift, r32, e32_zero));
      }
    } else {
      MG_TRY(vcycle<double>(c, 0, p, f, fshift, false, ahead));
      MG_TRY(residual_norm(c, p, f, fshift, r32, e32_zero));
    }
    ++*cycles;
    double sn[3];
    MG_TRY(issue_scalars(c, 3));
    ahead = spec && *cycles < max_cycles;
    if (ahead) MG_TRY(cycle_first_sweep());
    MG_TRY(wait_scalars(c, sn, 3));
    r = std::sqrt(sn[S_RNORM2]) / nf;
    if (hist) hist[nh] = r;
    ++nh;
    if (!std::isfinite(r) || r > kBreakdownGrowth * std::fmax(r0, 1.0)) {
      status = fail(MG_EBREAKDOWN, "residual %g after %d cycles (initial %g)", r, *cycles, r0);
      break;
    }
  }
  if (cur != p) MG_HIP(hipMemcpyAsync(p, cur, sizeof(double) * cells(a), hipMemcpyDeviceToDevice, c->stream));
  if (status == MG_OK && r > tol)
    status = fail(MG_ENOCONV, "relative residual %g > tol %g after %d cycles", r, tol, *cycles);
  // gauge: zero fluid mean, 0 in the body
  MG_HIP(mg::launch_masked_sum(p, a.mask, a.q, 0, nullptr, c->partials, &nb, c->stream));
  MG_TRY(reduce(c, nb, 1.0 / static_cast<double>(c->active), S_PMEAN));
  MG_HIP(mg::launch_gauge(p, a.mask, a.q, c->scal + S_PMEAN, c->stream));
  *n_hist = nh;
  *final_relres = r;
  return status;
}

// dense operator of the coarsest grid (host), column-major = row-major (symmetric)
void coarse_dense(const std::vector<double>& bx, const std::vector<double>& by, const std::vector<double>& bz,
                  const std::vector<uint8_t>& mask, int n, double h, std::vector<double>& A) {
  const int nc = n * n * n;
  A.assign(static_cast<size_t>(nc) * nc, 0.0);
  const double ih2 = 1.0 / (h * h);
  auto id = [n](int i, int j, int k) { return (k * n + j) * n + i; };
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const int c = id(i, j, k);
        if (!mask[c]) continue;
        const int nb[6] = {id((i + n - 1) % n, j, k), id((i + 1) % n, j, k), id(i, (j + n - 1) % n, k),
                           id(i, (j + 1) % n, k), k > 0 ? id(i, j, k - 1) : c, k < n - 1 ? id(i, j, k + 1) : c};
        const double b[6] = {bx[c], bx[nb[1]], by[c], by[nb[3]], bz[c], k < n - 1 ? bz[nb[5]] : 0.0};
        for (int f = 0; f < 6; ++f) {
          if (b[f] == 0.0) continue;
          A[static_cast<size_t>(c) * nc + nb[f]] += b[f] * ih2;
          A[static_cast<size_t>(c) * nc + c] -= b[f] * ih2;
        }
      }
}

// connected components of the active cells of the coarsest grid over faces with
// beta > 0; inactive cells get -1
std::vector<int> coarse_components(const std::vector<double>& bx, const std::vector<double>& by,
                                   const std::vector<double>& bz, const std::vector<uint8_t>& mask, int n) {
  const int nc = n * n * n;
  std::vector<int> comp(nc, -1);
  auto id = [n](int i, int j, int k) { return (k * n + j) * n + i; };
  int next = 0;
  std::vector<int> stack;
  for (int s0 = 0; s0 < nc; ++s0) {
    if (!mask[s0] || comp[s0] >= 0) continue;
    comp[s0] = next;
    stack.assign(1, s0);
    while (!stack.empty()) {
      const int c = stack.back();
      stack.pop_back();
      const int i = c % n, j = (c / n) % n, k = c / (n * n);
      const int nb[6] = {id((i + n - 1) % n, j, k), id((i + 1) % n, j, k), id(i, (j + n - 1) % n, k),
                         id(i, (j + 1) % n, k), k > 0 ? id(i, j, k - 1) : -1, k < n - 1 ? id(i, j, k + 1) : -1};
      const double b[6] = {bx[c], bx[nb[1]], by[c], by[nb[3]], bz[c], k < n - 1 ? bz[nb[5]] : 0.0};
      for (int f = 0; f < 6; ++f)
        if (nb[f] >= 0 && b[f] > 0.0 && mask[nb[f]] && comp[nb[f]] < 0) {
          comp[nb[f]] = next;
          stack.push_back(nb[f]);
        }
    }
    ++next;
  }
  return comp;
}

int check_level(mg_ctx* c, int level, int need_coarser) {
  if (!c) return fail(MG_EINVAL, "null context");
  if (level < 0 || level >= c->L - need_coarser) return fail(MG_EINVAL, "level %d out of range", level);
  return MG_OK;
}

}  // namespace

extern "C" void mg_destroy(mg_ctx* ctx);

namespace {

// Shared by mg_setup (finest face coefficients given) and mg_setup_from_rho (cell
// density given; face products formed here, or density and areas coarsened apart).
int setup_impl(mg_ctx** out, void* workspace, size_t ws_bytes, const double* bx, const double* by, const double* bz,
               const double* rho, const uint8_t* mask, const int dims[3], double h, int flags, void* hip_stream) {
  if (!out) return fail(MG_EINVAL, "null output pointer");
  *out = nullptr;
  int n = 0;
  if (mg::validate_dims(dims, &n) != 0) return fail(MG_EINVAL, "dims must be equal powers of two in [8, 1024]");
  if (!mask || (!rho && (!bx || !by || !bz))) return fail(MG_EINVAL, "null array pointer");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(MG_EINVAL, "h must be positive and finite");
  if (flags < 0 || flags > (MG_MIXED | MG_KRYLOV | MG_COARSEN_DENSITY | MG_FROM_RHO))
    return fail(MG_EINVAL, "unknown flags %d", flags);
  const bool density = (flags & MG_COARSEN_DENSITY) != 0;
  if (density && !rho) return fail(MG_EINVAL, "density coarsening needs the cell density (mg_setup_from_rho)");
  if ((flags & MG_FROM_RHO) && !rho) return fail(MG_EINVAL, "MG_FROM_RHO is for mg_setup_from_rho");
  mg::Plan plan;
  if (mg::build_plan(n, flags, &plan) != 0) return fail(MG_EINVAL, "unsupported grid");
  if (!workspace) return fail(MG_EWORKSPACE, "null workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % mg::kAlign != 0) return fail(MG_EWORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < plan.total) return fail(MG_EWORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, plan.total);

  mg_ctx* c = new mg_ctx;
  c->plan = plan;
  c->flags = flags;
  c->L = plan.levels;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<unsigned char*>(workspace);
  for (int l = 0; l < c->L; ++l) {
    const mg::LevelPlan& lp = plan.lv[l];
    Level& a = c->lv[l];
    a.n = lp.n;
    a.q = lp.log2n;
    a.h = std::ldexp(h, l);
    a.bx = at<double>(c->ws, lp.bx);
    a.by = at<double>(c->ws, lp.by);
    a.bz = at<double>(c->ws, lp.bz);
    a.mask = at<uint8_t>(c->ws, lp.mask);
    a.f = at<double>(c->ws, lp.f);
    a.e = at<double>(c->ws, lp.e);
    a.t = at<double>(c->ws, lp.t);
    a.bx32 = at<float>(c->ws, lp.bx32);
    a.by32 = at<float>(c->ws, lp.by32);
    a.bz32 = at<float>(c->ws, lp.bz32);
    a.f32 = at<float>(c->ws, lp.f32);
    a.e32 = at<float>(c->ws, lp.e32);
    a.t32 = at<float>(c->ws, lp.t32);
  }
  c->pinv = at<double>(c->ws, plan.pinv);
  c->partials = at<double>(c->ws, plan.partials);
  c->scal = at<double>(c->ws, plan.scalars);
  c->counters = at<long long>(c->ws, plan.counters);
  c->kr = at<double>(c->ws, plan.kr);
  c->kz = at<double>(c->ws, plan.kz);
  c->kd = at<double>(c->ws, plan.kd);
  c->kd2 = at<double>(c->ws, plan.kd2);
  c->kw = at<double>(c->ws, plan.kw);
  c->kr2 = at<double>(c->ws, plan.kr2);
  c->kd3 = at<double>(c->ws, plan.kd3);

  auto cleanup = [&](int rc) {
    mg_destroy(c);
    return rc;
  };
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host), sizeof(double) * S_COUNT, hipHostMallocDefault) !=
      hipSuccess) {
    c->host = nullptr;
    return cleanup(fail(MG_EHIP, "hipHostMalloc of the read-back buffer failed"));
  }
  if (hipEventCreateWithFlags(&c->read_done, hipEventDisableTiming) != hipSuccess) {
    c->read_done = nullptr;
    return cleanup(fail(MG_EHIP, "hipEventCreateWithFlags of the read-back event failed"));
  }
  hipStream_t s = c->stream;
  int rc = MG_OK;
  auto hip = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == MG_OK) rc = fail(MG_EHIP, "%s: %s", what, hipGetErrorString(e));
  };
  hip(hipMemsetAsync(c->counters, 0, 16 * sizeof(long long), s), "hipMemsetAsync(counters)");
  Level& f0 = c->lv[0];
  if (rho) {
    // density form of the finest coefficients, read by the finest-grid passes in place
    // of the three face arrays
    f0.rt = at<double>(c->ws, plan.lv[0].rt);
    if (density) {
      // open-face areas into the workspace, then validation and activity without
      // rewriting them, then the density form
      hip(mg::launch_coeffs_from_rho(nullptr, mask, f0.q, f0.bx, f0.by, f0.bz, s), "coeffs_from_rho");
      hip(mg::launch_setup_fine(f0.bx, f0.by, f0.bz, mask, f0.q, nullptr, nullptr, nullptr, f0.mask, c->counters, s),
          "setup_fine");
      hip(mg::launch_rho_tilde(rho, f0.mask, f0.q, f0.rt, s), "rho_tilde");
    } else {
      // face products, validation, activity and the density form in one pass
      hip(mg::launch_setup_from_rho(rho, mask, f0.q, f0.bx, f0.by, f0.bz, f0.mask, f0.rt, c->counters, s),
          "setup_from_rho");
    }
  } else {
    hip(mg::launch_setup_fine(bx, by, bz, mask, f0.q, f0.bx, f0.by, f0.bz, f0.mask, c->counters, s), "setup_fine");
  }
  if (rho) {
    if (plan.lv[0].rt32 != mg::kAbsent) {
      // the FP32 cycles form their finest faces from an FP32 copy (one-pass sweep grids,
      // so that smoother and residual use the same FP32 operator)
      if (!mg::fused_sweep_supported(f0.q)) return cleanup(fail(MG_EINVAL, "internal: FP32 density copy below 64^3"));
      f0.rt32 = at<float>(c->ws, plan.lv[0].rt32);
      hip(mg::launch_to_f32(f0.rt, f0.rt32, cells(f0), s), "to_f32(rt)");
    }
  }
  for (int l = 1; l < c->L; ++l) {
    const Level& a = c->lv[l - 1];
    Level& b = c->lv[l];
    hip(mg::launch_coarsen(a.bx, a.by, a.bz, a.mask, b.q, b.bx, b.by, b.bz, b.mask, s), "coarsen");
  }
  if (density) {
    // the coarsening section 3.1 rejects: density restricted cell centre to cell centre
    // (held in each level's second buffer), areas as above, faces re-formed per level
    for (int l = 1; l < c->L; ++l) {
      const double* fine_rho = l == 1 ? rho : c->lv[l - 1].t;
      hip(mg::launch_restrict_rho(fine_rho, c->lv[l - 1].mask, c->lv[l].q, c->lv[l].t, s), "restrict_rho");
    }
    for (int l = 0; l < c->L; ++l) {
      Level& a = c->lv[l];
      hip(mg::launch_area_to_beta(l == 0 ? rho : a.t, a.q, a.bx, a.by, a.bz, s), "area_to_beta");
    }
  }
  if (flags & MG_MIXED) {
    // (a finest grid with an FP32 density copy never reads its FP32 face arrays)
    for (int l = f0.rt32 ? 1 : 0; l < c->L; ++l) {
      const Level& a = c->lv[l];
      hip(mg::launch_to_f32(a.bx, a.bx32, cells(a), s), "to_f32");
      hip(mg::launch_to_f32(a.by, a.by32, cells(a), s), "to_f32");
      hip(mg::launch_to_f32(a.bz, a.bz32, cells(a), s), "to_f32");
    }
  }
  // coarsest operator to the host, FP64 pseudo-inverse back to the device
  const Level& cl = c->lv[c->L - 1];
  const int nc = static_cast<int>(cells(cl));
  std::vector<double> hbx(nc), hby(nc), hbz(nc), A, P;
  std::vector<uint8_t> hm(nc);
  long long cnt[3] = {0, 0, 0};
  hip(hipMemcpyAsync(hbx.data(), cl.bx, nc * sizeof(double), hipMemcpyDeviceToHost, s), "copy coarse bx");
  hip(hipMemcpyAsync(hby.data(), cl.by, nc * sizeof(double), hipMemcpyDeviceToHost, s), "copy coarse by");
  hip(hipMemcpyAsync(hbz.data(), cl.bz, nc * sizeof(double), hipMemcpyDeviceToHost, s), "copy coarse bz");
  hip(hipMemcpyAsync(hm.data(), cl.mask, nc, hipMemcpyDeviceToHost, s), "copy coarse mask");
  hip(hipMemcpyAsync(cnt, c->counters, sizeof cnt, hipMemcpyDeviceToHost, s), "copy counters");
  hip(hipStreamSynchronize(s), "hipStreamSynchronize(setup)");
  if (rc != MG_OK) return cleanup(rc);
  if (cnt[0] > 0)
    return cleanup(fail(MG_EINVAL, "%lld face coefficients are negative or not finite%s", cnt[0],
                        rho ? " (density must be positive and finite in fluid cells)" : ""));
  if (cnt[1] == 0) return cleanup(fail(MG_EINVAL, "no fluid cell has an open face"));
  c->active = cnt[1];
  c->dropped = cnt[2];
  coarse_dense(hbx, hby, hbz, hm, cl.n, cl.h, A);
  // the null space is known exactly from the graph; eigendecomposition only as fallback
  if (!mg::graph_pinv(nc, A, coarse_components(hbx, hby, hbz, hm, cl.n), 1e-14, P))
    mg::symmetric_pinv(nc, A, kPinvRtol, P);
  hip(hipMemcpyAsync(c->pinv, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice, s), "upload pinv");
  hip(hipStreamSynchronize(s), "hipStreamSynchronize(pinv)");
  if (rc != MG_OK) return cleanup(rc);
  *out = c;
  return MG_OK;
}

// One lane: a copy of ctx whose per-solve arrays live in `ws` (laid out by
// build_lane_plan) and whose work runs on a new non-blocking stream of `device`.
int make_lane(mg_ctx* ctx, unsigned char* ws, const mg::Plan& lp, int device, mg_ctx** out) {
  mg_ctx* c = new mg_ctx(*ctx);
  c->lanes.clear();
  c->host = nullptr;
  c->read_done = nullptr;
  c->order_event = nullptr;
  c->stream = nullptr;
  c->own_stream = false;
  c->device = device;
  for (int l = 0; l < c->L; ++l) {
    Level& a = c->lv[l];
    const mg::LevelPlan& p = lp.lv[l];
    a.f = at<double>(ws, p.f);
    a.e = at<double>(ws, p.e);
    a.t = at<double>(ws, p.t);
    a.f32 = at<float>(ws, p.f32);
    a.e32 = at<float>(ws, p.e32);
    a.t32 = at<float>(ws, p.t32);
  }
  c->partials = at<double>(ws, lp.partials);
  c->scal = at<double>(ws, lp.scalars);
  c->kr = at<double>(ws, lp.kr);
  c->kz = at<double>(ws, lp.kz);
  c->kd = at<double>(ws, lp.kd);
  c->kd2 = at<double>(ws, lp.kd2);
  c->kw = at<double>(ws, lp.kw);
  c->kr2 = at<double>(ws, lp.kr2);
  c->kd3 = at<double>(ws, lp.kd3);
  *out = c;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host), sizeof(double) * S_COUNT, hipHostMallocDefault) != hipSuccess) {
    c->host = nullptr;
    return fail(MG_EHIP, "hipHostMalloc of a lane's read-back buffer failed");
  }
  if (hipEventCreateWithFlags(&c->read_done, hipEventDisableTiming) != hipSuccess) {
    c->read_done = nullptr;
    return fail(MG_EHIP, "hipEventCreateWithFlags of a lane's read-back event failed");
  }
  if (hipEventCreateWithFlags(&c->order_event, hipEventDisableTiming) != hipSuccess) {
    c->order_event = nullptr;
    return fail(MG_EHIP, "hipEventCreateWithFlags of a lane's order event failed");
  }
  // non-blocking: no implicit ordering against the default stream, on which the caller
  // (and the context's own lane) may run; default priority
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(MG_EHIP, "hipStreamCreate failed");
  c->stream = s;
  c->own_stream = true;
  return MG_OK;
}

struct LaneResult {
  int rc = MG_OK, nh = 0, cyc = 0;
  double rm = 0.0, fr = 0.0;
  std::string err;
};

// Right-hand side b of a batch on lane w of W (lane 0 = the context itself on the
// caller's stream) runs solve_one unchanged, so each result is bit for bit that of the
// one-at-a-time loop.  A lane stops after an argument or HIP error, as that loop does.
void run_lane(mg_ctx* c, int w, int W, const double* f, double* p, int batch, long long n3, double tol,
              int max_cycles, double* hist, std::vector<LaneResult>* res) {
  if (w > 0 && hipSetDevice(c->device) != hipSuccess) {
    for (int b = w; b < batch; b += W) {
      (*res)[b].rc = MG_EHIP;
      (*res)[b].err = "hipSetDevice in a lane thread failed";
    }
    return;
  }
  for (int b = w; b < batch; b += W) {
    LaneResult& o = (*res)[b];
    double* hb = hist ? hist + static_cast<long long>(b) * (max_cycles + 1) : nullptr;
    o.rc = solve_one(c, f + b * n3, p + b * n3, tol, max_cycles, hb, &o.nh, &o.rm, &o.fr, &o.cyc);
    if (o.rc != MG_OK) o.err = g_error;
    if (o.rc == MG_EINVAL || o.rc == MG_EHIP) break;
  }
}

// mg_solve over lanes: the lane streams start after the caller's earlier work, one host
// thread per extra lane drives its share of the batch, and the caller's stream waits for
// every lane's last work before anything queued after this call.
int solve_lanes(mg_ctx* ctx, const double* f, double* p, int batch, double tol, int max_cycles, double* hist,
                std::vector<LaneResult>& res) {
  const int W = std::min(static_cast<int>(ctx->lanes.size()) + 1, batch);
  const long long n3 = cells(ctx->lv[0]);
  MG_HIP(hipEventRecord(ctx->order_event, ctx->stream));
  for (int w = 1; w < W; ++w) MG_HIP(hipStreamWaitEvent(ctx->lanes[w - 1]->stream, ctx->order_event, 0));
  std::vector<std::thread> threads;
  std::vector<int> unthreaded;   // lanes whose thread could not be started
  for (int w = 1; w < W; ++w) {
    try {
      threads.emplace_back(run_lane, ctx->lanes[w - 1], w, W, f, p, batch, n3, tol, max_cycles, hist, &res);
    } catch (...) {   // nothing may be thrown across the C ABI: run that lane from here
      unthreaded.push_back(w);
    }
  }
  run_lane(ctx, 0, W, f, p, batch, n3, tol, max_cycles, hist, &res);
  for (int w : unthreaded) run_lane(ctx->lanes[w - 1], w, W, f, p, batch, n3, tol, max_cycles, hist, &res);
  for (auto& t : threads) t.join();
  int rc = MG_OK;
  for (int w = 1; w < W; ++w) {
    mg_ctx* lane = ctx->lanes[w - 1];
    hipError_t e = hipEventRecord(lane->order_event, lane->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->stream, lane->order_event, 0);
    if (e != hipSuccess && rc == MG_OK) rc = fail(MG_EHIP, "joining lane %d: %s", w, hipGetErrorString(e));
  }
  return rc;
}

}  // namespace

// ---------------------------------------------------------------- a solve that allocates nothing

// mg_solve_static keeps the arrays one solve writes (the layout of one lane,
// build_lane_plan) in this file-scope device array instead of the context's workspace.
// Every GPU the library runs on holds its own copy until the process ends.  In host
// code the name `scratch` is a host-side stand-in, not the device memory: the device
// address comes from hipGetSymbolAddress, once per device with that device current,
// and only that address is handed to kernels.
constexpr size_t kStaticScratchBytes = static_cast<size_t>(32) << 20;
constexpr int kMaxStaticDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mutex;
unsigned char* g_scratch_ptr[kMaxStaticDevices] = {};

int static_scratch(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxStaticDevices) return fail(MG_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(MG_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return MG_OK;
}

// Points a context's per-solve arrays into another block laid out by build_lane_plan
// and puts the context's own back on destruction (no allocation either way).
class ScratchSwap {
 public:
  ScratchSwap(mg_ctx* c, unsigned char* base, const mg::Plan& lp) : c_(c) {
    for (int l = 0; l < c->L; ++l) saved_[l] = c->lv[l];
    partials_ = c->partials;
    scal_ = c->scal;
    kr_ = c->kr;
    kz_ = c->kz;
    kd_ = c->kd;
    kd2_ = c->kd2;
    kw_ = c->kw;
    kr2_ = c->kr2;
    kd3_ = c->kd3;
    for (int l = 0; l < c->L; ++l) {
      Level& a = c->lv[l];
      const mg::LevelPlan& q = lp.lv[l];
      a.f = l > 0 ? at<double>(base, q.f) : a.f;
      a.e = l > 0 ? at<double>(base, q.e) : a.e;
      a.t = at<double>(base, q.t);
      if (c->flags & MG_MIXED) {
        a.f32 = at<float>(base, q.f32);
        a.e32 = at<float>(base, q.e32);
        a.t32 = at<float>(base, q.t32);
      }
    }
    c->partials = at<double>(base, lp.partials);
    c->scal = at<double>(base, lp.scalars);
    c->kr = at<double>(base, lp.kr);
    c->kz = at<double>(base, lp.kz);
    c->kd = at<double>(base, lp.kd);
    c->kd2 = at<double>(base, lp.kd2);
    c->kw = at<double>(base, lp.kw);
    c->kr2 = at<double>(base, lp.kr2);
    c->kd3 = at<double>(base, lp.kd3);
  }
  ~ScratchSwap() {
    for (int l = 0; l < c_->L; ++l) c_->lv[l] = saved_[l];
    c_->partials = partials_;
    c_->scal = scal_;
    c_->kr = kr_;
    c_->kz = kz_;
    c_->kd = kd_;
    c_->kd2 = kd2_;
    c_->kw = kw_;
    c_->kr2 = kr2_;
    c_->kd3 = kd3_;
  }
  ScratchSwap(const ScratchSwap&) = delete;
  ScratchSwap& operator=(const ScratchSwap&) = delete;

 private:
  mg_ctx* c_;
  Level saved_[mg::kMaxLevels];
  double *partials_, *scal_, *kr_, *kz_, *kd_, *kd2_, *kw_, *kr2_, *kd3_;
};

}  // namespace

extern "C" {

const char* mg_last_error(void) { return g_error.c_str(); }

size_t mg_workspace_size(const int dims[3], int flags) {
  int n = 0;
  mg::Plan plan;
  if (mg::validate_dims(dims, &n) != 0 || mg::build_plan(n, flags, &plan) != 0) return 0;
  return plan.total;
}

int mg_coeffs_from_rho(const double* rho, const uint8_t* mask, const int dims[3], double* bx, double* by, double* bz,
                       void* hip_stream) {
  int n = 0;
  if (mg::validate_dims(dims, &n) != 0) return fail(MG_EINVAL, "dims must be equal powers of two in [8, 1024]");
  if (!rho || !mask || !bx || !by || !bz) return fail(MG_EINVAL, "null array pointer");
  int q = 0;
  while ((1 << q) < n) ++q;
  MG_HIP(mg::launch_coeffs_from_rho(rho, mask, q, bx, by, bz, static_cast<hipStream_t>(hip_stream)));
  return MG_OK;
}


int mg_setup(mg_ctx** out, void* workspace, size_t ws_bytes, const double* bx, const double* by, const double* bz,
             const uint8_t* mask, const int dims[3], double h, int flags, void* hip_stream) {
  return setup_impl(out, workspace, ws_bytes, bx, by, bz, nullptr, mask, dims, h, flags, hip_stream);
}

int mg_cut_cells(const double* psi, const int dims[3], int samples, double* ax, double* ay, double* az,
                 double* vol, int32_t* merge_to, void* hip_stream) {
  int n = 0;
  if (mg::validate_dims(dims, &n) != 0) return fail(MG_EINVAL, "dims must be equal powers of two in [8, 1024]");
  if (!psi || !ax || !ay || !az || !vol || !merge_to) return fail(MG_EINVAL, "null array pointer");
  if (samples != 2 && samples != 4 && samples != 8 && samples != 16)
    return fail(MG_EINVAL, "samples must be 2, 4, 8 or 16 (got %d)", samples);
  int q = 0;
  while ((1 << q) < n) ++q;
  MG_HIP(mg::launch_cut_cells(psi, q, samples, ax, ay, az, vol, merge_to, static_cast<hipStream_t>(hip_stream)));
  return MG_OK;
}

int mg_cut_coeffs(const double* rho, const double* ax, const double* ay, const double* az, const double* vol,
                  const int32_t* merge_to, const int dims[3], double* bx, double* by, double* bz, uint8_t* mask,
                  void* hip_stream) {
  int n = 0;
  if (mg::validate_dims(dims, &n) != 0) return fail(MG_EINVAL, "dims must be equal powers of two in [8, 1024]");
  if (!rho || !ax || !ay || !az || !vol || !merge_to || !bx || !by || !bz || !mask)
    return fail(MG_EINVAL, "null array pointer");
  int q = 0;
  while ((1 << q) < n) ++q;
  MG_HIP(mg::launch_cut_coeffs(rho, ax, ay, az, vol, merge_to, q, bx, by, bz, mask,
                               static_cast<hipStream_t>(hip_stream)));
  return MG_OK;
}

int mg_merge_rhs(const int32_t* merge_to, const double* f, double* f_merged, const int dims[3], void* hip_stream) {
  int n = 0;
  if (mg::validate_dims(dims, &n) != 0) return fail(MG_EINVAL, "dims must be equal powers of two in [8, 1024]");
  if (!merge_to || !f || !f_merged) return fail(MG_EINVAL, "null array pointer");
  if (f == f_merged) return fail(MG_EINVAL, "f_merged must not alias f");
  int q = 0;
  while ((1 << q) < n) ++q;
  MG_HIP(mg::launch_merge_rhs(merge_to, f, f_merged, q, static_cast<hipStream_t>(hip_stream)));
  return MG_OK;
}

int mg_merge_fill(const int32_t* merge_to, double* p, const int dims[3], void* hip_stream) {
  int n = 0;
  if (mg::validate_dims(dims, &n) != 0) return fail(MG_EINVAL, "dims must be equal powers of two in [8, 1024]");
  if (!merge_to || !p) return fail(MG_EINVAL, "null array pointer");
  int q = 0;
  while ((1 << q) < n) ++q;
  MG_HIP(mg::launch_merge_fill(merge_to, p, q, static_cast<hipStream_t>(hip_stream)));
  return MG_OK;
}

int mg_setup_from_rho(mg_ctx** out, void* workspace, size_t ws_bytes, const double* rho, const uint8_t* mask,
                      const int dims[3], double h, int flags, void* hip_stream) {
  if (!rho) return fail(MG_EINVAL, "null density pointer");
  return setup_impl(out, workspace, ws_bytes, nullptr, nullptr, nullptr, rho, mask, dims, h, flags, hip_stream);
}

int mg_set_stream(mg_ctx* ctx, void* hip_stream) {
  if (!ctx) return fail(MG_EINVAL, "null context");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return MG_OK;
}

int mg_solve(mg_ctx* ctx, const double* f, double* p, int batch, double tol, int max_cycles, double* hist,
             int* n_hist, mg_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return fail(MG_EINVAL, "null context");
  if (!f || !p) return fail(MG_EINVAL, "null array pointer");
  if (batch < 1) return fail(MG_EINVAL, "batch must be >= 1");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MG_EINVAL, "tol must be positive and finite");
  if (max_cycles < 0) return fail(MG_EINVAL, "max_cycles must be >= 0");
  std::vector<LaneResult> res(batch);
  if (!ctx->lanes.empty() && batch > 1) {
    MG_TRY(solve_lanes(ctx, f, p, batch, tol, max_cycles, hist, res));
  } else {
    run_lane(ctx, 0, 1, f, p, batch, cells(ctx->lv[0]), tol, max_cycles, hist, &res);
  }
  // outcomes in batch order: the first argument or HIP error ends the call; otherwise
  // the status and message of the first item that did not converge
  int status = MG_OK, total_cycles = 0, first_bad = -1;
  double removed = 0.0, worst = 0.0;
  for (int b = 0; b < batch; ++b) {
    const LaneResult& o = res[b];
    if (n_hist) n_hist[b] = o.nh;
    total_cycles += o.cyc;
    removed = o.rm;
    worst = std::fmax(worst, o.fr);
    if (o.rc == MG_EINVAL || o.rc == MG_EHIP) {
      g_error = o.err;
      return o.rc;
    }
    if (o.rc != MG_OK && status == MG_OK) {
      status = o.rc;
      first_bad = b;
    }
  }
  if (first_bad >= 0) g_error = res[first_bad].err;
  if (stats) {
    stats->cycles = total_cycles;
    stats->levels = ctx->L;
    stats->active_cells = ctx->active;
    stats->dropped_cells = ctx->dropped;
    stats->removed_mean = removed;
    stats->final_relres = worst;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->ws_bytes = ctx->plan.total;
  }
  return status;
}

int mg_solve_static(mg_ctx* ctx, const double* f, double* p, int batch, double tol, int max_cycles, double* hist,
                    int* n_hist, mg_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return fail(MG_EINVAL, "null context");
  if (!f || !p) return fail(MG_EINVAL, "null array pointer");
  if (batch < 1) return fail(MG_EINVAL, "batch must be >= 1");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MG_EINVAL, "tol must be positive and finite");
  if (max_cycles < 0) return fail(MG_EINVAL, "max_cycles must be >= 0");
  mg::Plan lp;
  if (mg::build_lane_plan(ctx->lv[0].n, ctx->flags, &lp) != 0) return fail(MG_EINVAL, "unsupported grid");
  if (lp.total > kStaticScratchBytes)
    return fail(MG_EINVAL,
                "mg_solve_static: a %d^3 solve with flags %d needs %zu bytes of scratch, more than the %zu-byte "
                "static scratch (up to 128^3 in FP64, 64^3 with MG_MIXED or MG_KRYLOV); use mg_solve",
                ctx->lv[0].n, ctx->flags, lp.total, kStaticScratchBytes);
  int device = 0;
  MG_HIP(hipGetDevice(&device));
  if (ctx->stream) {
    hipDevice_t sdev = 0;
    MG_HIP(hipStreamGetDevice(ctx->stream, &sdev));
    if (static_cast<int>(sdev) != device)
      return fail(MG_EINVAL, "the context's stream is on device %d, the current device is %d", static_cast<int>(sdev),
                  device);
  }
  unsigned char* base = nullptr;
  MG_TRY(static_scratch(device, &base));
  const long long n3 = cells(ctx->lv[0]);
  int status = MG_OK, total_cycles = 0;
  double removed = 0.0, worst = 0.0;
  char first_msg[512] = "";
  {
    ScratchSwap swap(ctx, base, lp);
    for (int b = 0; b < batch; ++b) {
      double* hb = hist ? hist + static_cast<long long>(b) * (max_cycles + 1) : nullptr;
      int nh = 0, cyc = 0;
      double rm = 0.0, fr = 0.0;
      const int rc = solve_one(ctx, f + b * n3, p + b * n3, tol, max_cycles, hb, &nh, &rm, &fr, &cyc);
      if (n_hist) n_hist[b] = nh;
      if (rc == MG_EINVAL || rc == MG_EHIP) return rc;   // g_error holds the message
      total_cycles += cyc;
      removed = rm;
      worst = std::fmax(worst, fr);
      if (rc != MG_OK && status == MG_OK) {
        status = rc;
        std::snprintf(first_msg, sizeof first_msg, "%s", g_error.c_str());
      }
    }
  }
  if (status != MG_OK) g_error = first_msg;
  if (stats) {
    stats->cycles = total_cycles;
    stats->levels = ctx->L;
    stats->active_cells = ctx->active;
    stats->dropped_cells = ctx->dropped;
    stats->removed_mean = removed;
    stats->final_relres = worst;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->ws_bytes = ctx->plan.total;
  }
  return status;
}

int mg_apply(mg_ctx* ctx, const double* p, double* Ap, int batch) {
  if (!ctx) return fail(MG_EINVAL, "null context");
  if (!p || !Ap || batch < 1) return fail(MG_EINVAL, "bad arguments");
  const Level& a = ctx->lv[0];
  for (int b = 0; b < batch; ++b)
    MG_HIP(mg::launch_apply(p + b * cells(a), a.bx, a.by, a.bz, a.q, a.h, Ap + b * cells(a), ctx->stream));
  return MG_OK;
}

int mg_coeff_grad(mg_ctx* ctx, const double* mu, const double* p, int batch, double* gbx, double* gby, double* gbz,
                  double* grho) {
  if (!ctx) return fail(MG_EINVAL, "null context");
  if (!mu || !p || batch < 1) return fail(MG_EINVAL, "bad arguments");
  const Level& a = ctx->lv[0];
  MG_HIP(mg::launch_coeff_grad(mu, p, batch, a.bx, a.by, a.bz, a.mask, a.q, a.h, gbx, gby, gbz, grho, ctx->stream));
  return MG_OK;
}

int mg_divergence(mg_ctx* ctx, const double* ux, const double* uy, const double* uz, const double* rx,
                  const double* ry, const double* rz, double dt, double* f) {
  if (!ctx) return fail(MG_EINVAL, "null context");
  if (!ux || !uy || !uz || !f) return fail(MG_EINVAL, "null array pointer");
  if ((rx || ry || rz) && !(rx && ry && rz)) return fail(MG_EINVAL, "give all three R components or none");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(MG_EINVAL, "dt must be positive and finite");
  const Level& a = ctx->lv[0];
  MG_HIP(mg::launch_divergence(ux, uy, uz, rx, ry, rz, dt, a.mask, a.q, a.h, f, ctx->stream));
  return MG_OK;
}

int mg_project(mg_ctx* ctx, double* ux, double* uy, double* uz, const double* rx, const double* ry, const double* rz,
               double dt, const double* p) {
  if (!ctx) return fail(MG_EINVAL, "null context");
  if (!ux || !uy || !uz || !p) return fail(MG_EINVAL, "null array pointer");
  if ((rx || ry || rz) && !(rx && ry && rz)) return fail(MG_EINVAL, "give all three R components or none");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(MG_EINVAL, "dt must be positive and finite");
  const Level& a = ctx->lv[0];
  MG_HIP(mg::launch_project(ux, uy, uz, rx, ry, rz, dt, p, a.bx, a.by, a.bz, a.mask, a.q, a.h, ctx->stream));
  return MG_OK;
}

void mg_destroy(mg_ctx* ctx) {
  if (!ctx) return;
  for (mg_ctx* lane : ctx->lanes) mg_destroy(lane);
  if (ctx->own_stream && ctx->stream) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamDestroy(ctx->stream);
  }
  if (ctx->host) (void)hipHostFree(ctx->host);
  if (ctx->read_done) (void)hipEventDestroy(ctx->read_done);
  if (ctx->order_event) (void)hipEventDestroy(ctx->order_event);
  delete ctx;
}

size_t mg_lane_workspace_size(const int dims[3], int flags) {
  int n = 0;
  mg::Plan plan;
  if (mg::validate_dims(dims, &n) != 0 || mg::build_lane_plan(n, flags, &plan) != 0) return 0;
  return plan.total;
}

int mg_add_lanes(mg_ctx* ctx, void* workspace, size_t ws_bytes, int lanes) {
  if (!ctx) return fail(MG_EINVAL, "null context");
  if (ctx->own_stream) return fail(MG_EINVAL, "a lane cannot have lanes");
  if (!ctx->lanes.empty()) return fail(MG_EINVAL, "this context already has %zu lanes", ctx->lanes.size());
  if (lanes < 1 || lanes > MG_MAX_LANES) return fail(MG_EINVAL, "lanes must be in [1, %d] (got %d)", MG_MAX_LANES, lanes);
  mg::Plan lp;
  if (mg::build_lane_plan(ctx->lv[0].n, ctx->flags, &lp) != 0) return fail(MG_EINVAL, "unsupported grid");
  if (!workspace) return fail(MG_EWORKSPACE, "null workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % mg::kAlign != 0) return fail(MG_EWORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes / lp.total < static_cast<size_t>(lanes))
    return fail(MG_EWORKSPACE, "workspace %zu bytes < %d x %zu needed", ws_bytes, lanes, lp.total);
  int device = 0;
  MG_HIP(hipGetDevice(&device));
  if (ctx->stream) {   // the lanes' streams must live on the device of the context's stream
    hipDevice_t sdev = 0;
    MG_HIP(hipStreamGetDevice(ctx->stream, &sdev));
    if (static_cast<int>(sdev) != device)
      return fail(MG_EINVAL, "the context's stream is on device %d, the current device is %d", static_cast<int>(sdev),
                  device);
  }
  if (!ctx->order_event && hipEventCreateWithFlags(&ctx->order_event, hipEventDisableTiming) != hipSuccess) {
    ctx->order_event = nullptr;
    return fail(MG_EHIP, "hipEventCreateWithFlags of the order event failed");
  }
  std::vector<mg_ctx*> made;
  for (int w = 0; w < lanes; ++w) {
    mg_ctx* lane = nullptr;
    const int rc = make_lane(ctx, static_cast<unsigned char*>(workspace) + static_cast<size_t>(w) * lp.total, lp,
                             device, &lane);
    made.push_back(lane);
    if (rc != MG_OK) {
      for (mg_ctx* m : made) mg_destroy(m);
      return rc;
    }
  }
  ctx->lanes = made;
  return MG_OK;
}

int mg_level_info(mg_ctx* ctx, int level, int* n, double* h) {
  MG_TRY(check_level(ctx, level, 0));
  if (n) *n = ctx->lv[level].n;
  if (h) *h = ctx->lv[level].h;
  return ctx->L;
}

int mg_level_coeffs(mg_ctx* ctx, int level, double* bx, double* by, double* bz, uint8_t* mask) {
  MG_TRY(check_level(ctx, level, 0));
  const Level& a = ctx->lv[level];
  const size_t nb = sizeof(double) * cells(a);
  if (bx) MG_HIP(hipMemcpyAsync(bx, a.bx, nb, hipMemcpyDeviceToDevice, ctx->stream));
  if (by) MG_HIP(hipMemcpyAsync(by, a.by, nb, hipMemcpyDeviceToDevice, ctx->stream));
  if (bz) MG_HIP(hipMemcpyAsync(bz, a.bz, nb, hipMemcpyDeviceToDevice, ctx->stream));
  if (mask) MG_HIP(hipMemcpyAsync(mask, a.mask, cells(a), hipMemcpyDeviceToDevice, ctx->stream));
  return MG_OK;
}

int mg_smooth(mg_ctx* ctx, int prec, int level, void* p, const void* f, int sweeps, int order) {
  MG_TRY(check_level(ctx, level, 0));
  MG_TRY(check_prec(ctx, prec));
  if (!p || !f || sweeps < 0 || (order != MG_PRE && order != MG_POST)) return fail(MG_EINVAL, "bad arguments");
  if (prec == MG_PREC_F64)
    return smooth<double>(ctx, level, static_cast<double*>(p), static_cast<const double*>(f), nullptr, sweeps, order);
  return smooth<float>(ctx, level, static_cast<float*>(p), static_cast<const float*>(f), nullptr, sweeps, order);
}

int mg_residual_restrict(mg_ctx* ctx, int prec, int level, const void* p, const void* f, void* fc) {
  MG_TRY(check_level(ctx, level, 1));
  MG_TRY(check_prec(ctx, prec));
  if (!p || !f || !fc) return fail(MG_EINVAL, "null array pointer");
  if (prec == MG_PREC_F64) {
    const View<double> nx = ctx->v64(level + 1);
    return residual_restrict<double>(ctx, level, static_cast<const double*>(p), static_cast<const double*>(f),
                                     nullptr, static_cast<double*>(fc), nx.t);
  }
  const View<float> nx = ctx->v32(level + 1);
  return residual_restrict<float>(ctx, level, static_cast<const float*>(p), static_cast<const float*>(f), nullptr,
                                  static_cast<float*>(fc), nx.t);
}

int mg_prolong_add(mg_ctx* ctx, int prec, int level, const void* ec, void* p) {
  MG_TRY(check_level(ctx, level, 1));
  MG_TRY(check_prec(ctx, prec));
  if (!ec || !p) return fail(MG_EINVAL, "null array pointer");
  const Level& a = ctx->lv[level];
  if (prec == MG_PREC_F64)
    MG_HIP(mg::launch_prolong_add<double>(static_cast<const double*>(ec), static_cast<double*>(p), a.mask, a.q,
                                          ctx->stream));
  else
    MG_HIP(mg::launch_prolong_add<float>(static_cast<const float*>(ec), static_cast<float*>(p), a.mask, a.q,
                                         ctx->stream));
  return MG_OK;
}

int mg_coarse_solve(mg_ctx* ctx, int prec, const void* f, void* e) {
  if (!ctx) return fail(MG_EINVAL, "null context");
  MG_TRY(check_prec(ctx, prec));
  if (!f || !e) return fail(MG_EINVAL, "null array pointer");
  const Level& a = ctx->lv[ctx->L - 1];
  if (prec == MG_PREC_F64)
    MG_HIP(mg::launch_coarse_solve<double>(static_cast<const double*>(f), static_cast<double*>(e), ctx->pinv, a.mask,
                                           ctx->stream));
  else
    MG_HIP(mg::launch_coarse_solve<float>(static_cast<const float*>(f), static_cast<float*>(e), ctx->pinv, a.mask,
                                          ctx->stream));
  return MG_OK;
}

int mg_vcycle(mg_ctx* ctx, int prec, void* p, const void* f) {
  if (!ctx) return fail(MG_EINVAL, "null context");
  MG_TRY(check_prec(ctx, prec));
  if (!p || !f) return fail(MG_EINVAL, "null array pointer");
  if (prec == MG_PREC_F64) return vcycle<double>(ctx, 0, static_cast<double*>(p), static_cast<const double*>(f), nullptr);
  return vcycle<float>(ctx, 0, static_cast<float*>(p), static_cast<const float*>(f), nullptr);
}

}  // extern "C"
