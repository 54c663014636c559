// Launchers of the device kernels (internal host API of the library).
//
// Arrays follow the layout of include/mg.h: [k][j][i] with x fastest, low-face
// storage of the face coefficients.  `q` is log2 of the cells per side of the grid
// a kernel works on.  Every launcher queues work on `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mg {

// beta = 2 / (rho_L + rho_R): the face product of two cell densities (the harmonic mean
// of 1/rho over the face, section 3.1).  The quotient is the hardware reciprocal of the
// sum refined by two Newton steps r <- r + r (1 - s r), each of which squares the
// relative error, then doubled (exact): within about an ulp of the rounded quotient
// for sums in [1e-300, 1e300].  A density of +inf (an inactive cell, or the far side
// of a wall) gives 0: the reciprocal of +inf is +0, and the Newton steps multiply it by
// the sum clamped to the largest finite value (a finite sum is used as it is), which
// keeps it +0 where the unclamped sum would make inf * 0.  Every place that forms beta
// from densities calls this, so the stored coefficients and those formed on the fly
// agree bit for bit.
__device__ __forceinline__ double face_beta(double a, double b) {
  const double s = a + b;
  const double sc = __builtin_fmin(s, __DBL_MAX__);
  double r = __builtin_amdgcn_rcp(s);
  double e = __builtin_fma(-sc, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-sc, r, 1.0);
  r = __builtin_fma(r, e, r);
  return 2.0 * r;
}

// The FP32 face product of the mixed-precision cycles' density form: the FP32
// reciprocal and one Newton step (within about an ulp of the rounded FP32 quotient),
// +inf densities handled as in FP64.
__device__ __forceinline__ float face_beta(float a, float b) {
  const float s = a + b;
  const float sc = __builtin_fminf(s, __FLT_MAX__);
  float r = __builtin_amdgcn_rcpf(s);
  const float e = __builtin_fmaf(-sc, r, 1.0f);
  r = __builtin_fmaf(r, e, r);
  return 2.0f * r;
}

// The quotient of a Gauss-Seidel update, numerator over the diagonal D > 0 (a sum of at
// most six face products, far from the ends of the range): the reciprocal of D, the
// product, and one correction from the exact remainder n - D q (Markstein's scheme).
// With the reciprocal itself refined by a Newton step (FP64; FP32 takes the hardware
// reciprocal as it is, since its result only corrects an FP64 iterate), the quotient is
// within an ulp of the rounded one and in practice is the rounded one, in fewer
// instructions than the IEEE division and with a shorter dependency chain.  Every sweep
// calls it, so the one-pass, two-sweep, block and half-sweep paths give the same bits.
__device__ __forceinline__ double gs_quotient(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
  const double q = n * r;
  return __builtin_fma(__builtin_fma(-d, q, n), r, q);
}
__device__ __forceinline__ float gs_quotient(float n, float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  const float q = n * r;
  return __builtin_fmaf(__builtin_fmaf(-d, q, n), r, q);
}

// ---- setup --------------------------------------------------------------------
// beta_f = o_f 2/(rho_L + rho_R); with rho == nullptr the open-face areas o_f (0 or 1)
hipError_t launch_coeffs_from_rho(const double* rho, const uint8_t* mask, int q,
                                  double* bx, double* by, double* bz, hipStream_t s);
// rt = rho on active cells (mask after setup), +inf elsewhere: the density form of the
// finest coefficients, beta_f = 2/(rt_L + rt_R), which the finest-grid passes may read
// instead of the three face arrays (bit-identical coefficients)
hipError_t launch_rho_tilde(const double* rho, const uint8_t* mask, int q, double* rt, hipStream_t s);
// coarse rho = mean of rho over the active children (1 if none)
hipError_t launch_restrict_rho(const double* rho, const uint8_t* mask, int qc, double* crho, hipStream_t s);
// beta = area * 2/(rho_L + rho_R) in place on the open faces
hipError_t launch_area_to_beta(const double* rho, int q, double* bx, double* by, double* bz, hipStream_t s);
// counters[0] += non-finite or negative beta values, [1] += active cells, [2] += dropped;
// bx == nullptr: validate and mark only (the coefficients are already closed in place)
hipError_t launch_setup_fine(const double* ubx, const double* uby, const double* ubz,
                             const uint8_t* umask, int q, double* bx, double* by, double* bz,
                             uint8_t* mask, long long* counters, hipStream_t s);
// the three above for a hierarchy built from rho, in one pass: face products, their
// validation and the active cells (counters as launch_setup_fine), and rt
hipError_t launch_setup_from_rho(const double* rho, const uint8_t* umask, int q, double* bx, double* by, double* bz,
                                 uint8_t* mask, double* rt, long long* counters, hipStream_t s);
hipError_t launch_coarsen(const double* bx, const double* by, const double* bz, const uint8_t* mask,
                          int qc, double* cbx, double* cby, double* cbz, uint8_t* cmask, hipStream_t s);
hipError_t launch_to_f32(const double* src, float* dst, long long count, hipStream_t s);

// ---- cut cells (setup) ---------------------------------------------------------
// Cells with 0 < fluid fraction < kMergeFraction merge with a neighbour.
constexpr double kMergeFraction = 0.25;
// psi at corners [(N+1)][N][N] -> open-area fractions (low faces), fluid fractions and
// the merge map (flat target index or -1); samples per direction is a power of two
hipError_t launch_cut_cells(const double* psi, int q, int samples, double* ax, double* ay, double* az, double* vol,
                            int32_t* merge_to, hipStream_t s);
// face coefficients of the merged cut-cell operator and its activity mask
hipError_t launch_cut_coeffs(const double* rho, const double* ax, const double* ay, const double* az,
                             const double* vol, const int32_t* merge_to, int q, double* bx, double* by, double* bz,
                             uint8_t* mask, hipStream_t s);
// g = f with the donors' sources moved onto their targets; p on donors = p on targets
hipError_t launch_merge_rhs(const int32_t* merge_to, const double* f, double* g, int q, hipStream_t s);
hipError_t launch_merge_fill(const int32_t* merge_to, double* p, int q, hipStream_t s);

// ---- V-cycle steps (T = double or float) ----------------------------------------
// fshift: device scalar subtracted from f on active cells (nullptr = none)
template <typename T>
hipError_t launch_rbgs_half(T* p, const T* f, const T* bx, const T* by, const T* bz, int q,
                            double h, int colour, const double* fshift, hipStream_t s);
// One full red-black sweep in one pass, out of place (pin -> pout, distinct buffers);
// order 0 = red then black, 1 = black then red.  Grids with at least 64 cells per side.
// rt != nullptr: coefficients from the density form instead of bx, by, bz.  zero_in:
// the input is known to be zero (a correction's first sweep), so pin is not read.
int fused_sweep_supported(int q);
// One red-black sweep of a 32^3 or 64^3 grid (face arrays) in one launch, a block of
// cells per workgroup: pin -> pout (distinct), order and zero_in as launch_rbgs_fused,
// whose bits it gives.
int box_sweep_supported(int q);
template <typename T>
hipError_t launch_rbgs_box(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q, double h,
                           int order, const double* fshift, int zero_in, hipStream_t s);
// The same sweep, then the residual of its output restricted as launch_residual_restrict
// does (fc, ec = 0 on the grid below), bit for bit.
template <typename T>
hipError_t launch_rbgs_box_restrict(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q,
                                    double h, int order, const double* fshift, T* fc, T* ec, hipStream_t s);
// The same sweep of pin + mask * prolong(ec), bit for bit launch_prolong_add(ec, pin)
// followed by launch_rbgs_box; pin itself is not changed.
template <typename T>
hipError_t launch_rbgs_box_prolong(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q,
                                   double h, int order, const double* fshift, const T* ec, const uint8_t* mask,
                                   hipStream_t s);
// What the FP64 two-sweep pass of flexible CG does besides its sweeps (w null: nothing).
struct Fused2Extra {
  const double* w = nullptr;        // w = A d of the current direction
  double* partials = nullptr;       // one partial sum per workgroup (see below)
  double* rnew = nullptr;           // residual update: r - alpha w, written here
  const double* s_dr = nullptr;     // residual update: alpha = *s_dr / *s_dw,
  const double* s_dw = nullptr;
  double* s_alpha = nullptr;        // also stored here
};
// Two red-black sweeps in one pass (density form, grids of 256^3 and up): pin -> pout
// (distinct), order as launch_rbgs_fused; bit for bit two one-pass sweeps.  With x->w
// (FP64): one partial sum per workgroup into x->partials, their number into *nblocks
// (at most kNumPartials); without zero_in the sum is pout . w; with zero_in (the first
// pre-smoothing of a preconditioner, f = r, no fshift) the pass sweeps with and writes
// r - alpha w to x->rnew (not f), and the sum is its squared norm.
int fused2_supported(int q);
template <typename T>
hipError_t launch_rbgs_fused2(const T* pin, T* pout, const T* f, const T* rt, int q, double h, int order,
                              const double* fshift, int zero_in, hipStream_t s, const Fused2Extra* x = nullptr,
                              int* nblocks = nullptr);
template <typename T>
hipError_t launch_rbgs_fused(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, const T* rt,
                             int q, double h, int order, const double* fshift, int zero_in, hipStream_t s);
template <typename T>
hipError_t launch_residual_restrict(const T* p, const T* f, const T* bx, const T* by, const T* bz, const T* rt,
                                    int q, double h, const double* fshift, T* fc, T* ec_zero,
                                    hipStream_t s);
template <typename T>
hipError_t launch_prolong_add(const T* ec, T* p, const uint8_t* mask, int q, hipStream_t s);
template <typename T>
hipError_t launch_coarse_solve(const T* f, T* e, const double* pinv, const uint8_t* mask, hipStream_t s);

// Levels of the single-workgroup sub-cycle: entry 0 is the first grid it handles
// (at most 16^3), the last entry the 4^3 grid.  e[0] must be zero on entry (or hold
// the guess), f[0] the right-hand side; fshift applies to level 0 only.
constexpr int kCoarseCycleMaxN = 16;
template <typename T>
struct CoarseCycle {
  int nlev;
  int q[4];
  const T* bx[4];
  const T* by[4];
  const T* bz[4];
  const uint8_t* mask[4];
  T* f[4];
  T* e[4];
  T h2[4];
  T inv_h2[4];
  const double* pinv;
  const double* fshift;
};
template <typename T>
hipError_t launch_coarse_cycle(const CoarseCycle<T>& a, hipStream_t s);

// ---- z-marching FP64 residual passes (grids of 32^3 and up) ------------------------
// Same results as the grid-stride kernels below (per cell), each plane of p and of the
// coefficients read once per column; rt != nullptr selects the density form.
int march_supported(int q);
hipError_t launch_residual_norm_march(const double* p, const double* f, const double* bx, const double* by,
                                      const double* bz, const double* rt, int q, double h, const double* fshift,
                                      float* r32, float* e32, double* r64, double* z64, double* partials,
                                      int* nblocks, hipStream_t s);
// (FP64 and FP32: the restriction is the one pass an FP32 cycle marches)
template <typename T>
hipError_t launch_residual_restrict_march(const T* p, const T* f, const T* bx, const T* by, const T* bz, const T* rt,
                                          int q, double h, const double* fshift, T* fc, T* ec, hipStream_t s);
// p + e (e in FP32, added on active cells) written to pout, and the norm pass of that
// sum: partials, r32, e32 as launch_residual_norm_march.  The density form only (rt is
// required); pout must not overlap p, and e32 (cleared) must be null or not overlap e.  The update and residual of one mixed-precision
// refinement step in one pass.
hipError_t launch_residual_norm_update_march(const double* p, const float* e, double* pout, const double* f,
                                             const double* rt, int q, double h, const double* fshift, float* r32,
                                             float* e32, double* partials, int* nblocks, hipStream_t s);
hipError_t launch_fcg_aw_march(const double* d, const double* r, const double* bx, const double* by, const double* bz,
                               const double* rt, int q, double h, double* w, double* part_dw, double* part_dr,
                               int* nblocks, hipStream_t s);
// The flexible-CG direction and product in one pass (grids of 32^3 and up): dn = z +
// beta d (beta = -*s_zw / *s_dw; with s_zw = s_dw = null the first direction dn = z,
// and d is not used), w = A dn, partial sums of dn.w and dn.r, and p += *s_alpha d
// (the previous step's update, skipped on the first step).  z is z64 or z32 (exactly
// one non-null); dn must not be d.
// With df (density-form grids of 128^3 and up, not the first step), p's update every
// second step: df->skip leaves this step's update to the next one (p is not touched,
// *s_alpha is saved to df->s_alpha_save); otherwise p += *df->s_alpha_prev df->d_prev
// (the update left by the step before, d_prev distinct from d and dn) and then
// p += *s_alpha d, the same operations in the same order as two steps apart.
struct FcgxDefer {
  bool skip = false;
  double* s_alpha_save = nullptr;
  const double* d_prev = nullptr;
  const double* s_alpha_prev = nullptr;
};
int fcgx_defer_supported(const double* rt, int q);
hipError_t launch_fcg_x_march(const double* z64, const float* z32, const double* d, double* dn, double* p,
                              const double* s_zw, const double* s_dw, const double* s_alpha, const double* r,
                              const double* bx, const double* by, const double* bz, const double* rt, int q, double h,
                              double* w, double* part_dw, double* part_dr, int* nblocks, hipStream_t s,
                              const FcgxDefer* df = nullptr);

// ---- FP64 finest-grid passes ------------------------------------------------------
// partials[blockIdx] = sum over active cells of r^2, r = (f - fshift) - A p; optional
// r32 = float(r) and e32 = 0 (mixed-precision refinement); returns the block count used.
// optional outputs (each may be null): r32 = float(r), e32 = 0, r64 = r, z64 = 0
hipError_t launch_residual_norm(const double* p, const double* f, const double* bx, const double* by,
                                const double* bz, const double* rt, int q, double h, const double* fshift,
                                float* r32, float* e32_zero, double* r64, double* z64, double* partials,
                                int* nblocks, hipStream_t s);
// flexible CG: w = A d with partial d.w and d.r; the residual update r -= alpha w
// (alpha = dr/dw read on the device and stored to *s_alpha) with partial ||r||^2; the
// update p += *s_alpha d; partial z.w; dn = z + beta d (with p += *s_alpha d when p is
// given; beta and the update skipped when s_zw is null, dn = z; dn may be d)
hipError_t launch_fcg_aw(const double* d, const double* r, const double* bx, const double* by, const double* bz,
                         const double* rt, int q, double h, double* w, double* part_dw, double* part_dr, int* nblocks,
                         hipStream_t s);
hipError_t launch_fcg_rupdate(double* r, const double* w, const double* s_dr, const double* s_dw, double* s_alpha,
                              int q, double* z_zero, float* r32, float* e32_zero, double* part_rr, int* nblocks,
                              hipStream_t s);
hipError_t launch_fcg_padd(double* p, const double* d, const double* s_alpha, int q, hipStream_t s);
// p += *s_alpha0 d0, then p += *s_alpha d (two updates left pending, in their order)
hipError_t launch_fcg_padd2(double* p, const double* d0, const double* s_alpha0, const double* d, const double* s_alpha,
                            int q, hipStream_t s);
hipError_t launch_fcg_zw(const double* z64, const float* z32, const double* w, int q, double* part, int* nblocks,
                         hipStream_t s);
hipError_t launch_fcg_dir(const double* z64, const float* z32, const double* d, double* dn, double* p,
                          const double* s_zw, const double* s_dw, const double* s_alpha, int q, hipStream_t s);
// mode 0: partials = sum_active x ; mode 1: sum_active (x - *shift)^2
hipError_t launch_masked_sum(const double* x, const uint8_t* mask, int q, int mode, const double* shift,
                             double* partials, int* nblocks, hipStream_t s);
// out[0] = scale * sum(partials[0..nparts))  (single block, fixed order)
hipError_t launch_reduce_final(const double* partials, int nparts, double scale, double* out, hipStream_t s);
// p = mask ? p - *mean : 0   (mean may be nullptr: p = mask ? p : 0)
hipError_t launch_gauge(double* p, const uint8_t* mask, int q, const double* mean, hipStream_t s);
// p += mask ? double(e32) : 0
hipError_t launch_update_p(double* p, const float* e32, const uint8_t* mask, int q, hipStream_t s);
hipError_t launch_apply(const double* p, const double* bx, const double* by, const double* bz, int q,
                        double h, double* Ap, hipStream_t s);
hipError_t launch_coeff_grad(const double* mu, const double* p, int batch, const double* bx,
                             const double* by, const double* bz, const uint8_t* mask, int q, double h,
                             double* gbx, double* gby, double* gbz, double* grho, hipStream_t s);

// Runge-Kutta stage around the solve: f = div(U + dt R)/dt, and the projection
// U <- o_f (U + dt R - dt beta grad p) on the faces (R may be null)
hipError_t launch_divergence(const double* ux, const double* uy, const double* uz, const double* rx, const double* ry,
                             const double* rz, double dt, const uint8_t* mask, int q, double h, double* f,
                             hipStream_t s);
hipError_t launch_project(double* ux, double* uy, double* uz, const double* rx, const double* ry, const double* rz,
                          double dt, const double* p, const double* bx, const double* by, const double* bz,
                          const uint8_t* mask, int q, double h, hipStream_t s);

}  // namespace mg
