/*
 * mg.h - C ABI of the MI355X multigrid pressure-projection solver.
 *
 * The library solves the pressure Poisson equation of the free-surface flow solver
 * (paper section 2, eq. (pois); finite-volume form eq. (integral2)):
 *
 *     div( (1/rho) grad p ) = f
 *
 * on a uniform cell-centred N x N x N grid with spacing h, periodic in x and y and
 * with walls (zero normal flux) at both z ends, with an immersed body whose faces
 * carry no flux.  Discrete operator, for every fluid cell c:
 *
 *     (A p)_c = h^-2 * sum over the six faces f of c of beta_f (p_neighbour - p_c)
 *
 * where beta_f is the face product "1/rho times open area" that section 3.1 forms on
 * the finest grid and moves to the coarse grids as one unit.  The method is geometric
 * multigrid (section 3.1): V(2,2) cycles of red-black Gauss-Seidel, 8-child mean
 * restriction, trilinear prolongation, face-product coarsening (mean of the 4
 * coincident fine faces) down to 4^3, and an FP64 pseudo-inverse solve there.
 *
 * Layout.  Every array pointer is a DEVICE pointer to a C-contiguous [N][N][N] array
 * indexed [k][j][i] (x fastest), unless marked HOST.  Face arrays use low-face
 * storage: bx[k][j][i] couples cells (i-1 mod N, j, k) and (i, j, k); by likewise
 * in j; bz[k][j][i] couples (i, j, k-1) and (i, j, k), so bz[0][..] is the bottom wall
 * (forced to 0) and the top wall is implicit.  mask: 1 = fluid, 0 = body.
 * Batched arrays are [batch][N][N][N].
 *
 * Ownership.  The caller owns every array and the workspace (device memory of
 * mg_workspace_size() bytes, 256-byte aligned).  The library never allocates device
 * memory.  mg_setup copies the finest coefficients into the workspace, so the caller
 * may free or reuse its beta arrays afterwards; the workspace must outlive the
 * context.  A context is not thread-safe; distinct contexts are independent.
 *
 * Streams.  All device work is ordered on the HIP stream given to mg_setup (or set
 * later with mg_set_stream); NULL means the default stream.  Entry points that
 * report numbers to the host (mg_setup, mg_solve) synchronise that stream.  A context
 * with lanes (mg_add_lanes) also runs batch items on its lanes' own streams, joined to
 * that stream at the start and end of each mg_solve.
 *
 * Errors.  Every int-returning function returns MG_OK or a negative code and never
 * throws across the ABI; mg_last_error() returns a thread-local message.  Invalid
 * arguments are detected on the host before any device work is queued.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx mg_ctx;

enum {
  MG_OK = 0,
  MG_EINVAL = -1,      /* bad dims, pointer, tolerance, flags, or beta < 0 / non-finite */
  MG_EWORKSPACE = -2,  /* workspace NULL, misaligned or smaller than mg_workspace_size */
  MG_EHIP = -3,        /* a HIP runtime call failed (message names it) */
  MG_ENOCONV = -4,     /* max_cycles reached before tol; p holds the last iterate */
  MG_EBREAKDOWN = -5   /* residual non-finite or grew 1e3-fold; p holds the last iterate */
};

/* mg_setup flags (MG_MIXED and MG_KRYLOV may be combined) */
enum {
  MG_FP64 = 0,   /* FP64 V-cycles */
  MG_MIXED = 1,  /* FP32 V-cycles inside FP64 iterative refinement (FP64 residual,
                    update and coarsest solve); the workspace also holds FP32 copies */
  MG_KRYLOV = 2, /* outer iteration = flexible conjugate gradients preconditioned by one
                    V(2,2) cycle per step (FP32 cycle with MG_MIXED); all vector updates
                    and dot products FP64.  Removes the few error modes a V-cycle misses
                    at steep, non-grid-aligned density interfaces.  Five more FP64
                    finest-grid vectors in the workspace (up to seven with MG_FROM_RHO,
                    see there). */
  MG_COARSEN_DENSITY = 4, /* mg_setup_from_rho only: the coarsening section 3.1 rejects -
                    density restricted cell centre to cell centre (mean over active
                    children), open areas restricted separately (mean of 4 faces), and
                    beta = area * 2/(rho_L + rho_R) re-formed on every grid.  The finest
                    operator is unchanged; for comparison with the default. */
  MG_FROM_RHO = 8 /* mg_workspace_size and mg_setup_from_rho only (pass the same flags to
                    both): the workspace is for a setup from the density, so an MG_MIXED
                    context on a grid of 64^3 and up leaves out the FP32 face arrays of its
                    finest grid, which its FP32 cycles form from the density instead (12
                    bytes per cell less); an MG_KRYLOV context on a grid of 128^3 and up
                    gets a third direction vector, with which it updates the solution every
                    second step, and in FP64 on a grid of 256^3 and up a second residual,
                    with which its preconditioner's first pass also updates the residual
                    in place of a pass of its own (8 bytes per cell more each).  Without it
                    the size covers both setups (and those updates keep their passes). */
};

/* precision selector of the component entry points */
enum { MG_PREC_F64 = 0, MG_PREC_F32 = 1 };

/* smoothing order of mg_smooth */
enum { MG_PRE = 0 /* red then black */, MG_POST = 1 /* black then red */ };

typedef struct {
  int cycles;           /* V-cycles (one per refinement / CG step), summed over the batch */
  int levels;           /* grids in the hierarchy, finest N down to 4 */
  long long active_cells;  /* fluid cells with at least one open face on the finest grid */
  long long dropped_cells; /* fluid cells with no open face: no equation, treated as body */
  double removed_mean;  /* fluid mean removed from f (last batch item) */
  double final_relres;  /* ||P f - A p|| / ||P f|| at exit (largest over the batch) */
  double seconds;       /* host wall time of the call */
  size_t ws_bytes;      /* workspace bytes in use */
} mg_stats;

/*
 * Workspace bytes for an N^3 grid (dims[0] = dims[1] = dims[2] = N, N a power of two,
 * 8 <= N <= 1024) with the given flags, or 0 if the arguments are invalid.
 * Pure host arithmetic: callable without a GPU.
 */
size_t mg_workspace_size(const int dims[3], int flags);

/*
 * Face coefficients from cell density (eq. (density) gives rho from the VOF fraction;
 * section 3.1 forms 1/rho times the open area on the faces of the finest grid):
 *     beta_f = o_f * 2 / (rho_L + rho_R),   o_f = mask_L * mask_R,   z walls 0.
 * rho > 0 in fluid cells (body values unused).  Writes bx, by, bz (caller-owned).  The
 * quotient is the reciprocal of the sum refined by Newton steps, within an ulp of the
 * correctly rounded one (the same function forms every density-derived coefficient).
 */
int mg_coeffs_from_rho(const double* rho, const uint8_t* mask, const int dims[3],
                       double* bx, double* by, double* bz, void* hip_stream);

/*
 * Build the multigrid hierarchy (section 3.1): copy the finest face products into
 * the workspace, zero faces touching the body and the bottom wall, mark fluid cells
 * with no open face inactive, coarsen the face products level by level (coarse face
 * = mean of its 4 fine faces, coarse cell active if any child is and it keeps an open
 * face), and form the FP64 pseudo-inverse of the 4^3 operator on the host.
 * beta must be >= 0 and finite; h > 0.  On success *out is a new context.
 */
int mg_setup(mg_ctx** out, void* workspace, size_t ws_bytes,
             const double* bx, const double* by, const double* bz,
             const uint8_t* mask, const int dims[3], double h, int flags, void* hip_stream);

/*
 * As mg_setup, but from the cell density: the finest face products
 * beta_f = o_f 2/(rho_L + rho_R) are formed in the workspace (no caller beta arrays),
 * then coarsened as one unit (section 3.1), or with MG_COARSEN_DENSITY as density and
 * area separately.  rho must be positive and finite in fluid cells (MG_EINVAL).  The
 * context also keeps the density (+inf on inactive cells), and the finest-grid passes
 * of mg_solve re-form beta from it instead of reading the three face arrays: the same
 * operator bit for bit, with a third less memory traffic.  In MG_MIXED contexts the
 * FP32 cycles on grids of 64^3 and up form their finest beta from an FP32 copy of the
 * density (within a few FP32 ulps of the rounded FP64 beta; the FP64 refinement is
 * unaffected).
 */
int mg_setup_from_rho(mg_ctx** out, void* workspace, size_t ws_bytes, const double* rho,
                      const uint8_t* mask, const int dims[3], double h, int flags, void* hip_stream);

/* Change the stream used by later calls on this context. */
int mg_set_stream(mg_ctx* ctx, void* hip_stream);

/*
 * Solve A p_b = P f_b for b = 0..batch-1 (P removes the fluid mean of f; section 3.1
 * method, V(2,2) cycles until ||P f - A p||_2 / ||P f||_2 <= tol, checked after every
 * cycle, refinement step or CG step).  p is in/out: initial guess in, solution out, with zero
 * fluid mean and 0 in the body.  hist (HOST, may be NULL) receives batch rows of
 * max_cycles+1 relative residuals, hist[b*(max_cycles+1)+0] for the initial guess;
 * n_hist (HOST, may be NULL) receives the entries written per item.  stats may be NULL.
 * A right-hand side whose projection is zero to rounding (||P f|| <= 64 eps ||f|| over
 * the fluid cells, eps = 2^-52, e.g. f = 0 or a constant f) has the solution p = 0:
 * p is set to 0 and hist holds the single entry 0, with no cycle.
 * Returns MG_ENOCONV / MG_EBREAKDOWN with p and hist valid when a solve stops early.
 */
int mg_solve(mg_ctx* ctx, const double* f, double* p, int batch, double tol, int max_cycles,
             double* hist, int* n_hist, mg_stats* stats);

/*
 * Concurrent right-hand sides of one hierarchy, e.g. the batch of adjoint solves of a
 * differentiated projection (A mu_b = P w_b, every b on the same operator).  Small
 * grids leave most of the GPU idle in each launch, so solving several right-hand
 * sides at once on separate streams raises throughput; the results are bit for bit
 * those of solving them one after another.
 *
 * mg_lane_workspace_size: bytes of one lane's scratch (the arrays a solve writes:
 * right-hand sides, corrections and second buffers of every grid, the flexible-CG
 * vectors, reduction partials and scalars) for these dims and flags; 0 if unsupported.
 *
 * mg_add_lanes: gives ctx `lanes` extra lanes (1 <= lanes <= MG_MAX_LANES, once per
 * context).  workspace: DEVICE memory of at least lanes x mg_lane_workspace_size bytes,
 * 256-byte aligned, owned by the caller and outliving ctx; lane w uses the w-th slice.
 * Each lane gets a non-blocking HIP stream of default priority (created on the current
 * device, destroyed by mg_destroy), a pinned read-back buffer and two events; no device
 * memory is allocated.  From then on mg_solve with batch > 1 solves up to 1 + lanes
 * items at a time: item b on lane b mod (1 + lanes), lane 0 being ctx on its own stream,
 * each extra lane driven by a host thread of its own.  The lane streams start after the
 * work already queued on ctx's stream, and ctx's stream waits for all of them before
 * anything queued after mg_solve.  Errors: MG_EINVAL (null ctx, lanes out of range, lanes
 * already added, or a current device other than that of ctx's stream), MG_EWORKSPACE
 * (workspace null, misaligned or too small), MG_EHIP.  On error no lane is added.
 */
#define MG_MAX_LANES 16
size_t mg_lane_workspace_size(const int dims[3], int flags);
int mg_add_lanes(mg_ctx* ctx, void* workspace, size_t ws_bytes, int lanes);

/*
 * mg_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same solve, bit
 * for bit, with every array it writes besides p (the right-hand sides, corrections and
 * second buffers of the grids, the flexible-CG vectors, reduction partials and device
 * scalars) in a static device array of the library, 32 MiB per GPU, instead of the
 * context's workspace.  The caller passes f, p, hist, n_hist and stats as for mg_solve;
 * the batch is solved item after item on the context's stream (its lanes are not used).
 * The call makes no allocation on the device (no hipMalloc, hipFree or allocating
 * library routine).  Limit: the scratch of one solve must fit the 32 MiB, which holds
 * grids up to 128^3 in FP64 and up to 64^3 with MG_MIXED or MG_KRYLOV; a larger context
 * gets MG_EINVAL with the sizes in the message.  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (a solve initialises whatever it reads):
 * calls that overlap on one GPU - from two host threads, or on two streams without
 * ordering between them - race and give wrong results.  Errors as mg_solve, plus
 * MG_EINVAL if the current device is not that of the context's stream.
 */
int mg_solve_static(mg_ctx* ctx, const double* f, double* p, int batch, double tol, int max_cycles,
                    double* hist, int* n_hist, mg_stats* stats);

/*
 * Ap_b = A p_b on the finest grid: the discrete operator of eq. (pois) in the
 * finite-volume form of eq. (integral2), (A p)_c = h^-2 sum over the faces of c of
 * beta_f (p_neighbour - p_c), with the context's face products (section 3.1); 0 on
 * inactive cells.  p and Ap are DEVICE [batch][N][N][N] arrays owned by the caller;
 * Ap is overwritten.  Stream-ordered, no synchronisation.  MG_EINVAL for a null
 * context or pointer or batch < 1.
 */
int mg_apply(mg_ctx* ctx, const double* p, double* Ap, int batch);

/*
 * Gradient of L through the solve (adjoint method; the paper does not differentiate):
 * with p_b the solutions and mu_b the adjoint solutions (A mu_b = P dL/dp_b),
 *     g_f = o_f h^-2 sum_b (mu_b,R - mu_b,L)(p_b,R - p_b,L)          (= dL/dbeta_f)
 *     grho_c = -1/2 sum over the faces f of c of beta_f^2 g_f          (= dL/drho_c)
 * the second valid when beta came from mg_coeffs_from_rho.  Any of gbx, gby, gbz,
 * grho may be NULL to skip it.  Outputs are overwritten, not accumulated.
 */
int mg_coeff_grad(mg_ctx* ctx, const double* mu, const double* p, int batch,
                  double* gbx, double* gby, double* gbz, double* grho);

/*
 * The Runge-Kutta stage around the solve (section 2.1, eqs. (poisson1) / (poisson2) and
 * (runge1) / (runge2), in the finite-volume form of eq. (integral2)).  Velocities are
 * the normal components on the faces, in the low-face storage of the coefficients
 * (ux[k][j][i] on the face between (i-1, j, k) and (i, j, k), ...).  A face is open when
 * both cells are active and it is not a z wall; R (the non-pressure terms) may be NULL.
 *   mg_divergence:  f_c = (1/h) sum_faces (+-)(U_f + dt R_f) / dt on active cells, else 0
 *   mg_project:     U_f <- U_f + dt R_f - dt beta_f (p_hi - p_lo) / h on open faces, 0 on
 *                   closed ones (a body at rest), in place
 * With A p = f solved, the projected field has zero discrete divergence.  dt > 0.
 */
int mg_divergence(mg_ctx* ctx, const double* ux, const double* uy, const double* uz,
                  const double* rx, const double* ry, const double* rz, double dt, double* f);
int mg_project(mg_ctx* ctx, double* ux, double* uy, double* uz,
               const double* rx, const double* ry, const double* rz, double dt, const double* p);

/*
 * Cut cells (section 2.2: the body as a signed distance psi, positive in the fluid;
 * finite volumes with the open fraction of each face, eq. (integral2); cells under a
 * quarter full merged with a neighbour along the steepest gradient of psi).  These
 * build the coefficients and the mask that mg_setup takes; the paper leaves the
 * formulas to a reference, so the library fixes this reading:
 *
 *   mg_cut_cells:  psi (DEVICE, [N+1][N][N]) holds psi at the cell corners (i h, j h, k h),
 *     k = 0..N, x and y periodic.  ax, ay, az ([N][N][N], low-face storage) receive the
 *     open-area fraction of each face: the fraction of samples x samples midpoint
 *     samples of the bilinear interpolant of the face's corners where psi > 0 (az on
 *     the bottom wall is 0).  vol receives the fluid fraction of each cell from
 *     samples^3 samples of the trilinear interpolant.  merge_to receives, for each cell
 *     with 0 < vol < 1/4, the flat index (k N + j) N + i of the face neighbour it merges
 *     into: along the largest component of the gradient of the trilinear psi at the cell
 *     centre (ties x, y, z), on the side where psi grows, provided that cell lies inside
 *     the z walls and has vol >= 1/4; -1 everywhere else.  samples is 2, 4, 8 or 16.
 *     Sample values are summed in a fixed order without fused multiply-adds, so every
 *     inside/outside decision is reproducible bit for bit.
 *   mg_cut_coeffs:  bx, by, bz = open area x 2/(rho_L + rho_R) on faces between two kept
 *     cells (vol > 0 and not merged away), else 0; mask = kept.  A face between two
 *     donors that merge side by side (same direction) into face-neighbour targets adds
 *     its area to the face between the targets; other donor faces are dropped.
 *   mg_merge_rhs:  f_merged = f plus, on each target, the sources of its donors; 0 on
 *     donors (call before mg_solve).
 *   mg_merge_fill:  after the solve, p on each donor = p on its target (in place).
 * All are stream-ordered on hip_stream and return MG_EINVAL for bad dims or pointers.
 */
int mg_cut_cells(const double* psi, const int dims[3], int samples, double* ax, double* ay, double* az,
                 double* vol, int32_t* merge_to, void* hip_stream);
int mg_cut_coeffs(const double* rho, const double* ax, const double* ay, const double* az, const double* vol,
                  const int32_t* merge_to, const int dims[3], double* bx, double* by, double* bz, uint8_t* mask,
                  void* hip_stream);
int mg_merge_rhs(const int32_t* merge_to, const double* f, double* f_merged, const int dims[3], void* hip_stream);
int mg_merge_fill(const int32_t* merge_to, double* p, const int dims[3], void* hip_stream);

void mg_destroy(mg_ctx* ctx);

/* Thread-local message describing the last failure on this thread ("" if none). */
const char* mg_last_error(void);

/* ---------------------------------------------------------------------------------
 * Component entry points: single steps of the V-cycle on one level of an existing
 * hierarchy, for verification and per-kernel timing.  prec selects FP64 (double*)
 * or FP32 (float*, MIXED contexts only) arrays; level 0 is the finest grid.
 * Arrays are caller-owned device arrays of the level's size.
 * ------------------------------------------------------------------------------ */

/* Size and spacing of one grid; returns the number of grids (> 0) or an error code. */
int mg_level_info(mg_ctx* ctx, int level, int* n, double* h);

/* Copy a level's face coefficients (FP64) and activity mask out of the hierarchy. */
int mg_level_coeffs(mg_ctx* ctx, int level, double* bx, double* by, double* bz, uint8_t* mask);

/* `sweeps` red-black Gauss-Seidel sweeps on level `level` for A p = f, order MG_PRE
 * (red then black) or MG_POST (black then red); red = (i+j+k) even. */
int mg_smooth(mg_ctx* ctx, int prec, int level, void* p, const void* f, int sweeps, int order);

/* fc = 8-child mean of r = f - A p on level `level`, written at level+1 size. */
int mg_residual_restrict(mg_ctx* ctx, int prec, int level, const void* p, const void* f, void* fc);

/* p += mask * trilinear(ec): ec at level+1 size, p at level `level`. */
int mg_prolong_add(mg_ctx* ctx, int prec, int level, const void* ec, void* p);

/* e = A_c^+ (f - fluid mean of f) on the coarsest grid, in FP64 whatever prec. */
int mg_coarse_solve(mg_ctx* ctx, int prec, const void* f, void* e);

/* One V(2,2) cycle on the finest grid for A p = f, f already compatible (FP32 cycles
 * with prec = MG_PREC_F32 on MIXED contexts). */
int mg_vcycle(mg_ctx* ctx, int prec, void* p, const void* f);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
