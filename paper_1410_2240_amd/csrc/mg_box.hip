// One red-black Gauss-Seidel sweep of a small grid (32^3 and 64^3, face arrays) in a
// single launch (CDNA4).
//
// On grids this small a sweep costs latency, not bytes: two half-sweep launches, or a
// z-march whose steps each wait for a load, take several microseconds for a few
// hundred kilobytes.  Here each workgroup owns an 8 x 8 x 8 block of cells and issues
// every load it needs in one round: p on the block and a 2-cell halo (12^3 cells, into
// LDS), and f and the six face coefficients of each cell it updates (into registers).
// It then updates the first colour on the block and on a 1-cell ring around it (from old
// values only), and after a barrier the second colour on the block, whose neighbours are
// all in LDS by then: exactly the result of two half-sweeps.  The sweep is out of place
// (p_in -> p_out), since workgroups read halo cells that others write.  The update is
// that of the one-pass z-marching sweep (the same fused multiply-adds in the same order
// and the same quotient), so both give the same bits.
//
// Two variants take the launches around a V-cycle's coarse correction (section 3.1's
// cycle: smooth, restrict the residual, correct from the grid below, smooth).  The
// restricting one is the second pre-smoothing sweep: with a 3-cell halo it also updates
// the second colour on a 1-cell ring, so the block's residual can be formed from final
// values, and it writes the mean of each 2^3 child set to the grid below.  The
// prolongating one is the first post-smoothing sweep: while staging p it adds the
// trilinear interpolation of the coarse correction on active cells.  Both give the bits
// of the separate residual-restriction and prolongation passes.
#include "mg_buffer.h"
#include "mg_kernels.h"

namespace mg {

namespace {

using buf::Rsrc;
using buf::ld1;

constexpr int kBB = 8;    // block edge
constexpr int kBT = 256;  // threads per workgroup
static_assert(kBB * kBB * kBB == 2 * kBT, "two block cells per thread");

enum : int { kBoxPlain = 0, kBoxRestrict = 1, kBoxProlong = 2 };

// Staged box: the block and an H-cell halo.  The first colour is updated on the block and
// an (H-1)-cell ring, the second on the block and an (H-2)-cell ring.  A plain sweep (and
// one that first adds the prolongated coarse correction) needs H = 2; one that also forms
// the residual of the block, whose stencil reaches one cell out, needs H = 3.
template <int MODE>
struct BoxGeom {
  static constexpr int H = MODE == kBoxRestrict ? 3 : 2;
  static constexpr int E = kBB + 2 * H;
  static constexpr int Cells = E * E * E;
  static constexpr int E1 = kBB + 2 * (H - 1);
  static constexpr int N1 = E1 * E1 * E1 / 2;
  static constexpr int E2 = kBB + 2 * (H - 2);
  static constexpr int N2 = E2 * E2 * E2 / 2;
};

// the whole array as one buffer resource; a cell outside the grid in z is addressed at
// the array's end, where the range check makes the load return 0
template <typename T>
__device__ __forceinline__ Rsrc whole_rsrc(const T* a, int q) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(a), static_cast<short>(0),
                                           static_cast<int>(sizeof(T) << (3 * q)), buf::kBufferWord3);
}

// byte offset of cell (i, j, k), x and y periodic
template <typename T>
__device__ __forceinline__ unsigned off3(int i, int j, int k, int q) {
  const int m = (1 << q) - 1;
  if (k < 0 || k > m) return static_cast<unsigned>(sizeof(T)) << (3 * q);
  return static_cast<unsigned>((((k << q) | (j & m)) << q) | (i & m)) * static_cast<unsigned>(sizeof(T));
}

template <typename T>
struct BoxCoef {
  T f, xm, xp, ym, yp, zm, zp;
};

// f and the faces of cell (i, j, k): low faces at the cell's own index, high faces at the
// next cell's (the top wall's reads 0, the bottom wall's is stored as 0)
template <typename T>
__device__ __forceinline__ BoxCoef<T> load_coef(Rsrc rf, Rsrc rx, Rsrc ry, Rsrc rz, int i, int j, int k, int q) {
  const unsigned oc = off3<T>(i, j, k, q);
  BoxCoef<T> C;
  C.f = ld1(rf, oc, T());
  C.xm = ld1(rx, oc, T());
  C.xp = ld1(rx, off3<T>(i + 1, j, k, q), T());
  C.ym = ld1(ry, oc, T());
  C.yp = ld1(ry, off3<T>(i, j + 1, k, q), T());
  C.zm = ld1(rz, oc, T());
  C.zp = ld1(rz, off3<T>(i, j, k + 1, q), T());
  return C;
}

__device__ __forceinline__ double fma_b(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_b(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// the Gauss-Seidel update of box cell c (an index into a staged box of edge E)
template <typename T, int E>
__device__ __forceinline__ void box_gs(T* P, int c, const BoxCoef<T>& C, T h2, T fs) {
  constexpr int kY = E, kZ = E * E;
  const T D = C.xm + C.xp + C.ym + C.yp + C.zm + C.zp;
  if (D > T(0)) {
    const T S = fma_b(C.zp, P[c + kZ], fma_b(C.zm, P[c - kZ], fma_b(C.yp, P[c + kY], fma_b(C.ym, P[c - kY],
                fma_b(C.xp, P[c + 1], C.xm * P[c - 1])))));
    P[c] = gs_quotient(fma_b(-h2, C.f - fs, S), D);
  }
}

// r = (f - fs) - A p at box cell c, 0 on inactive cells: the flux sum and product of the
// residual passes, in their order
template <typename T, int E>
__device__ __forceinline__ T box_residual(const T* P, int c, const BoxCoef<T>& C, T inv_h2, T fs) {
  constexpr int kY = E, kZ = E * E;
  const T pc = P[c];
  const T D = C.xm + C.xp + C.ym + C.yp + C.zm + C.zp;
  const T s = fma_b(C.zp, P[c + kZ] - pc, fma_b(C.zm, P[c - kZ] - pc, fma_b(C.yp, P[c + kY] - pc,
              fma_b(C.ym, P[c - kY] - pc, fma_b(C.xp, P[c + 1] - pc, C.xm * (P[c - 1] - pc))))));
  return D > T(0) ? fma_b(-inv_h2, s, C.f - fs) : T(0);
}

// what the restricting and prolongating variants read or write besides the sweep's arrays
template <typename T>
struct BoxExtra {
  T* fc;                  // restrict: mean of the block's residuals over each 2^3 child set
  T* ec;                  // restrict: the coarse correction, zeroed
  const T* ecin;          // prolong: the coarse correction, added to p before the sweep
  const uint8_t* mask;    // prolong: active cells of this grid (the correction lands there only)
  T inv_h2;
};

template <typename T, int MODE, bool ZIN>
__global__ __launch_bounds__(kBT) void k_rbgs_box(const T* __restrict__ pin, T* __restrict__ pout,
                                                  const T* __restrict__ f, const T* __restrict__ bx,
                                                  const T* __restrict__ by, const T* __restrict__ bz, int q, T h2,
                                                  int first, const double* __restrict__ fshift, BoxExtra<T> xa) {
  using G = BoxGeom<MODE>;
  constexpr int H = G::H, E = G::E;
  constexpr int kPerS = (G::Cells + kBT - 1) / kBT, kPer1 = (G::N1 + kBT - 1) / kBT, kPer2 = (G::N2 + kBT - 1) / kBT;
  // box cell (x, y, z) is grid cell (i0 - H + x, j0 - H + y, k0 - H + z), at (z E + y) E + x
  __shared__ T P[G::Cells];
  // restrict: the block's residuals; prolong: the coarse correction around the box (8^3)
  __shared__ T X[MODE == kBoxPlain ? 1 : 2 * kBT];
  const int n = 1 << q, nb = n / kBB;
  const int tid = threadIdx.x, b = blockIdx.x;
  const int i0 = (b % nb) * kBB, j0 = ((b / nb) % nb) * kBB, k0 = (b / (nb * nb)) * kBB;
  const T fs = fshift ? static_cast<T>(*fshift) : T(0);
  const Rsrc rp = whole_rsrc(pin, q), rf = whole_rsrc(f, q);
  const Rsrc rx = whole_rsrc(bx, q), ry = whole_rsrc(by, q), rz = whole_rsrc(bz, q);

  // ---- one round of loads: the box of p, the coefficients of every cell this thread
  // updates (and, restricting, of its block cells), the coarse correction (prolonging)
  T sv[kPerS];
  bool live[kPerS];   // prolong: an active cell inside the grid
#pragma unroll
  for (int u = 0; u < kPerS; ++u) {
    const int e = tid + u * kBT;
    const int x = e % E, y = (e / E) % E, z = e / (E * E);
    const int gi = i0 - H + x, gj = j0 - H + y, gk = k0 - H + z;
    sv[u] = (ZIN || e >= G::Cells) ? T(0) : ld1(rp, off3<T>(gi, gj, gk, q), T());
    live[u] = false;
    if constexpr (MODE == kBoxProlong) {
      if (e < G::Cells && gk >= 0 && gk < n) live[u] = xa.mask[off3<uint8_t>(gi, gj, gk, q)] != 0;
    }
  }
  T ev[2];
  if constexpr (MODE == kBoxProlong) {
    const int qc = q - 1, mc = (1 << qc) - 1;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + u * kBT;
      const int x = e % 8, y = (e / 8) % 8, z = e / 64;
      const int K = min(max((k0 >> 1) - 2 + z, 0), mc);   // parent reused beyond a z wall
      ev[u] = xa.ecin[(((K << qc) | (((j0 >> 1) - 2 + y) & mc)) << qc) | (((i0 >> 1) - 2 + x) & mc)];
    }
  }
  BoxCoef<T> c1[kPer1];
  int l1[kPer1];   // box index of the cell (-1: none)
#pragma unroll
  for (int u = 0; u < kPer1; ++u) {
    const int e = tid + u * kBT;
    l1[u] = -1;
    if (e < G::N1) {
      const int row = e / (G::E1 / 2), xh = e % (G::E1 / 2);
      const int yy = row % G::E1, zz = row / G::E1;
      const int gi0 = i0 - (H - 1), gy = j0 - (H - 1) + yy, gz = k0 - (H - 1) + zz;
      const int lx = 2 * xh + ((first + gi0 + gy + gz) & 1);   // colour: parity of i + j + k
      l1[u] = ((zz + 1) * E + (yy + 1)) * E + (lx + 1);
      c1[u] = load_coef<T>(rf, rx, ry, rz, gi0 + lx, gy, gz, q);
    }
  }
  BoxCoef<T> c2[kPer2];
  int l2[kPer2];
#pragma unroll
  for (int u = 0; u < kPer2; ++u) {
    const int e = tid + u * kBT;
    l2[u] = -1;
    if (e < G::N2) {
      const int row = e / (G::E2 / 2), xh = e % (G::E2 / 2);
      const int yy = row % G::E2, zz = row / G::E2;
      const int gi0 = i0 - (H - 2), gy = j0 - (H - 2) + yy, gz = k0 - (H - 2) + zz;
      const int lx = 2 * xh + ((1 - first + gi0 + gy + gz) & 1);
      l2[u] = ((zz + 2) * E + (yy + 2)) * E + (lx + 2);
      c2[u] = load_coef<T>(rf, rx, ry, rz, gi0 + lx, gy, gz, q);
    }
  }
  BoxCoef<T> cr[2];   // restrict: block cells tid and tid + 256
  if constexpr (MODE == kBoxRestrict) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + u * kBT;
      cr[u] = load_coef<T>(rf, rx, ry, rz, i0 + e % kBB, j0 + (e / kBB) % kBB, k0 + e / (kBB * kBB), q);
    }
  }

  // ---- prolong: p + the trilinear coarse correction on active cells, with the fused
  // multiply-adds of the prolongation pass in its order (x weights, then y, then z)
  if constexpr (MODE == kBoxProlong) {
    X[tid] = ev[0];
    X[tid + kBT] = ev[1];
    __syncthreads();
    const T w3 = T(0.75), w1 = T(0.25);
#pragma unroll
    for (int u = 0; u < kPerS; ++u) {
      if (!live[u]) continue;
      const int e = tid + u * kBT;
      const int ox = e % E - H, oy = (e / E) % E - H, oz = e / (E * E) - H;   // from the block origin
      const int cx = (ox >> 1) + 2, cy = (oy >> 1) + 2, cz = (oz >> 1) + 2;     // parent in the coarse box
      const int xs = (ox & 1) ? cx + 1 : cx - 1, ya = (oy & 1) ? cy + 1 : cy - 1, zb = (oz & 1) ? cz + 1 : cz - 1;
      auto ax = [&](int zz, int yy) {
        const T e1 = X[(zz * 8 + yy) * 8 + cx], e0 = X[(zz * 8 + yy) * 8 + xs];
        return fma_b(w3, e1, w1 * e0);
      };
      const T a11 = ax(cz, cy), a1y = ax(cz, ya), az1 = ax(zb, cy), azy = ax(zb, ya);
      const T lo = fma_b(w3, a11, w1 * a1y);
      const T hi = fma_b(w3, az1, w1 * azy);
      const T out = fma_b(w3, lo, w1 * hi);
      sv[u] += out;
    }
  }
#pragma unroll
  for (int u = 0; u < kPerS; ++u) {
    const int e = tid + u * kBT;
    if (e < G::Cells) P[e] = sv[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer1; ++u)
    if (l1[u] >= 0) box_gs<T, E>(P, l1[u], c1[u], h2, fs);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer2; ++u)
    if (l2[u] >= 0) box_gs<T, E>(P, l2[u], c2[u], h2, fs);
  __syncthreads();
  // ---- restrict: the residual of each block cell, then the mean over each coarse cell's
  // children in the order of the restriction passes: (row 2J, plane 2K), (row 2J+1, plane
  // 2K), (row 2J, plane 2K+1), (row 2J+1, plane 2K+1), each pair as x-even + x-odd
  if constexpr (MODE == kBoxRestrict) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + u * kBT;
      const int c = ((e / (kBB * kBB) + H) * E + ((e / kBB) % kBB + H)) * E + (e % kBB + H);
      X[e] = box_residual<T, E>(P, c, cr[u], xa.inv_h2, fs);
    }
    __syncthreads();
    if (tid < 64) {
      const int cx = tid % 4, cy = (tid / 4) % 4, cz = tid / 16;
      auto r = [&](int dz, int dy, int dx) { return X[((2 * cz + dz) * kBB + (2 * cy + dy)) * kBB + (2 * cx + dx)]; };
      T sum = T(0);
      sum += r(0, 0, 0) + r(0, 0, 1);
      sum += r(0, 1, 0) + r(0, 1, 1);
      sum += r(1, 0, 0) + r(1, 0, 1);
      sum += r(1, 1, 0) + r(1, 1, 1);
      const int qc = q - 1;
      const int C = (((((k0 >> 1) + cz) << qc) | ((j0 >> 1) + cy)) << qc) | ((i0 >> 1) + cx);
      xa.fc[C] = sum * T(0.125);
      xa.ec[C] = T(0);
    }
  }
  // ---- the block out: rows of 8 cells
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * kBT;
    const int x = e % kBB, y = (e / kBB) % kBB, z = e / (kBB * kBB);
    pout[(static_cast<long long>(k0 + z) << (2 * q)) | ((j0 + y) << q) | (i0 + x)] =
        P[((z + H) * E + (y + H)) * E + (x + H)];
  }
}

template <typename T, int MODE, bool ZIN>
hipError_t launch_box(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q, double h,
                      int order, const double* fshift, const BoxExtra<T>& xa, hipStream_t s) {
  const int nb = (1 << q) / kBB;
  const T h2 = static_cast<T>(h * h);
  const int first = order == 0 ? 0 : 1;   // pre-smoothing: red first; post-smoothing: black first
  hipLaunchKernelGGL((k_rbgs_box<T, MODE, ZIN>), dim3(static_cast<unsigned>(nb * nb * nb)), dim3(kBT), 0, s, pin,
                     pout, f, bx, by, bz, q, h2, first, fshift, xa);
  return hipGetLastError();
}

}  // namespace

int box_sweep_supported(int q) { return q == 5 || q == 6; }

template <typename T>
hipError_t launch_rbgs_box(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q, double h,
                           int order, const double* fshift, int zero_in, hipStream_t s) {
  if (!box_sweep_supported(q) || pin == pout) return hipErrorInvalidValue;
  const BoxExtra<T> none{};
  return zero_in ? launch_box<T, kBoxPlain, true>(pin, pout, f, bx, by, bz, q, h, order, fshift, none, s)
                 : launch_box<T, kBoxPlain, false>(pin, pout, f, bx, by, bz, q, h, order, fshift, none, s);
}

template <typename T>
hipError_t launch_rbgs_box_restrict(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q,
                                    double h, int order, const double* fshift, T* fc, T* ec, hipStream_t s) {
  if (!box_sweep_supported(q) || pin == pout || !fc || !ec) return hipErrorInvalidValue;
  BoxExtra<T> xa{};
  xa.fc = fc;
  xa.ec = ec;
  xa.inv_h2 = static_cast<T>(1.0 / (h * h));
  return launch_box<T, kBoxRestrict, false>(pin, pout, f, bx, by, bz, q, h, order, fshift, xa, s);
}

template <typename T>
hipError_t launch_rbgs_box_prolong(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q,
                                   double h, int order, const double* fshift, const T* ec, const uint8_t* mask,
                                   hipStream_t s) {
  if (!box_sweep_supported(q) || pin == pout || !ec || !mask) return hipErrorInvalidValue;
  BoxExtra<T> xa{};
  xa.ecin = ec;
  xa.mask = mask;
  return launch_box<T, kBoxProlong, false>(pin, pout, f, bx, by, bz, q, h, order, fshift, xa, s);
}

#define MG_BOX_INSTANCES(T)                                                                                           \
  template hipError_t launch_rbgs_box<T>(const T*, T*, const T*, const T*, const T*, const T*, int, double, int,      \
                                         const double*, int, hipStream_t);                                            \
  template hipError_t launch_rbgs_box_restrict<T>(const T*, T*, const T*, const T*, const T*, const T*, int, double, \
                                                  int, const double*, T*, T*, hipStream_t);                           \
  template hipError_t launch_rbgs_box_prolong<T>(const T*, T*, const T*, const T*, const T*, const T*, int, double,  \
                                                 int, const double*, const T*, const uint8_t*, hipStream_t);
MG_BOX_INSTANCES(double)
MG_BOX_INSTANCES(float)
#undef MG_BOX_INSTANCES

}  // namespace mg
