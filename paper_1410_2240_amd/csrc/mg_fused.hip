// One full red-black Gauss-Seidel sweep in a single pass over memory (CDNA4).
//
// Two half-sweep launches read every cache line of p, f and the three face arrays
// twice.  Here each workgroup owns a TX x TY tile of x-y cells and a chunk of KC
// z-planes, and marches up the chunk: at step k it updates the first colour on plane
// k+1 and then the second colour on plane k.  The second colour on plane k needs the
// first colour on planes k-1, k, k+1 already updated, and the first colour on plane k+1
// needs the second colour on planes k, k+1, k+2 still old, so this wavefront order gives
// exactly the result of two half-sweeps.  Planes of p are staged in LDS with a 2-cell
// halo; the first colour is also updated on a 1-cell ring around the tile (from old
// values only), so every second-colour update at the tile edge finds its neighbours
// without waiting for another workgroup.  The sweep is out of place (p_in -> p_out):
// workgroups read halo cells that other workgroups write.
//
// Loads: a step issues the loads of the following planes before its barriers (the p
// plane three ahead into registers, f and the face coefficients of both cells of the
// thread's x-pair two ahead, as 16-byte loads so each cache line is fetched once for
// both colours), so memory latency overlaps the work on the current planes.
//
// Traffic per sweep: p, f and the three face arrays read once and p written once
// (6 scalars per cell), plus halo and chunk-boundary overlap served mostly by L2.
//
// Density form (finest grid of a hierarchy built from rho, FP64): instead of the three
// face arrays the sweep reads rt = rho on active cells, +inf elsewhere, and forms each
// face coefficient as 2 / (rt_L + rt_R) (face_beta, as the setup does), which is 0
// wherever a face touches an inactive cell or a wall and otherwise bit for bit the
// stored coefficient.  That is 4 scalars per cell per sweep instead of 6, for nine
// reciprocals per x-pair and plane (each face once).
#include <algorithm>

#include "mg_buffer.h"
#include "mg_kernels.h"

#include <type_traits>

namespace mg {

namespace {

using buf::Vec2;
using buf::Rsrc;
using buf::plane_rsrc;
using buf::off_of;
using buf::ld1;
using buf::ld2;

// in-plane byte offsets around a thread's x-pair (i even, i+1) in row j
struct PairOffsets {
  unsigned c;    // the pair
  unsigned xl;   // cell i-1
  unsigned xr;   // cell i+2
  unsigned yd;   // the pair in row j-1
  unsigned yu;   // the pair in row j+1
};

// f and the six face coefficients of one cell: everything but p that its update reads
template <typename T>
struct Coef {
  T f, xm, xp, ym, yp, zm, zp;
};

template <typename T>
__device__ __forceinline__ Coef<T> load_cell(const T* __restrict__ f, const T* __restrict__ bx,
                                             const T* __restrict__ by, const T* __restrict__ bz, int i, int j, int kk,
                                             int q) {
  // planes outside the grid read as 0 (no coefficients, no source)
  Coef<T> C;
  const unsigned oc = off_of<T>(i, j, q), ox = off_of<T>(i + 1, j, q), oy = off_of<T>(i, j + 1, q);
  const Rsrc xk = plane_rsrc(bx, kk, q), yk = plane_rsrc(by, kk, q);
  C.f = ld1(plane_rsrc(f, kk, q), oc, T());
  C.xm = ld1(xk, oc, T());
  C.xp = ld1(xk, ox, T());
  C.ym = ld1(yk, oc, T());
  C.yp = ld1(yk, oy, T());
  C.zm = ld1(plane_rsrc(bz, kk, q), oc, T());
  C.zp = ld1(plane_rsrc(bz, kk + 1, q), oc, T());   // top wall: plane n reads 0
  return C;
}

// The coefficients of both cells of an x-pair (i even, i+1) on one plane, loaded with
// 2-wide loads so that each cache line is fetched once for both colours.
template <typename T>
struct PairRaw {
  typename Vec2<T>::type f, bx, by, byu, bz, bzu;
  T bxr;   // x face above the odd cell (low face of i+2)
};

template <typename T>
__device__ __forceinline__ void load_pair(PairRaw<T>& R, const T* __restrict__ f, const T* __restrict__ bx,
                                          const T* __restrict__ by, const T* __restrict__ bz, const PairOffsets& o,
                                          int kk, int q) {
  const Rsrc xk = plane_rsrc(bx, kk, q), yk = plane_rsrc(by, kk, q);
  R.f = ld2(plane_rsrc(f, kk, q), o.c, T());
  R.bx = ld2(xk, o.c, T());
  R.bxr = ld1(xk, o.xr, T());
  R.by = ld2(yk, o.c, T());
  R.byu = ld2(yk, o.yu, T());
  R.bz = ld2(plane_rsrc(bz, kk, q), o.c, T());
  R.bzu = ld2(plane_rsrc(bz, kk + 1, q), o.c, T());   // top wall: plane n reads 0
}

// coefficients of the even (ODD = false) or odd (ODD = true) cell of a pair
template <bool ODD, typename T>
__device__ __forceinline__ Coef<T> cell_of(const PairRaw<T>& R) {
  Coef<T> C;
  if (ODD) {
    C.f = R.f.y;
    C.xm = R.bx.y;
    C.xp = R.bxr;
    C.ym = R.by.y;
    C.yp = R.byu.y;
    C.zm = R.bz.y;
    C.zp = R.bzu.y;
  } else {
    C.f = R.f.x;
    C.xm = R.bx.x;
    C.xp = R.bx.y;
    C.ym = R.by.x;
    C.yp = R.byu.x;
    C.zm = R.bz.x;
    C.zp = R.bzu.x;
  }
  return C;
}

// ---- density form
template <typename T>
__device__ __forceinline__ T beta_rho(T a, T b) { return face_beta(a, b); }

// f and the in-plane densities around an x-pair of one plane; the pair's own densities
// (c) come from the z window the kernel keeps
template <typename T>
struct PairRho {
  typename Vec2<T>::type f, c, s, n;   // f, rt of the pair, rt of the pair in rows j-1 and j+1
  T l, r;                              // rt at i-1 and i+2
};

// A plane outside the grid reads as 0 through its buffer descriptor; its densities are
// +inf (beyond a z wall).  The replacement is a separate step, applied where the values
// are first used: done at the load, it would make the compiler wait for a prefetch in
// the step that issues it instead of the step that consumes it.
template <typename T>
__device__ __forceinline__ typename Vec2<T>::type wall_rho(typename Vec2<T>::type v, int kk, int q) {
  const T inf = __builtin_huge_val();
  const bool in = kk >= 0 && kk < (1 << q);
  return typename Vec2<T>::type{in ? v.x : inf, in ? v.y : inf};
}

template <typename T>
__device__ __forceinline__ typename Vec2<T>::type load_centre_raw(const T* __restrict__ rt, unsigned oc, int kk,
                                                                  int q) {
  return ld2(plane_rsrc(rt, kk, q), oc, T());
}

template <typename T>
__device__ __forceinline__ typename Vec2<T>::type load_centre(const T* __restrict__ rt, unsigned oc, int kk, int q) {
  return wall_rho<T>(load_centre_raw(rt, oc, kk, q), kk, q);
}

// raw loads of a plane's f and in-plane densities (planes outside the grid read 0)
template <typename T>
__device__ __forceinline__ void load_pair_rho_raw(PairRho<T>& R, const T* __restrict__ f, const T* __restrict__ rt,
                                                  typename Vec2<T>::type centre, const PairOffsets& o, int kk, int q) {
  const Rsrc rk = plane_rsrc(rt, kk, q);
  R.c = centre;
  R.f = ld2(plane_rsrc(f, kk, q), o.c, T());
  R.l = ld1(rk, o.xl, T());
  R.r = ld1(rk, o.xr, T());
  R.s = ld2(rk, o.yd, T());
  R.n = ld2(rk, o.yu, T());
}

// the wall replacement of a plane's densities loaded by load_pair_rho_raw (the centre
// included: replacing it twice is harmless)
template <typename T>
__device__ __forceinline__ void wall_pair_rho(PairRho<T>& R, int kk, int q) {
  using V2 = typename Vec2<T>::type;
  R.c = wall_rho<T>(R.c, kk, q);
  const V2 lr = wall_rho<T>(V2{R.l, R.r}, kk, q);
  R.l = lr.x;
  R.r = lr.y;
  R.s = wall_rho<T>(R.s, kk, q);
  R.n = wall_rho<T>(R.n, kk, q);
}

template <typename T>
__device__ __forceinline__ void load_pair_rho(PairRho<T>& R, const T* __restrict__ f, const T* __restrict__ rt,
                                              typename Vec2<T>::type centre, const PairOffsets& o, int kk, int q) {
  load_pair_rho_raw(R, f, rt, centre, o, kk, q);
  wall_pair_rho(R, kk, q);
}

// Both cells' coefficients of a pair from its plane's densities, every face once: zm
// holds the pair's faces to the plane below (computed with that plane), `above` the
// pair's densities on the plane above.  Returns the pair's faces to the plane above.
template <typename T>
__device__ __forceinline__ typename Vec2<T>::type pair_coef_rho(const PairRho<T>& R, typename Vec2<T>::type zm,
                                                                typename Vec2<T>::type above, Coef<T>& even,
                                                                Coef<T>& odd) {
  using V2 = typename Vec2<T>::type;
  const T x1 = beta_rho(R.c.x, R.c.y);
  const V2 zp{beta_rho(R.c.x, above.x), beta_rho(R.c.y, above.y)};
  even = Coef<T>{R.f.x, beta_rho(R.l, R.c.x), x1, beta_rho(R.s.x, R.c.x), beta_rho(R.c.x, R.n.x), zm.x, zp.x};
  odd = Coef<T>{R.f.y, x1, beta_rho(R.c.y, R.r), beta_rho(R.s.y, R.c.y), beta_rho(R.c.y, R.n.y), zm.y, zp.y};
  return zp;
}

// one cell's coefficients (the ring cells and the prologue)
template <typename T>
__device__ __forceinline__ Coef<T> load_cell_rho(const T* __restrict__ f, const T* __restrict__ rt, int i, int j,
                                                 int kk, int q) {
  Coef<T> C;
  const int n = 1 << q;
  if (kk < 0 || kk >= n) {
    C.f = C.xm = C.xp = C.ym = C.yp = C.zm = C.zp = T(0);
    return C;
  }
  const unsigned oc = off_of<T>(i, j, q);
  const Rsrc rk = plane_rsrc(rt, kk, q);
  const T rc = ld1(rk, oc, T());
  C.f = ld1(plane_rsrc(f, kk, q), oc, T());
  C.xm = beta_rho(ld1(rk, off_of<T>(i - 1, j, q), T()), rc);
  C.xp = beta_rho(rc, ld1(rk, off_of<T>(i + 1, j, q), T()));
  C.ym = beta_rho(ld1(rk, off_of<T>(i, j - 1, q), T()), rc);
  C.yp = beta_rho(rc, ld1(rk, off_of<T>(i, j + 1, q), T()));
  C.zm = kk > 0 ? beta_rho(ld1(plane_rsrc(rt, kk - 1, q), oc, T()), rc) : T(0);
  C.zp = kk < n - 1 ? beta_rho(rc, ld1(plane_rsrc(rt, kk + 1, q), oc, T())) : T(0);
  return C;
}

// A ring cell's f and densities as raw loads (its plane and the planes below and above
// through their buffer descriptors, 0 outside the grid) ...
template <typename T>
struct CellRho {
  T f, c, l, r, s, n, lo, hi;
};

template <typename T>
__device__ __forceinline__ CellRho<T> load_cell_rho_raw(const T* __restrict__ f, const T* __restrict__ rt, int i,
                                                        int j, int kk, int q) {
  CellRho<T> R;
  const unsigned oc = off_of<T>(i, j, q);
  const Rsrc rk = plane_rsrc(rt, kk, q);
  R.f = ld1(plane_rsrc(f, kk, q), oc, T());
  R.c = ld1(rk, oc, T());
  R.l = ld1(rk, off_of<T>(i - 1, j, q), T());
  R.r = ld1(rk, off_of<T>(i + 1, j, q), T());
  R.s = ld1(rk, off_of<T>(i, j - 1, q), T());
  R.n = ld1(rk, off_of<T>(i, j + 1, q), T());
  R.lo = ld1(plane_rsrc(rt, kk - 1, q), oc, T());
  R.hi = ld1(plane_rsrc(rt, kk + 1, q), oc, T());
  return R;
}

// ... and its coefficients once they are needed: densities beyond a z wall become +inf,
// which closes those faces, so this equals load_cell_rho bit for bit (a plane outside
// the grid gets f = 0 and six closed faces)
template <typename T>
__device__ __forceinline__ Coef<T> cell_coef_rho(const CellRho<T>& R, int kk, int q) {
  using V2 = typename Vec2<T>::type;
  const V2 cl = wall_rho<T>(V2{R.c, R.l}, kk, q);
  const V2 rs = wall_rho<T>(V2{R.r, R.s}, kk, q);
  const T nn = wall_rho<T>(V2{R.n, R.n}, kk, q).x;
  const T lo = wall_rho<T>(V2{R.lo, R.lo}, kk - 1, q).x;
  const T hi = wall_rho<T>(V2{R.hi, R.hi}, kk + 1, q).x;
  const T c = cl.x;
  Coef<T> C;
  C.f = R.f;
  C.xm = beta_rho(cl.y, c);
  C.xp = beta_rho(c, rs.x);
  C.ym = beta_rho(rs.y, c);
  C.yp = beta_rho(c, nn);
  C.zm = beta_rho(lo, c);
  C.zp = beta_rho(c, hi);
  return C;
}

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// A staged plane keeps each row split by column parity, [row][c & 1][c >> 1], so a wave
// updating one colour reads consecutive words (no LDS bank conflicts).
template <typename T, int W>
__device__ __forceinline__ T& at(T (*pl)[2][W / 2], int r, int c) {
  return pl[r][c & 1][c >> 1];
}

// Gauss-Seidel update of the cell at (r, c) of staged plane `cur`; lo / hi are its z
// neighbours below and above.
template <typename T, int W>
__device__ __forceinline__ void gs(T (*cur)[2][W / 2], int r, int c, T lo, T hi, const Coef<T>& C, T h2, T fs) {
  const T D = C.xm + C.xp + C.ym + C.yp + C.zm + C.zp;
  if (D > T(0)) {
    // explicit fused multiply-adds: the rounding is fixed by the source, whichever form
    // the coefficients come in
    const T S = fmad(C.zp, hi, fmad(C.zm, lo, fmad(C.yp, at<T, W>(cur, r + 1, c), fmad(C.ym, at<T, W>(cur, r - 1, c),
                fmad(C.xp, at<T, W>(cur, r, c + 1), C.xm * at<T, W>(cur, r, c - 1))))));
    at<T, W>(cur, r, c) = gs_quotient(fmad(-h2, C.f - fs, S), D);
  }
}


// Tiles of TX x TY cells, one thread per x-pair of tile cells: 64 x 8 and 128 x 8 for
// N = 64 and 128 (the x halo wraps onto the tile's own cache lines), 128 x 16 above
// (one wave per tile row; fewer halo rows and ring cells per tile cell than 256 x 8).
template <typename T, int TX, int TY, bool RHO, bool ZIN>
__global__ __launch_bounds__(TX / 2 * TY) void k_rbgs_fused(const T* __restrict__ pin, T* __restrict__ pout,
                                                              const T* __restrict__ f, const T* __restrict__ bx,
                                                              const T* __restrict__ by, const T* __restrict__ bz,
                                                              const T* __restrict__ rt, int q, int kc, T h2,
                                                              int first, const double* __restrict__ fshift) {
  using V2 = typename Vec2<T>::type;
  constexpr int NT = TX / 2 * TY;
  constexpr int W = TX + 4;                 // columns i0-2 .. i0+TX+1
  constexpr int H = TY + 4;                 // rows    j0-2 .. j0+TY+1
  constexpr int BOX = H * (W / 2);          // pairs per staged plane
  constexpr int PER = (BOX + NT - 1) / NT;  // pairs per thread
  __shared__ T L[4][H][2][W / 2];
  // FP64: the second colour's coefficients, carried from one step to the next, wait in
  // LDS (each thread its own column of words) rather than in 14 registers, which the
  // prefetches of the next planes need
  constexpr bool CARRY_LDS = sizeof(T) == 8;
  __shared__ T CB[CARRY_LDS ? 7 : 1][CARRY_LDS ? NT : 1];
  const int n = 1 << q, m = n - 1;
  const int tid = threadIdx.x;
  // Consecutive logical tiles run on one XCD (blocks are dealt to the 8 XCDs in turn):
  // the y-neighbours of a tile are then co-resident and its halo rows hit that L2.
  const int G = gridDim.x;
  const int bid = blockIdx.x;
  const int lid = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;
  const int ntx = n / TX, nty = n / TY;
  const int i0 = (lid % ntx) * TX;
  const int j0 = ((lid / ntx) % nty) * TY;
  const int k0 = (lid / (ntx * nty)) * kc;
  const int k1 = k0 + kc;
  const T fs = fshift ? static_cast<T>(*fshift) : T(0);
  // A step branches on the colour parity of the thread's row, and contains barriers:
  // every wave must hold rows of one parity.  A wave spans R = 64 / (TX/2) rows (R = 1
  // for TX >= 128); in each group of 2R tile rows one wave takes the even rows and the
  // next wave the odd ones (TX = 64: (0,2), (1,3), (4,6), (5,7); TX = 32: (0,2,4,6),
  // (1,3,5,7)).
  constexpr int R = TX >= 128 ? 1 : 128 / TX;
  static_assert(TY % (2 * R) == 0, "tile rows must split into waves of one parity");
  const int xt = tid % (TX / 2);
  const int half = tid / (TX / 2);
  const int jt = ((half / R) / 2) * (2 * R) + 2 * (half % R) + (half / R) % 2;
  const int jrow = j0 + jt;
  const int ipair = i0 + 2 * xt;
  const PairOffsets po{off_of<T>(ipair, jrow, q), off_of<T>(ipair - 1, jrow, q), off_of<T>(ipair + 2, jrow, q),
                       off_of<T>(ipair, jrow - 1, q), off_of<T>(ipair, jrow + 1, q)};

  // ---- staged p planes: global -> registers (one plane ahead) -> LDS
  V2 pn[PER];
  unsigned op[PER];   // in-plane offsets of this thread's pairs of the staged box
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + u * NT;
    const int r = e / (W / 2), cp = e % (W / 2);
    op[u] = e < BOX ? off_of<T>(i0 - 2 + 2 * cp, j0 - 2 + r, q) : 0u;   // past the box: a harmless load
  }
  auto fetch_plane = [&](int kk) {   // a plane outside the grid reads as 0
    if constexpr (ZIN) {   // the input is known to be zero: nothing to read
#pragma unroll
      for (int u = 0; u < PER; ++u) pn[u] = V2{T(0), T(0)};
    } else {
      const Rsrc pk = plane_rsrc(pin, kk, q);
#pragma unroll
      for (int u = 0; u < PER; ++u) pn[u] = ld2(pk, op[u], T());
    }
  };
  auto store_plane = [&](int slot) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT;
      if (e < BOX) {
        const int r = e / (W / 2), cp = e % (W / 2);
        L[slot][r][0][cp] = pn[u].x;
        L[slot][r][1][cp] = pn[u].y;
      }
    }
  };

  // ---- the ring cell of the first colour this thread updates (threads 0 .. TX+TY-1)
  // rows j0-1 and j0+TY (TX/2 cells each), columns i0-1 / i0+TX (one cell per tile row)
  auto ring_cell = [&](int kk, int& r, int& c, int& i, int& j) {
    if (tid < TX) {
      const int side = tid / (TX / 2), x = tid % (TX / 2);
      r = side ? TY + 2 : 1;
      j = (j0 - 2 + r) & m;
      const int bit = (first + j + kk + i0) & 1;
      c = 2 * x + bit + 2;
      i = i0 + 2 * x + bit;
    } else {
      const int rr = tid - TX;
      j = j0 + rr;
      r = rr + 2;
      const bool left = ((i0 - 1 + j + kk) & 1) == first;
      c = left ? 1 : TX + 2;
      i = (left ? i0 - 1 : i0 + TX) & m;
    }
  };
  const bool has_ring = tid < TX + TY;

  // first-colour / second-colour cell of this thread's pair on plane kk
  auto first_odd = [&](int kk) { return ((first + jrow + kk) & 1) != 0; };
  const int rt_ = jt + 2, ct = 2 * xt + 2;   // the pair's place in a staged plane

  // ---- prologue.  Plane kk is staged in slot kk & 3; plane k0-2 of the pair in registers.
  auto slot = [](int kk) { return kk & 3; };
  // one cell's coefficients in either form
  auto coef_at = [&](int i, int j, int kk) {
    if constexpr (RHO)
      return load_cell_rho(f, rt, i, j, kk, q);
    else
      return load_cell(f, bx, by, bz, i, j, kk, q);
  };
  int rr_, rc_, ri_, rj_;
  PairRaw<T> raw;        // both cells' coefficients of the plane above the current one
  PairRho<T> rraw;       // density form: the same plane's f and in-plane densities
  V2 rc_hi;              // density form: the pair's densities two planes up
  V2 zlo;                // density form: the pair's faces between the current plane and the next
  Coef<T> black_cur;     // second colour's coefficients on the current plane (or in CB)
  auto put_black = [&](const Coef<T>& C) {
    if constexpr (CARRY_LDS) {
      CB[0][tid] = C.f;
      CB[1][tid] = C.xm;
      CB[2][tid] = C.xp;
      CB[3][tid] = C.ym;
      CB[4][tid] = C.yp;
      CB[5][tid] = C.zm;
      CB[6][tid] = C.zp;
    } else {
      black_cur = C;
    }
  };
  auto get_black = [&]() {
    if constexpr (CARRY_LDS)
      return Coef<T>{CB[0][tid], CB[1][tid], CB[2][tid], CB[3][tid], CB[4][tid], CB[5][tid], CB[6][tid]};
    else
      return black_cur;
  };
  T below0, below1;      // the pair's finished values on the plane under the current one
  {
    const Coef<T> red_m1 = coef_at(ipair + first_odd(k0 - 1), jrow, k0 - 1);
    const Coef<T> red_0 = coef_at(ipair + first_odd(k0), jrow, k0);
    put_black(coef_at(ipair + !first_odd(k0), jrow, k0));
    Coef<T> ring_0;
    if (has_ring) {
      ring_cell(k0, rr_, rc_, ri_, rj_);
      ring_0 = coef_at(ri_, rj_, k0);
    }
    T pm2_0 = T(0), pm2_1 = T(0);   // the pair on plane k0-2
    if constexpr (!ZIN) {
      const V2 v = ld2(plane_rsrc(pin, k0 - 2, q), po.c, T());   // 0 below the grid
      pm2_0 = v.x;
      pm2_1 = v.y;
    }
    if constexpr (RHO) {
      const V2 rc0 = load_centre(rt, po.c, k0, q);
      load_pair_rho(rraw, f, rt, load_centre(rt, po.c, k0 + 1, q), po, k0 + 1, q);
      rc_hi = load_centre(rt, po.c, k0 + 2, q);
      zlo = V2{beta_rho(rc0.x, rraw.c.x), beta_rho(rc0.y, rraw.c.y)};
    } else {
      load_pair(raw, f, bx, by, bz, po, k0 + 1, q);
    }
    fetch_plane(k0 - 1);
    store_plane(slot(k0 - 1));
    fetch_plane(k0);
    store_plane(slot(k0));
    fetch_plane(k0 + 1);
    store_plane(slot(k0 + 1));
    fetch_plane(k0 + 2);
    __syncthreads();
    const int sm = slot(k0 - 1), s0 = slot(k0), s1 = slot(k0 + 1);
    if (k0 - 1 >= 0) {
      const int o = first_odd(k0 - 1);
      gs<T, W>(L[sm], rt_, ct + o, o ? pm2_1 : pm2_0, at<T, W>(L[s0], rt_, ct + o), red_m1, h2, fs);
    }
    below0 = at<T, W>(L[sm], rt_, ct);   // own cells: only this thread wrote them
    below1 = at<T, W>(L[sm], rt_, ct + 1);
    {
      const int c = ct + first_odd(k0);
      gs<T, W>(L[s0], rt_, c, at<T, W>(L[sm], rt_, c), at<T, W>(L[s1], rt_, c), red_0, h2, fs);
    }
    if (has_ring) {
      ring_cell(k0, rr_, rc_, ri_, rj_);
      gs<T, W>(L[s0], rr_, rc_, at<T, W>(L[sm], rr_, rc_), at<T, W>(L[s1], rr_, rc_), ring_0, h2, fs);
    }
    // Enter the loop with no load in flight.  The compiler counts outstanding loads
    // across the loop entry and the back edge together; a prefetch still pending from
    // here would make it wait for every load, this step's prefetches included, at the
    // first use of a staged plane in every step.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  // One step, for the first colour on plane k+1 sitting in the odd (ODD1) or even cell
  // of the pair; a wave holds rows of one parity, so the choice is uniform per wave.
  // On entry: plane k (first colour done on
  // tile + ring) in slot k, plane k+1 (old) in slot k+1, pn = plane k+2, raw = the
  // coefficients of plane k+1, black_cur = the second colour's on plane k.  One barrier
  // per step (after staging plane k+2): four slots let the next step stage its plane
  // while a slower wave of this step still reads planes k .. k+2.
  auto step = [&](int k, auto odd_tag) {
    constexpr bool ODD1 = decltype(odd_tag)::value;
    const int s0 = slot(k), s1 = slot(k + 1), s2 = slot(k + 2);
    // the ring cell's loads first: they are used right after the barrier, and waiting
    // for them must not wait for the prefetches of the planes above (the density form
    // forms the ring cell's faces after the barrier for the same reason)
    Coef<T> ring_c;
    CellRho<T> ring_raw;
    if (has_ring) {
      ring_cell(k + 1, rr_, rc_, ri_, rj_);
      if constexpr (RHO)
        ring_raw = load_cell_rho_raw(f, rt, ri_, rj_, k + 1, q);
      else
        ring_c = load_cell(f, bx, by, bz, ri_, rj_, k + 1, q);
    }
    store_plane(s2);                   // plane k+2
    fetch_plane(k + 3);
    PairRaw<T> raw_next;
    PairRho<T> rraw_next;
    V2 rc_next;
    if constexpr (RHO) {   // the wall replacement waits for the next step
      load_pair_rho_raw(rraw_next, f, rt, rc_hi, po, k + 2, q);
      rc_next = load_centre_raw(rt, po.c, k + 3, q);
    } else {
      load_pair(raw_next, f, bx, by, bz, po, k + 2, q);
    }
    __syncthreads();
    // both cells' coefficients on plane k+1: the first colour's now, the second's next step
    Coef<T> red, black_next;
    if constexpr (RHO) {
      Coef<T> ev, od;
      wall_pair_rho(rraw, k + 1, q);
      rc_hi = wall_rho<T>(rc_hi, k + 2, q);
      zlo = pair_coef_rho(rraw, zlo, rc_hi, ev, od);
      red = ODD1 ? od : ev;
      black_next = ODD1 ? ev : od;
    } else {
      red = cell_of<ODD1>(raw);
      black_next = cell_of<!ODD1>(raw);
    }
    if (k + 1 < n) {                   // first colour on plane k+1, tile and ring
      const int c = ct + ODD1;
      gs<T, W>(L[s1], rt_, c, at<T, W>(L[s0], rt_, c), at<T, W>(L[s2], rt_, c), red, h2, fs);
      if (has_ring) {
        if constexpr (RHO) ring_c = cell_coef_rho(ring_raw, k + 1, q);
        gs<T, W>(L[s1], rr_, rc_, at<T, W>(L[s0], rr_, rc_), at<T, W>(L[s2], rr_, rc_), ring_c, h2, fs);
      }
    }
    // no barrier: the second colour on plane k reads the first colour on plane k+1 only
    // in its own column, which this thread has just updated
    {                                  // second colour on plane k (same column), plane out
      const int c = ct + ODD1;
      gs<T, W>(L[s0], rt_, c, ODD1 ? below1 : below0, at<T, W>(L[s1], rt_, c), get_black(), h2, fs);
      below0 = at<T, W>(L[s0], rt_, ct);
      below1 = at<T, W>(L[s0], rt_, ct + 1);
      char* out = reinterpret_cast<char*>(pout + (static_cast<long long>(k) << (2 * q))) + po.c;
      if constexpr (sizeof(T) == 8) {
        // FP64: a streaming store (the plane out is read by the next pass, not this one);
        // it leaves the cache lines this sweep re-reads in place
        typedef T NV __attribute__((ext_vector_type(2)));
        const NV v = {below0, below1};
        __builtin_nontemporal_store(v, reinterpret_cast<NV*>(out));
      } else {
        *reinterpret_cast<V2*>(out) = V2{below0, below1};
      }
    }
    put_black(black_next);
    if constexpr (RHO) {
      rraw = rraw_next;   // plane k+2, replaced at the start of the next step
      rc_hi = rc_next;    // plane k+3
    } else {
      raw = raw_next;
    }
  };
  // The colour of a thread's first cell alternates from plane to plane and is uniform
  // per wave.  FP32: two steps per iteration, in one of two loops chosen once (kc is
  // even), so each loop body is straight-line code whose memory waits the compiler counts
  // exactly.  FP64 keeps one step per iteration: two would exceed the register budget
  // of 1024-thread workgroups and spill.
  if constexpr (sizeof(T) == 8) {
    for (int k = k0; k < k1; ++k) {
      if (first_odd(k + 1))
        step(k, std::true_type{});
      else
        step(k, std::false_type{});
    }
  } else if (first_odd(k0 + 1)) {
    for (int k = k0; k < k1; k += 2) {
      step(k, std::true_type{});
      step(k + 1, std::false_type{});
    }
  } else {
    for (int k = k0; k < k1; k += 2) {
      step(k, std::false_type{});
      step(k + 1, std::true_type{});
    }
  }
}

template <typename T, int TX, int TY, bool ZIN>
hipError_t launch_tx(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, const T* rt, int q,
                     double h, int order, const double* fshift, hipStream_t s) {
  const int n = 1 << q;
  constexpr int threads = TX / 2 * TY;
  const long long tiles = static_cast<long long>(n / TX) * (n / TY);
  // z-chunk: as long as possible while every compute unit still gets `want`
  // workgroups at once: 256 compute units x one workgroup of 1024 threads, or of
  // smaller ones as many as fit (FP64 fits half as many as FP32).  Each chunk pays a
  // prologue of two extra planes and a full load latency before its march settles
  // (about 17 us per chunk, from 32-plane against whole-column chunks at 512^3), so
  // on 512^3 and 1024^3 grids a chunk spans the whole z column.
  const long long want = 256LL * std::max(1, 1024 / threads / (sizeof(T) == 8 ? 2 : 1));
  int kc = n;
  while (kc > 4 && tiles * (n / kc) < want) kc /= 2;
  if (kc > n) kc = n;
  const long long blocks = tiles * (n / kc);
  const T h2 = static_cast<T>(h * h);
  const int first = order == 0 ? 0 : 1;   // pre-smoothing: red first; post-smoothing: black first
  const dim3 grid(static_cast<unsigned>(blocks));
  if (rt) {
    hipLaunchKernelGGL((k_rbgs_fused<T, TX, TY, true, ZIN>), grid, dim3(threads), 0, s, pin, pout, f, bx, by, bz, rt, q, kc,
                       h2, first, fshift);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_rbgs_fused<T, TX, TY, false, ZIN>), grid, dim3(threads), 0, s, pin, pout, f, bx, by, bz, rt, q, kc, h2,
                     first, fshift);
  return hipGetLastError();
}

}  // namespace

// (a 32^3 grid is faster with two half-sweeps: the one-pass sweep's prologue dominates)
int fused_sweep_supported(int q) { return (1 << q) >= 64; }

template <typename T, bool ZIN>
hipError_t launch_shape(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, const T* rt, int q,
                        double h, int order, const double* fshift, hipStream_t s) {
  const int n = 1 << q;
  if (n == 64) return launch_tx<T, 64, 8, ZIN>(pin, pout, f, bx, by, bz, rt, q, h, order, fshift, s);
  if (n == 128) return launch_tx<T, 128, 8, ZIN>(pin, pout, f, bx, by, bz, rt, q, h, order, fshift, s);
  return launch_tx<T, 128, 16, ZIN>(pin, pout, f, bx, by, bz, rt, q, h, order, fshift, s);
}

template <typename T>
hipError_t launch_rbgs_fused(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, const T* rt,
                             int q, double h, int order, const double* fshift, int zero_in, hipStream_t s) {
  if ((1 << q) < 64) return hipErrorInvalidValue;
  return zero_in ? launch_shape<T, true>(pin, pout, f, bx, by, bz, rt, q, h, order, fshift, s)
                 : launch_shape<T, false>(pin, pout, f, bx, by, bz, rt, q, h, order, fshift, s);
}

template hipError_t launch_rbgs_fused<double>(const double*, double*, const double*, const double*, const double*,
                                              const double*, const double*, int, double, int, const double*, int,
                                              hipStream_t);
template hipError_t launch_rbgs_fused<float>(const float*, float*, const float*, const float*, const float*,
                                             const float*, const float*, int, double, int, const double*, int,
                                             hipStream_t);

}  // namespace mg
