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
#include "mg_kernels.h"

#include <type_traits>

namespace mg {

namespace {

__device__ __forceinline__ int cell(int i, int j, int k, int q) { return (((k << q) + j) << q) + i; }

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
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
  Coef<T> C;
  const int n = 1 << q, m = n - 1;
  if (kk < 0 || kk >= n) {
    C.f = C.xm = C.xp = C.ym = C.yp = C.zm = C.zp = T(0);
    return C;
  }
  const int c = cell(i, j, kk, q);
  C.f = f[c];
  C.xm = bx[c];
  C.xp = bx[cell((i + 1) & m, j, kk, q)];
  C.ym = by[c];
  C.yp = by[cell(i, (j + 1) & m, kk, q)];
  C.zm = bz[c];
  C.zp = kk < m ? bz[c + (1 << (2 * q))] : T(0);
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
                                          const T* __restrict__ by, const T* __restrict__ bz, int i, int j, int kk,
                                          int q) {
  using V2 = typename Vec2<T>::type;
  const int n = 1 << q, m = n - 1;
  if (kk < 0 || kk >= n) {
    R.f = R.bx = R.by = R.byu = R.bz = R.bzu = V2{T(0), T(0)};
    R.bxr = T(0);
    return;
  }
  const int c = cell(i, j, kk, q);
  R.f = *reinterpret_cast<const V2*>(f + c);
  R.bx = *reinterpret_cast<const V2*>(bx + c);
  R.bxr = bx[cell((i + 2) & m, j, kk, q)];
  R.by = *reinterpret_cast<const V2*>(by + c);
  R.byu = *reinterpret_cast<const V2*>(by + cell(i, (j + 1) & m, kk, q));
  R.bz = *reinterpret_cast<const V2*>(bz + c);
  R.bzu = kk < m ? *reinterpret_cast<const V2*>(bz + c + (1 << (2 * q))) : V2{T(0), T(0)};
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
    const T S = C.xm * at<T, W>(cur, r, c - 1) + C.xp * at<T, W>(cur, r, c + 1) + C.ym * at<T, W>(cur, r - 1, c) +
                C.yp * at<T, W>(cur, r + 1, c) + C.zm * lo + C.zp * hi;
    at<T, W>(cur, r, c) = (S - h2 * (C.f - fs)) / D;
  }
}

constexpr int kTY = 8;

// Tiles span TX = min(N, 256) cells in x, so for N <= 256 the x halo wraps onto the
// tile's own cache lines, and TY = 8 rows; one thread per x-pair of tile cells.
template <typename T, int TX>
__global__ __launch_bounds__(TX / 2 * kTY) void k_rbgs_fused(const T* __restrict__ pin, T* __restrict__ pout,
                                                              const T* __restrict__ f, const T* __restrict__ bx,
                                                              const T* __restrict__ by, const T* __restrict__ bz,
                                                              int q, int kc, T h2, int first,
                                                              const double* __restrict__ fshift) {
  using V2 = typename Vec2<T>::type;
  constexpr int TY = kTY;
  constexpr int NT = TX / 2 * TY;
  constexpr int W = TX + 4;                 // columns i0-2 .. i0+TX+1
  constexpr int H = TY + 4;                 // rows    j0-2 .. j0+TY+1
  constexpr int BOX = H * (W / 2);          // pairs per staged plane
  constexpr int PER = (BOX + NT - 1) / NT;  // pairs per thread
  __shared__ T L[4][H][2][W / 2];
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
  const int second = 1 - first;
  const T fs = fshift ? static_cast<T>(*fshift) : T(0);
  // A step branches on the colour parity of the thread's row, and contains barriers:
  // every wave must hold rows of one parity.  With 32 pairs per row a wave spans two
  // rows, so rows are paired as (0,2), (1,3), (4,6), (5,7).
  const int xt = tid % (TX / 2);
  const int half = tid / (TX / 2);
  const int jt = TX >= 128 ? half : ((half & ~3) | ((half & 1) << 1) | ((half >> 1) & 1));
  static_assert(TX >= 64, "a wave must not span rows of both parities");
  const int jrow = j0 + jt;
  const int ipair = i0 + 2 * xt;

  // ---- staged p planes: global -> registers (one plane ahead) -> LDS
  V2 pn[PER];
  auto fetch_plane = [&](int kk) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT;
      if (e < BOX && kk >= 0 && kk < n) {
        const int r = e / (W / 2), cp = e % (W / 2);
        pn[u] = *reinterpret_cast<const V2*>(pin + cell((i0 - 2 + 2 * cp) & m, (j0 - 2 + r) & m, kk, q));
      } else {
        pn[u] = V2{T(0), T(0)};
      }
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
  const int rt = jt + 2, ct = 2 * xt + 2;   // the pair's place in a staged plane

  // ---- prologue.  Plane kk is staged in slot kk & 3; plane k0-2 of the pair in registers.
  auto slot = [](int kk) { return kk & 3; };
  int rr_, rc_, ri_, rj_;
  PairRaw<T> raw;        // both cells' coefficients of the plane above the current one
  Coef<T> black_cur;     // second colour's coefficients on the current plane
  T below0, below1;      // the pair's finished values on the plane under the current one
  {
    const Coef<T> red_m1 = load_cell(f, bx, by, bz, ipair + first_odd(k0 - 1), jrow, k0 - 1, q);
    const Coef<T> red_0 = load_cell(f, bx, by, bz, ipair + first_odd(k0), jrow, k0, q);
    black_cur = load_cell(f, bx, by, bz, ipair + !first_odd(k0), jrow, k0, q);
    Coef<T> ring_0;
    if (has_ring) {
      ring_cell(k0, rr_, rc_, ri_, rj_);
      ring_0 = load_cell(f, bx, by, bz, ri_, rj_, k0, q);
    }
    T pm2_0 = T(0), pm2_1 = T(0);   // the pair on plane k0-2
    if (k0 - 2 >= 0) {
      pm2_0 = pin[cell(ipair, jrow, k0 - 2, q)];
      pm2_1 = pin[cell(ipair + 1, jrow, k0 - 2, q)];
    }
    load_pair(raw, f, bx, by, bz, ipair, jrow, k0 + 1, q);
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
      gs<T, W>(L[sm], rt, ct + o, o ? pm2_1 : pm2_0, at<T, W>(L[s0], rt, ct + o), red_m1, h2, fs);
    }
    below0 = at<T, W>(L[sm], rt, ct);   // own cells: only this thread wrote them
    below1 = at<T, W>(L[sm], rt, ct + 1);
    {
      const int c = ct + first_odd(k0);
      gs<T, W>(L[s0], rt, c, at<T, W>(L[sm], rt, c), at<T, W>(L[s1], rt, c), red_0, h2, fs);
    }
    if (has_ring) {
      ring_cell(k0, rr_, rc_, ri_, rj_);
      gs<T, W>(L[s0], rr_, rc_, at<T, W>(L[sm], rr_, rc_), at<T, W>(L[s1], rr_, rc_), ring_0, h2, fs);
    }
    __syncthreads();
  }

  // One step, for the first colour on plane k+1 sitting in the odd (ODD1) or even cell
  // of the pair; a wave covers part of one tile row, so the choice is uniform per wave
  // whenever a row holds at least 64 pairs.  On entry: plane k (first colour done on
  // tile + ring) in slot k, plane k+1 (old) in slot k+1, pn = plane k+2, raw = the
  // coefficients of plane k+1, black_cur = the second colour's on plane k.  One barrier
  // per step (after staging plane k+2): four slots let the next step stage its plane
  // while a slower wave of this step still reads planes k .. k+2.
  auto step = [&](int k, auto odd_tag) {
    constexpr bool ODD1 = decltype(odd_tag)::value;
    const int s0 = slot(k), s1 = slot(k + 1), s2 = slot(k + 2);
    store_plane(s2);                   // plane k+2
    fetch_plane(k + 3);
    PairRaw<T> raw_next;
    load_pair(raw_next, f, bx, by, bz, ipair, jrow, k + 2, q);
    Coef<T> ring_c;
    if (has_ring) {
      ring_cell(k + 1, rr_, rc_, ri_, rj_);
      ring_c = load_cell(f, bx, by, bz, ri_, rj_, k + 1, q);
    }
    __syncthreads();
    if (k + 1 < n) {                   // first colour on plane k+1, tile and ring
      const int c = ct + ODD1;
      gs<T, W>(L[s1], rt, c, at<T, W>(L[s0], rt, c), at<T, W>(L[s2], rt, c), cell_of<ODD1>(raw), h2, fs);
      if (has_ring) gs<T, W>(L[s1], rr_, rc_, at<T, W>(L[s0], rr_, rc_), at<T, W>(L[s2], rr_, rc_), ring_c, h2, fs);
    }
    // no barrier: the second colour on plane k reads the first colour on plane k+1 only
    // in its own column, which this thread has just updated
    {                                  // second colour on plane k (same column), plane out
      const int c = ct + ODD1;
      gs<T, W>(L[s0], rt, c, ODD1 ? below1 : below0, at<T, W>(L[s1], rt, c), black_cur, h2, fs);
      below0 = at<T, W>(L[s0], rt, ct);
      below1 = at<T, W>(L[s0], rt, ct + 1);
      *reinterpret_cast<V2*>(pout + cell(ipair, jrow, k, q)) = V2{below0, below1};
    }
    black_cur = cell_of<!ODD1>(raw);
    raw = raw_next;
  };
  for (int k = k0; k < k1; ++k) {
    if (first_odd(k + 1))
      step(k, std::true_type{});
    else
      step(k, std::false_type{});
  }
}

template <typename T, int TX>
hipError_t launch_tx(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q, double h,
                     int order, const double* fshift, hipStream_t s) {
  const int n = 1 << q;
  constexpr int threads = TX / 2 * kTY;
  const long long tiles = static_cast<long long>(n / TX) * (n / kTY);
  // z-chunk: as long as possible (overlap planes per chunk) while still giving each
  // compute unit the workgroups it can hold at once (FP64 needs about twice the
  // registers of FP32, so half as many fit)
  const long long want = 256LL * 1024 / threads / (sizeof(T) == 8 ? 2 : 1);
  int kc = 32;
  while (kc > 4 && tiles * (n / kc) < want) kc /= 2;
  if (kc > n) kc = n;
  const long long blocks = tiles * (n / kc);
  const T h2 = static_cast<T>(h * h);
  const int first = order == 0 ? 0 : 1;   // pre-smoothing: red first; post-smoothing: black first
  hipLaunchKernelGGL((k_rbgs_fused<T, TX>), dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, s, pin, pout, f,
                     bx, by, bz, q, kc, h2, first, fshift);
  return hipGetLastError();
}

}  // namespace

int fused_sweep_supported(int q) { return (1 << q) >= 64; }

template <typename T>
hipError_t launch_rbgs_fused(const T* pin, T* pout, const T* f, const T* bx, const T* by, const T* bz, int q,
                             double h, int order, const double* fshift, hipStream_t s) {
  const int n = 1 << q;
  if (n < 64) return hipErrorInvalidValue;
  if (n == 64) return launch_tx<T, 64>(pin, pout, f, bx, by, bz, q, h, order, fshift, s);
  if (n == 128) return launch_tx<T, 128>(pin, pout, f, bx, by, bz, q, h, order, fshift, s);
  return launch_tx<T, 256>(pin, pout, f, bx, by, bz, q, h, order, fshift, s);
}

template hipError_t launch_rbgs_fused<double>(const double*, double*, const double*, const double*, const double*,
                                              const double*, int, double, int, const double*, hipStream_t);
template hipError_t launch_rbgs_fused<float>(const float*, float*, const float*, const float*, const float*,
                                             const float*, int, double, int, const double*, hipStream_t);

}  // namespace mg
