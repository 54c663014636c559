// Two red-black Gauss-Seidel sweeps in a single pass over memory (CDNA4, density form:
// the finest grid of a hierarchy built from rho, FP64 cycles and the FP32 cycles of a
// mixed-precision solve).
//
// A V(2,2) cycle smooths twice in a row before the restriction and twice after the
// prolongation.  The one-pass sweep (mg_fused.hip) reads p, f and the density once per
// sweep; this kernel does both sweeps of a pair in one march up z, so they are read once
// for the two.  Call the four half-sweeps A1, B1, A2, B2 (A the colour that goes first).
// At step k a workgroup does A1 on plane k+3, B1 on plane k+2, A2 on plane k+1 and B2 on
// plane k, and writes plane k out.  Each half-sweep needs the one before it on the planes
// either side (B1 on k+2 reads A1 on k+1..k+3, A2 on k+1 reads B1 on k..k+2, B2 on k reads
// A2 on k-1..k+1), and each reads the other colour on its own plane as the step before
// left it, so this order gives exactly the four half-sweeps one after another.
//
// Tiles of 128 x 16 cells (FP32) or 32 x 32 (FP64).  Neighbouring workgroups update the
// same halo cells, so every half-sweep is also computed on a ring around the tile, from
// values the workgroup has itself: A1 on a ring 3 cells wide, B1 on 2, A2 on 1, B2 on the
// tile.  Planes of p and of the density (rho on active cells, +inf elsewhere and beyond
// the z walls) are staged in LDS with a 4-cell halo (136 x 24 or 40 x 40 cells), six
// planes at a time: k..k+4 are read in step k, and the sixth slot takes plane k+5 while a
// slower wave is still in step k.  No thread reads plane k-1 from LDS in step k: the one
// value B2 needs from it (the cell below) the thread computed itself two steps earlier
// and keeps.
//
// Work is given out by column: a thread owns one x-pair of the tile and up to one x-pair
// of the ring, and at step k does all four updates in the one column of each pair whose
// cell on plane k+3 has colour A (the colours alternate with z, so the four planes' cells
// in that column are A, B, A, B).  Everything one update needs from the planes below and
// above is then in its own column: only the in-plane neighbours come from other threads,
// and those were written in an earlier step, before its barrier.  One barrier per step.
//
// A z-chunk [k0, k0 + kc) is entered six steps early: A1 from plane k0-3, B1 from k0-2,
// A2 from k0-1, B2 from k0 (all within the grid), recomputing what the chunk below
// computes on those planes from the same inputs, so chunks need no communication.
// The arithmetic of every update (the faces face_beta(rt_L, rt_R), their sum, the fused
// multiply-adds in a fixed order and the quotient) is that of the one-pass sweep, so two
// sweeps of either kernel give the same bits.
//
// In FP64 flexible CG the two passes of the preconditioner's finest grid also take two
// of the outer iteration's vector passes, reading w = A d as they go: the first
// (pre-smoothing from zero, f = r) forms the residual update r - alpha w where it reads
// f, sweeps with it, writes it out of place and sums its squares; the last
// (post-smoothing, writing z) sums z.w.  Each sum is one partial per workgroup.
#include <type_traits>

#include "mg_buffer.h"
#include "mg_kernels.h"
#include "mg_plan.h"

namespace mg {

namespace {

using buf::ld2;
using buf::off_of;
using buf::plane_rsrc;
using buf::Rsrc;

// Tile of a precision: FP32 128 x 16 (1024 threads, a wave per tile row); FP64 32 x 32
// (512 threads, a wave per four tile rows), whose six staged planes of p and the density
// with a 4-cell halo (40 x 40 cells, 154 KB) fit the 160 KB of LDS a workgroup has, with
// the same ring cells per tile cell as the FP32 tile.
template <typename T>
struct Shape;
template <>
struct Shape<float> {
  static constexpr int TX = 128, TY = 16;
};
template <>
struct Shape<double> {
  static constexpr int TX = 32, TY = 32;
};

constexpr int kSlots = 6;

// ring distance of box cell (r, c): 0 on the tile, up to 4 on the box edge
template <int TX, int TY>
__device__ __forceinline__ int ring_of(int r, int c) {
  const int dy = max(max(4 - r, r - (TY + 3)), 0);
  const int dx = max(max(4 - c, c - (TX + 3)), 0);
  return max(dx, dy);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// W (FP64, flexible CG): the pass also reads w = A d and sums per workgroup, into
// x.partials[blockIdx.x].  Post-smoothing of the preconditioner (not ZIN): the sum of
// pout * w over the tile.  Its first pre-smoothing (ZIN, f = r): the residual update
// r - alpha w (alpha = d.r / d.w) is formed where f is read and swept with, written to
// x.rnew on the tile, and the sum is that of its squares.
template <typename T, bool ZIN, bool W>
__global__ __launch_bounds__(Shape<T>::TX / 2 * Shape<T>::TY) void k_rbgs_fused2(
    const T* __restrict__ pin, T* __restrict__ pout, const T* __restrict__ f, const T* __restrict__ rt, int q, int kc,
    T h2, int first, const double* __restrict__ fshift, Fused2Extra x) {
  constexpr bool ZW = W && !ZIN, RU = W && ZIN;
  const double* __restrict__ w = x.w;
  using V2 = typename buf::Vec2<T>::type;
  constexpr int kTX = Shape<T>::TX, kTY = Shape<T>::TY;
  constexpr int kNT = kTX / 2 * kTY;          // one thread per tile x-pair
  constexpr int kH = kTY + 8, kW = kTX + 8;   // staged box: ring 4
  constexpr int kWP = kW / 2;                 // x-pairs per box row
  constexpr int kBoxPairs = kH * kWP;
  constexpr int kPer = (kBoxPairs + kNT - 1) / kNT;   // staged pairs per thread
  // ring pairs: box rows 1..3 and kTY+4..kTY+6 whole, the tile rows at pairs 0, 1, kWP-2, kWP-1
  constexpr int kRingPairs = 6 * kWP + kTY * 4;
  static_assert(kRingPairs <= kNT, "one ring pair per thread at most");
  __shared__ T P[kSlots][kH][2][kWP];
  __shared__ T R[kSlots][kH][2][kWP];
  const int n = 1 << q;
  const int tid = threadIdx.x;
  const int G = gridDim.x, bid = blockIdx.x;
  const int lid = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;   // neighbours on one XCD
  const int ntx = n / kTX, nty = n / kTY;
  const int i0 = (lid % ntx) * kTX;
  const int j0 = ((lid / ntx) % nty) * kTY;
  const int k0 = (lid / (ntx * nty)) * kc;
  const int k1 = k0 + kc;
  const T fs = fshift ? static_cast<T>(*fshift) : T(0);
  const T inf = __builtin_huge_val();

  // ---- LDS addressing.  Box cell (r, c) of slot s is element ((s kH + r) 2 + (c & 1)) kWP
  // + (c >> 1) of P and of R.  Slots go round with the plane's distance from the chunk's
  // first step ks, and the march is unrolled by the six slots, so every slot is known at
  // compile time: an access is an offset the thread computed once plus an immediate.
  constexpr int kRow = 2 * kWP;      // floats per box row
  constexpr int kSlot = kH * kRow;   // floats per slot
  T* const Pf = &P[0][0][0][0];
  T* const Rf = &R[0][0][0][0];
  using std::integral_constant;

  // ---- staging: box pair e = tid + u * kNT of each plane, global -> registers -> LDS
  unsigned so[kPer];
  int sl[kPer];   // LDS offset of the pair's even column in a slot (-1: none)
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = tid + u * kNT;
    const int r = e / kWP, x = e % kWP;
    sl[u] = e < kBoxPairs ? r * kRow + x : -1;
    so[u] = e < kBoxPairs ? off_of<T>(i0 - 4 + 2 * x, j0 - 4 + r, q) : 0u;
  }
  V2 pn[kPer], rn[kPer];
  auto fetch = [&](int kk) {   // a plane outside the grid reads 0
    const Rsrc pk = plane_rsrc(pin, kk, q), rk = plane_rsrc(rt, kk, q);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      pn[u] = ZIN ? V2{T(0), T(0)} : ld2(pk, so[u], T(0));
      rn[u] = ld2(rk, so[u], T(0));
    }
  };
  // plane kk into slot S; densities beyond a z wall are +inf, replaced here (not at the load)
  auto store = [&](int kk, auto s_tag) {
    constexpr int S = decltype(s_tag)::value * kSlot;
    if (kk >= 0 && kk < n) {   // the same for the whole workgroup: a branch, not selects
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        if (sl[u] >= 0) {
          Pf[S + sl[u]] = pn[u].x;
          Pf[S + sl[u] + kWP] = pn[u].y;
          Rf[S + sl[u]] = rn[u].x;
          Rf[S + sl[u] + kWP] = rn[u].y;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        if (sl[u] >= 0) {
          Pf[S + sl[u]] = pn[u].x;
          Pf[S + sl[u] + kWP] = pn[u].y;
          Rf[S + sl[u]] = inf;
          Rf[S + sl[u] + kWP] = inf;
        }
      }
    }
  };

  // A cell of the box in a slot: its own offset and that of its left neighbour (the
  // right one is the next element after the left one in either column parity).
  struct Cell {
    int own, left;
  };
  // column c = 2 x + o of box row r
  auto cell_of = [&](int r, int x, int o) {
    return o ? Cell{r * kRow + kWP + x, r * kRow + x} : Cell{r * kRow + x, r * kRow + kWP + x - 1};
  };

  // ---- the pairs this thread owns: one of the tile (wave = tile row), one of the ring.
  // Both work in the column of the pair whose cell on plane k+3 has colour A; with ks
  // even that is column (first + j + 1 + (k - ks)) & 1 of the pair, so there are two
  // cases, by the parity of k - ks.
  const int tr = tid / (kTX / 2) + 4;              // box row of the tile pair
  const int tcp = tid % (kTX / 2) + 2;             // box pair index (columns 2 tcp, 2 tcp + 1)
  const int tj = j0 + tr - 4;                      // its global row (no wrap: inside the tile)
  const unsigned tf_off = off_of<T>(i0 + 2 * (tcp - 2), tj, q);
  const int out_off = tr * kRow + tcp;             // the pair's even column
  const bool todd[2] = {((first + tj + 1) & 1) != 0, ((first + tj) & 1) != 0};
  const Cell tcell[2] = {cell_of(tr, tcp, todd[0]), cell_of(tr, tcp, todd[1])};
  const bool has_ring = tid < kRingPairs;
  int gr = 0, gcp = 0;
  if (tid < 6 * kWP) {
    const int row = tid / kWP;
    gr = row < 3 ? 1 + row : kTY + 1 + row;        // rows 1, 2, 3, 20, 21, 22
    gcp = tid % kWP;
  } else {
    const int e = tid - 6 * kWP;
    gr = 4 + e / 4;
    const int w = e % 4;
    gcp = w < 2 ? w : kWP - 4 + w;                 // pairs 0, 1, 66, 67
  }
  const int gj = j0 - 4 + gr;
  const unsigned gf_off = has_ring ? off_of<T>(i0 - 4 + 2 * gcp, gj, q) : 0u;
  const bool godd[2] = {((first + gj + 1) & 1) != 0, ((first + gj) & 1) != 0};
  const Cell gcell[2] = {cell_of(gr, gcp, godd[0]), cell_of(gr, gcp, godd[1])};
  const int gd[2] = {ring_of<kTX, kTY>(gr, 2 * gcp + godd[0]), ring_of<kTX, kTY>(gr, 2 * gcp + godd[1])};

  // f of the owned pairs, plane kk at index (kk - ks) mod 6 (planes k .. k+3 in use at
  // step k, k+4 arriving)
  V2 tfw[kSlots], gfw[kSlots];
  auto load_f = [&](int kk, V2& t, V2& g) {
    const Rsrc fk = plane_rsrc(f, kk, q);
    t = ld2(fk, tf_off, T(0));
    g = has_ring ? ld2(fk, gf_off, T(0)) : V2{T(0), T(0)};
  };

  // The six faces of a cell on the plane of slot S (the density below comes in as lo_r,
  // the one above from slot SA), and the Gauss-Seidel update of that cell from them.
  // The second sweep's update of a cell comes two steps after the first one's, in the
  // same column, on the same faces: they are kept in registers for it.
  struct Faces {
    T xm, xp, ym, yp, zm, zp;
  };
  auto faces = [&](auto s_tag, auto sa_tag, const Cell& x, T lo_r) {
    constexpr int S = decltype(s_tag)::value * kSlot, SA = decltype(sa_tag)::value * kSlot;
    const T rc = Rf[S + x.own];
    return Faces{face_beta(Rf[S + x.left], rc), face_beta(rc, Rf[S + x.left + 1]),
                 face_beta(Rf[S + x.own - kRow], rc), face_beta(rc, Rf[S + x.own + kRow]),
                 face_beta(lo_r, rc), face_beta(rc, Rf[SA + x.own])};
  };
  // The B1 update's z faces are those of A1 in the same column: on the plane above in
  // this step (its face below) and on the plane below two steps earlier (its face
  // above), formed from the same densities in the same order.  A1's faces are formed
  // whenever its column is worked on, also where its update is out of bounds (planes
  // beyond a wall hold +inf densities, which give faces of 0), so both are there
  // whenever B1 runs.
  auto faces_b1 = [&](auto s_tag, const Cell& x, T zm, T zp) {
    constexpr int S = decltype(s_tag)::value * kSlot;
    const T rc = Rf[S + x.own];
    return Faces{face_beta(Rf[S + x.left], rc), face_beta(rc, Rf[S + x.left + 1]),
                 face_beta(Rf[S + x.own - kRow], rc), face_beta(rc, Rf[S + x.own + kRow]), zm, zp};
  };
  // FP64 (registers to spare): the x face between a pair's two cells on a plane is formed
  // by the A1 update of one column and needed again by the B1 update of the other column
  // on the same plane a step later, so it is kept for it (one face fewer per step).
  constexpr bool kXKeep = sizeof(T) == 8;
  auto faces_b1x = [&](auto s_tag, const Cell& x, T zm, T zp, T xpair, bool odd) {
    constexpr int S = decltype(s_tag)::value * kSlot;
    const T rc = Rf[S + x.own];
    const T xo = face_beta(rc, Rf[S + (odd ? x.left + 1 : x.left)]);   // the face away from the partner
    return Faces{odd ? xpair : xo, odd ? xo : xpair, face_beta(Rf[S + x.own - kRow], rc),
                 face_beta(rc, Rf[S + x.own + kRow]), zm, zp};
  };
  auto gs = [&](auto s_tag, auto sa_tag, const Cell& x, const Faces& F, T lo_p, T fv) {
    constexpr int S = decltype(s_tag)::value * kSlot, SA = decltype(sa_tag)::value * kSlot;
    const T D = F.xm + F.xp + F.ym + F.yp + F.zm + F.zp;
    if (D > T(0)) {
      const T Sv = fma_t(F.zp, Pf[SA + x.own], fma_t(F.zm, lo_p, fma_t(F.yp, Pf[S + x.own + kRow],
                   fma_t(F.ym, Pf[S + x.own - kRow], fma_t(F.xp, Pf[S + x.left + 1], F.xm * Pf[S + x.left])))));
      Pf[S + x.own] = gs_quotient(fma_t(-h2, fv - fs, Sv), D);
    }
  };

  // lower bounds of the four half-sweeps in this chunk
  const int lo_a1 = max(k0 - 3, 0), lo_b1 = max(k0 - 2, 0), lo_a2 = max(k0 - 1, 0);
  // per parity of the step: the tile column's cell on plane k-1 (value after A2) for B2
  // on plane k, and the faces of the A1 and B1 updates for A2 and B2 two steps on
  // (tile), and of the ring's A1 for its A2
  T below_p[2] = {T(0), T(0)};
  double zw = 0.0;   // ZW: this thread's sum of pout * w; RU: of r_new^2 on its tile pair
  // RU: alpha, and w of the owned pairs on the plane whose f came in the step before
  const double alpha = RU ? *x.s_dr / *x.s_dw : 0.0;
  if (RU && blockIdx.x == 0 && tid == 0) *x.s_alpha = alpha;
  V2 wt{T(0), T(0)}, wg{T(0), T(0)};
  auto load_w = [&](int kk) {
    if constexpr (RU) {
      const Rsrc wk = plane_rsrc(w, kk, q);
      wt = ld2(wk, tf_off, T(0));
      wg = has_ring ? ld2(wk, gf_off, T(0)) : V2{T(0), T(0)};
    }
  };
  // RU: f of plane kk (in t, g) becomes r - alpha w (w in wt, wg); on the tile's own
  // planes it is written out and its squares summed
  auto update_r = [&](int kk, V2& t, V2& g) {
    if constexpr (RU) {
      t = V2{__builtin_fma(-alpha, wt.x, t.x), __builtin_fma(-alpha, wt.y, t.y)};
      g = V2{__builtin_fma(-alpha, wg.x, g.x), __builtin_fma(-alpha, wg.y, g.y)};
      if (kk >= k0 && kk < k1 && kk < n) {
        *reinterpret_cast<V2*>(reinterpret_cast<char*>(x.rnew + (static_cast<long long>(kk) << (2 * q))) + tf_off) = t;
        zw = __builtin_fma(t.y, t.y, __builtin_fma(t.x, t.x, zw));
      }
    }
  };
  Faces ta[2], tb[2], ga[2];
  T xt = T(0), xg = T(0);   // the pair's x face kept from the step before (tile, ring)

  // ---- prologue: planes ks .. ks+3 staged (slots 0..3), ks+4 in registers, f of ks .. ks+3
  const int ks = k0 - 6;   // even: chunks start at multiples of kc >= 8
  fetch(ks);
  store(ks, integral_constant<int, 0>{});
  fetch(ks + 1);
  store(ks + 1, integral_constant<int, 1>{});
  fetch(ks + 2);
  store(ks + 2, integral_constant<int, 2>{});
  fetch(ks + 3);
  store(ks + 3, integral_constant<int, 3>{});
  fetch(ks + 4);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    load_f(ks + d, tfw[d], gfw[d]);
    if constexpr (RU) {   // planes below the chunk: converted, not written; ks+3 in the first step
      load_w(ks + d);
      if (d < 3) update_r(ks + d, tfw[d], gfw[d]);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // one step; U = (k - ks) mod 6 at compile time, so slots and kept registers are named
  auto step = [&](int k, auto u_tag) {
    constexpr int U = decltype(u_tag)::value;
    constexpr int PAR = U & 1;   // parity of k - ks
    using S0 = integral_constant<int, U % kSlots>;   // slot (and f index) of plane k
    using S1 = integral_constant<int, (U + 1) % kSlots>;
    using S2 = integral_constant<int, (U + 2) % kSlots>;
    using S3 = integral_constant<int, (U + 3) % kSlots>;
    using S4 = integral_constant<int, (U + 4) % kSlots>;
    store(k + 4, S4{});
    fetch(k + 5);
    if constexpr (RU) update_r(k + 3, tfw[S3::value], gfw[S3::value]);   // f and w came last step
    load_f(k + 4, tfw[S4::value], gfw[S4::value]);
    if constexpr (RU) load_w(k + 4);
    V2 wk{T(0), T(0)};   // ZW: w of the tile pair on plane k, read while the step runs
    if constexpr (ZW) wk = ld2(plane_rsrc(w, k, q), tf_off, 0.0);
    __syncthreads();
    const int ka = k + 3, kb = k + 2, kA = k + 1;
    {
      const Cell c = tcell[PAR];
      const bool odd = todd[PAR];
      const Faces a2f = ta[PAR], b2f = tb[PAR];   // from step k-2, before this step's A1, B1
      ta[PAR] = faces(S3{}, S4{}, c, Rf[S2::value * kSlot + c.own]);
      const T xprev = xt;
      if constexpr (kXKeep) xt = odd ? ta[PAR].xm : ta[PAR].xp;
      if (ka >= lo_a1 && ka < n)
        gs(S3{}, S4{}, c, ta[PAR], Pf[S2::value * kSlot + c.own], odd ? tfw[S3::value].y : tfw[S3::value].x);
      if (kb >= lo_b1 && kb < n) {
        if constexpr (kXKeep) tb[PAR] = faces_b1x(S2{}, c, a2f.zp, ta[PAR].zm, xprev, odd);
        else tb[PAR] = faces_b1(S2{}, c, a2f.zp, ta[PAR].zm);
        gs(S2{}, S3{}, c, tb[PAR], Pf[S1::value * kSlot + c.own], odd ? tfw[S2::value].y : tfw[S2::value].x);
      }
      if (kA >= lo_a2 && kA < n)
        gs(S1{}, S2{}, c, a2f, Pf[S0::value * kSlot + c.own], odd ? tfw[S1::value].y : tfw[S1::value].x);
      if (k >= k0 && k < n) {
        gs(S0{}, S1{}, c, b2f, below_p[PAR], odd ? tfw[S0::value].y : tfw[S0::value].x);
        // plane k is final in both columns of the pair (the other one since A2 at step k-1)
        const T v0 = Pf[S0::value * kSlot + out_off], v1 = Pf[S0::value * kSlot + out_off + kWP];
        *reinterpret_cast<V2*>(reinterpret_cast<char*>(pout + (static_cast<long long>(k) << (2 * q))) + tf_off) =
            V2{v0, v1};
        if constexpr (ZW) zw = __builtin_fma(v1, wk.y, __builtin_fma(v0, wk.x, zw));
      }
      // this column's cell on plane k+1 is used by B2 on plane k+2, two steps on
      below_p[PAR] = Pf[S1::value * kSlot + c.own];
    }
    // the ring pair: as far as its ring distance allows (per lane)
    if (has_ring) {
      const Cell c = gcell[PAR];
      const bool odd = godd[PAR];
      const int d = gd[PAR];
      const Faces a2f = ga[PAR];
      const T xgprev = xg;
      if (d <= 3) {   // every ring pair's columns are within 3 cells of the tile
        ga[PAR] = faces(S3{}, S4{}, c, Rf[S2::value * kSlot + c.own]);
        if constexpr (kXKeep) xg = odd ? ga[PAR].xm : ga[PAR].xp;
        if (ka >= lo_a1 && ka < n)
          gs(S3{}, S4{}, c, ga[PAR], Pf[S2::value * kSlot + c.own], odd ? gfw[S3::value].y : gfw[S3::value].x);
      }
      if (d <= 2 && kb >= lo_b1 && kb < n) {
        Faces fb;
        if constexpr (kXKeep) fb = faces_b1x(S2{}, c, a2f.zp, ga[PAR].zm, xgprev, odd);
        else fb = faces_b1(S2{}, c, a2f.zp, ga[PAR].zm);
        gs(S2{}, S3{}, c, fb, Pf[S1::value * kSlot + c.own], odd ? gfw[S2::value].y : gfw[S2::value].x);
      }
      if (d <= 1 && kA >= lo_a2 && kA < n)
        gs(S1{}, S2{}, c, a2f, Pf[S0::value * kSlot + c.own], odd ? gfw[S1::value].y : gfw[S1::value].x);
    }
  };
  // kc + 6 steps, an even number, from an even plane; six to a round of the slots
  for (int k = ks; k < k1; k += kSlots) {
    step(k, integral_constant<int, 0>{});
    step(k + 1, integral_constant<int, 1>{});
    if (k + 2 < k1) {
      step(k + 2, integral_constant<int, 2>{});
      step(k + 3, integral_constant<int, 3>{});
    }
    if (k + 4 < k1) {
      step(k + 4, integral_constant<int, 4>{});
      step(k + 5, integral_constant<int, 5>{});
    }
  }
  if constexpr (W) {   // the workgroup's sum: waves in order, through the first LDS words
    for (int off = 32; off > 0; off >>= 1) zw += __shfl_xor(zw, off, 64);
    __syncthreads();   // every wave is past its last read of the staged planes
    double* red = reinterpret_cast<double*>(Pf);
    if ((tid & 63) == 0) red[tid >> 6] = zw;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int v = 0; v < kNT / 64; ++v) s += red[v];
      x.partials[blockIdx.x] = s;
    }
  }
}

}  // namespace

int fused2_supported(int q) { return (1 << q) >= 256; }

template <typename T>
hipError_t launch_rbgs_fused2(const T* pin, T* pout, const T* f, const T* rt, int q, double h, int order,
                              const double* fshift, int zero_in, hipStream_t s, const Fused2Extra* x, int* nblocks) {
  constexpr int TX = Shape<T>::TX, TY = Shape<T>::TY;
  const int n = 1 << q;
  if (!fused2_supported(q) || !rt || pin == pout) return hipErrorInvalidValue;
  const bool wx = x != nullptr && x->w != nullptr;
  if (wx && (sizeof(T) != 8 || !x->partials || !nblocks)) return hipErrorInvalidValue;
  if (wx && zero_in && (!x->rnew || static_cast<const void*>(x->rnew) == static_cast<const void*>(f) || !x->s_dr || !x->s_dw || !x->s_alpha || fshift))
    return hipErrorInvalidValue;
  const long long tiles = static_cast<long long>(n / TX) * (n / TY);
  // z-chunks as long as possible while every compute unit still gets a workgroup
  int kc = n;
  while (kc > 8 && tiles * (n / kc) < 256) kc /= 2;
  const long long blocks = tiles * (n / kc);
  if (wx && blocks > kNumPartials) return hipErrorInvalidValue;
  const T h2 = static_cast<T>(h * h);
  const int first = order == 0 ? 0 : 1;   // pre-smoothing: red first; post-smoothing: black first
  const dim3 grid(static_cast<unsigned>(blocks)), block(TX / 2 * TY);
  const Fused2Extra none{};
  if (wx) {
    if constexpr (sizeof(T) == 8) {
      if (zero_in)
        hipLaunchKernelGGL((k_rbgs_fused2<T, true, true>), grid, block, 0, s, pin, pout, f, rt, q, kc, h2, first,
                           fshift, *x);
      else
        hipLaunchKernelGGL((k_rbgs_fused2<T, false, true>), grid, block, 0, s, pin, pout, f, rt, q, kc, h2, first,
                           fshift, *x);
    }
    *nblocks = static_cast<int>(blocks);
  } else if (zero_in) {
    hipLaunchKernelGGL((k_rbgs_fused2<T, true, false>), grid, block, 0, s, pin, pout, f, rt, q, kc, h2, first, fshift,
                       none);
  } else {
    hipLaunchKernelGGL((k_rbgs_fused2<T, false, false>), grid, block, 0, s, pin, pout, f, rt, q, kc, h2, first,
                       fshift, none);
  }
  return hipGetLastError();
}

template hipError_t launch_rbgs_fused2<float>(const float*, float*, const float*, const float*, int, double, int,
                                              const double*, int, hipStream_t, const Fused2Extra*, int*);
template hipError_t launch_rbgs_fused2<double>(const double*, double*, const double*, const double*, int, double, int,
                                               const double*, int, hipStream_t, const Fused2Extra*, int*);

}  // namespace mg
