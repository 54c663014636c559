// Residual passes that march up z (CDNA4; FP64, and FP32 for the restriction).
//
// r = (f - fshift) - h^-2 sum_f beta_f (p_nb - p_c) on active cells (D = sum beta > 0),
// 0 elsewhere.  Each thread owns an x-pair (i even, i+1) in two rows (2J, 2J+1) of a
// TX x TY tile and walks up a chunk of planes.  The pair's p (and the coefficients it
// needs from the planes below and above) stay in registers from one plane to the next,
// so each plane of p and of the coefficients is read from memory once per column; the
// rows just below and above the thread's two rows and the x neighbours come from the
// caches (neighbouring threads load them as their own).  All loads address one plane
// through a buffer descriptor (mg_buffer.h).  Modes:
//   NORM      partial sums of r^2 per workgroup; optionally r32 = float(r), e32 = 0,
//             r64 = r, z64 = 0 (each output may be null)
//   RESTRICT  fc = mean of r over the 8 children of each coarse cell (the pair's two
//             cells on two rows and two planes), ec = 0
//   AW        w = A d (flexible CG) with partial sums of d.w and d.r
//   FCGX      the flexible-CG direction and product in one pass: d = z + beta d_old
//             (z in FP64 or FP32; d = z on the first step), w = A d, partial sums of
//             d.w and d.r, and the previous step's p += alpha d_old, deferred to this
//             pass (d_old, z are read at every point of the stencil; d goes to a
//             second buffer, since neighbouring threads still read d_old)
// Coefficients come from the face arrays, or (RHO) from the density form rt: each
// face is face_beta(rt_L, rt_R), formed once per plane and thread (the faces to the
// plane below are carried from the previous plane).  Sums are explicit fused
// multiply-adds in the same order as every other residual in the library, so the two
// forms give identical bits.
#include "mg_buffer.h"
#include "mg_kernels.h"
#include "mg_plan.h"

namespace mg {

namespace {

using buf::ld1;
using buf::ld2;
using buf::off_of;
using buf::plane_rsrc;
using buf::Rsrc;
using buf::Vec2;

constexpr int kMarchThreads = 256;
enum { kModeNorm = 0, kModeRestrict = 1, kModeAw = 2, kModeNormUpdate = 3, kModeFcgX = 4 };

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// T = float only in RESTRICT mode (the finest grid of an FP32 cycle)
template <typename T>
struct MarchArgs {
  const T* p;         // p, or d in AW mode
  const T* f;         // NORM / RESTRICT
  const T* bx;
  const T* by;
  const T* bz;
  const T* rt;
  const double* fshift;
  int q, kc;
  T inv_h2;
  // NORM
  float* r32;
  float* e32;
  double* r64;
  double* z64;
  double* partials;   // NORM: r^2; AW: d.w
  // RESTRICT
  T* fc;
  T* ec;
  // AW
  const double* r;
  double* w;
  double* partials2;  // AW: d.r
  // NORM with update: the residual of p + e (e in FP32, added on active cells), and
  // p + e written to pout
  const float* eu;
  double* pout;
  // FCGX (p = d_old): z (one of the two), beta = -s_zw / s_dw (none on the first step:
  // d = z), the new direction dn, and p += s_alpha d_old on pp (none on the first step)
  const double* zx64;
  const float* zx32;
  const double* s_zw;
  const double* s_dw;
  const double* s_alpha;
  double* dn;
  double* pp;
  // FCGX through LDS, p's update every second step: p += *s_alpha_prev dprev first (the
  // update the step before left), and *s_alpha saved to s_alpha_save (a step that leaves it)
  const double* dprev;
  const double* s_alpha_prev;
  double* s_alpha_save;
};

// The six faces of the two cells of an x-pair
template <typename T>
struct PF {
  T x0, x1, x2, ym0, ym1, yp0, yp1, zm0, zm1, zp0, zp1;
};

// r of the two cells of a pair from p at the cell, its x neighbours (pl, pr), the pair
// in the rows below / above and the planes below / above
template <typename T, typename V2 = typename Vec2<T>::type>
__device__ __forceinline__ void pair_r(const PF<T>& F, V2 pc, T pl, T pr, V2 pyd, V2 pyu, V2 pzd, V2 pzu, V2 fv, T fs,
                                       T inv_h2, T& r0, T& r1) {
  const T D0 = F.x0 + F.x1 + F.ym0 + F.yp0 + F.zm0 + F.zp0;
  const T D1 = F.x1 + F.x2 + F.ym1 + F.yp1 + F.zm1 + F.zp1;
  const T s0 = fmad(F.zp0, pzu.x - pc.x, fmad(F.zm0, pzd.x - pc.x, fmad(F.yp0, pyu.x - pc.x,
                    fmad(F.ym0, pyd.x - pc.x, fmad(F.x1, pc.y - pc.x, F.x0 * (pl - pc.x))))));
  const T s1 = fmad(F.zp1, pzu.y - pc.y, fmad(F.zm1, pzd.y - pc.y, fmad(F.yp1, pyu.y - pc.y,
                    fmad(F.ym1, pyd.y - pc.y, fmad(F.x2, pr - pc.y, F.x1 * (pc.x - pc.y))))));
  r0 = D0 > T(0) ? fmad(-inv_h2, s0, fv.x - fs) : T(0);
  r1 = D1 > T(0) ? fmad(-inv_h2, s1, fv.y - fs) : T(0);
}

// a 16-byte store that does not keep its lines in the caches
__device__ __forceinline__ void stream_store(double* dst, double2 v) {
  typedef double NV __attribute__((ext_vector_type(2)));
  const NV x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<NV*>(dst));
}

// p + e on active cells (density finite); the update of a mixed-precision refinement step
__device__ __forceinline__ double add_active(double p, float e, double rt) {
  return rt < __builtin_huge_val() ? p + static_cast<double>(e) : p;
}
__device__ __forceinline__ double2 add_active(double2 p, float2 e, double2 rt) {
  return double2{add_active(p.x, e.x, rt.x), add_active(p.y, e.y, rt.y)};
}

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kMarchThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kMarchThreads / 64; ++w) s += red[w];
  return s;   // valid in thread 0
}

template <typename T, bool RHO, int MODE, int TX>
__global__ __launch_bounds__(kMarchThreads) void k_residual_march(MarchArgs<T> a) {
  using V2 = typename Vec2<T>::type;
  static_assert(sizeof(T) == 8 || MODE == kModeRestrict, "FP32 marches restrict only");
  constexpr bool UPD = MODE == kModeNormUpdate;
  constexpr bool NORM = MODE == kModeNorm || UPD;
  constexpr bool FX = MODE == kModeFcgX;
  constexpr bool PROD = MODE == kModeAw || FX;   // w = A d and the two dot products
  static_assert(!UPD || RHO, "the update mode reads activity from the density form");
  constexpr int PAIRS = TX / 2;                 // x-pairs per tile row
  constexpr int RP = kMarchThreads / PAIRS;     // row pairs per tile
  constexpr int TY = 2 * RP;
  const int q = a.q, n = 1 << q;
  const T inf = __builtin_huge_val();
  const T zero = T(0);
  const int tid = threadIdx.x;
  const int G = gridDim.x, bid = blockIdx.x;
  const int lid = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;   // neighbours on one XCD
  const int ntx = n / TX, nty = n / TY;
  const int i0 = (lid % ntx) * TX;
  const int j0 = ((lid / ntx) % nty) * TY;
  const int k0 = (lid / (ntx * nty)) * a.kc;
  const int ip = i0 + 2 * (tid % PAIRS);
  const int ja = j0 + 2 * (tid / PAIRS), jb = ja + 1;
  const unsigned oa = off_of<T>(ip, ja, q), ob = off_of<T>(ip, jb, q);
  const unsigned od = off_of<T>(ip, ja - 1, q), ou = off_of<T>(ip, jb + 1, q);
  const unsigned ola = off_of<T>(ip - 1, ja, q), ora = off_of<T>(ip + 2, ja, q);
  const unsigned olb = off_of<T>(ip - 1, jb, q), orb = off_of<T>(ip + 2, jb, q);
  const T fs = (!PROD && a.fshift) ? static_cast<T>(*a.fshift) : zero;
  // FCGX: the new direction from z and d_old at one point of the stencil
  const bool fx_first = FX && a.s_zw == nullptr;
  const double fx_beta = (FX && !fx_first) ? -*a.s_zw / *a.s_dw : 0.0;
  auto zload2 = [&](int kk, unsigned off) -> double2 {
    if (a.zx64) return ld2(plane_rsrc(a.zx64, kk, q), off, 0.0);
    const float2 zf = ld2(plane_rsrc(a.zx32, kk, q), off >> 1, 0.0f);
    return double2{static_cast<double>(zf.x), static_cast<double>(zf.y)};
  };
  auto zload1 = [&](int kk, unsigned off) -> double {
    if (a.zx64) return ld1(plane_rsrc(a.zx64, kk, q), off, 0.0);
    return static_cast<double>(ld1(plane_rsrc(a.zx32, kk, q), off >> 1, 0.0f));
  };
  auto dn2 = [&](double2 d, double2 z) -> double2 {
    return fx_first ? z : double2{__builtin_fma(fx_beta, d.x, z.x), __builtin_fma(fx_beta, d.y, z.y)};
  };
  auto dn1 = [&](double d, double z) -> double { return fx_first ? z : __builtin_fma(fx_beta, d, z); };

  // window: the pair's p on the planes below, at and above the current one (rows a, b)
  const Rsrc p_lo = plane_rsrc(a.p, k0 - 1, q), p_c = plane_rsrc(a.p, k0, q);
  V2 pa_lo = ld2(p_lo, oa, zero), pb_lo = ld2(p_lo, ob, zero);
  V2 pa = ld2(p_c, oa, zero), pb = ld2(p_c, ob, zero);
  V2 dca{zero, zero}, dcb{zero, zero};   // FCGX: d_old of the pair on the current plane
  if constexpr (FX) {
    dca = pa;
    dcb = pb;
    pa_lo = dn2(pa_lo, zload2(k0 - 1, oa));
    pb_lo = dn2(pb_lo, zload2(k0 - 1, ob));
    pa = dn2(pa, zload2(k0, oa));
    pb = dn2(pb, zload2(k0, ob));
  }
  // faces to the plane below (carried), and for the density form the pair's density
  V2 za, zb;                 // zm of rows a, b on the current plane
  V2 ra, rb;                 // density form: rt of the pair on the current plane
  if constexpr (RHO) {
    const bool in_lo = k0 >= 1;
    const V2 la = ld2(plane_rsrc(a.rt, k0 - 1, q), oa, zero), lb = ld2(plane_rsrc(a.rt, k0 - 1, q), ob, zero);
    ra = ld2(plane_rsrc(a.rt, k0, q), oa, zero);
    rb = ld2(plane_rsrc(a.rt, k0, q), ob, zero);
    za = in_lo ? V2{face_beta(la.x, ra.x), face_beta(la.y, ra.y)} : V2{zero, zero};
    zb = in_lo ? V2{face_beta(lb.x, rb.x), face_beta(lb.y, rb.y)} : V2{zero, zero};
    if constexpr (UPD) {
      const Rsrc e_lo = plane_rsrc(a.eu, k0 - 1, q), e_c = plane_rsrc(a.eu, k0, q);
      pa_lo = add_active(pa_lo, ld2(e_lo, oa >> 1, 0.0f), la);
      pb_lo = add_active(pb_lo, ld2(e_lo, ob >> 1, 0.0f), lb);
      pa = add_active(pa, ld2(e_c, oa >> 1, 0.0f), ra);
      pb = add_active(pb, ld2(e_c, ob >> 1, 0.0f), rb);
    }
  } else {
    const Rsrc zk = plane_rsrc(a.bz, k0, q);
    za = ld2(zk, oa, zero);   // 0 on the bottom wall (stored) and below the grid
    zb = ld2(zk, ob, zero);
  }
  double acc = 0.0, acc2 = 0.0;
  T csum = zero;
  for (int k = k0; k < k0 + a.kc; ++k) {
    const Rsrc pk = plane_rsrc(a.p, k, q), pu = plane_rsrc(a.p, k + 1, q);
    V2 pa_hi = ld2(pu, oa, zero), pb_hi = ld2(pu, ob, zero);   // 0 above the grid
    V2 pd = ld2(pk, od, zero), pup = ld2(pk, ou, zero);
    T pla = ld1(pk, ola, zero), pra = ld1(pk, ora, zero);
    T plb = ld1(pk, olb, zero), prb = ld1(pk, orb, zero);
    V2 dha{zero, zero}, dhb{zero, zero};   // FCGX: d_old of the pair on the plane above
    if constexpr (FX) {
      dha = pa_hi;
      dhb = pb_hi;
      pa_hi = dn2(pa_hi, zload2(k + 1, oa));
      pb_hi = dn2(pb_hi, zload2(k + 1, ob));
      pd = dn2(pd, zload2(k, od));
      pup = dn2(pup, zload2(k, ou));
      pla = dn1(pla, zload1(k, ola));
      pra = dn1(pra, zload1(k, ora));
      plb = dn1(plb, zload1(k, olb));
      prb = dn1(prb, zload1(k, orb));
    }
    float2 ea_hi, eb_hi, ed, eup;   // UPD: the correction at the same places
    float ela, era, elb, erb;
    if constexpr (UPD) {
      const Rsrc ek = plane_rsrc(a.eu, k, q), eup_k = plane_rsrc(a.eu, k + 1, q);
      ea_hi = ld2(eup_k, oa >> 1, 0.0f);
      eb_hi = ld2(eup_k, ob >> 1, 0.0f);
      ed = ld2(ek, od >> 1, 0.0f);
      eup = ld2(ek, ou >> 1, 0.0f);
      ela = ld1(ek, ola >> 1, 0.0f);
      era = ld1(ek, ora >> 1, 0.0f);
      elb = ld1(ek, olb >> 1, 0.0f);
      erb = ld1(ek, orb >> 1, 0.0f);
    }
    V2 fa{zero, zero}, fb{zero, zero};
    if constexpr (!PROD) {
      const Rsrc fk = plane_rsrc(a.f, k, q);
      fa = ld2(fk, oa, zero);
      fb = ld2(fk, ob, zero);
    }
    PF<T> Fa, Fb;
    V2 za_next, zb_next;
    if constexpr (RHO) {
      const Rsrc rk = plane_rsrc(a.rt, k, q), rup = plane_rsrc(a.rt, k + 1, q);
      const bool in_hi = k + 1 < n;
      const V2 ha = ld2(rup, oa, zero), hb = ld2(rup, ob, zero);
      const V2 rd = ld2(rk, od, zero), rup2 = ld2(rk, ou, zero);
      const T rla = ld1(rk, ola, zero), rra = ld1(rk, ora, zero), rlb = ld1(rk, olb, zero), rrb = ld1(rk, orb, zero);
      if constexpr (UPD) {
        pa_hi = add_active(pa_hi, ea_hi, ha);
        pb_hi = add_active(pb_hi, eb_hi, hb);
        pd = add_active(pd, ed, rd);
        pup = add_active(pup, eup, rup2);
        pla = add_active(pla, ela, rla);
        pra = add_active(pra, era, rra);
        plb = add_active(plb, elb, rlb);
        prb = add_active(prb, erb, rrb);
      }
      const V2 ha_i{in_hi ? ha.x : inf, in_hi ? ha.y : inf}, hb_i{in_hi ? hb.x : inf, in_hi ? hb.y : inf};
      const T mid0 = face_beta(ra.x, rb.x), mid1 = face_beta(ra.y, rb.y);   // between rows a and b
      Fa.x0 = face_beta(rla, ra.x);
      Fa.x1 = face_beta(ra.x, ra.y);
      Fa.x2 = face_beta(ra.y, rra);
      Fa.ym0 = face_beta(rd.x, ra.x);
      Fa.ym1 = face_beta(rd.y, ra.y);
      Fa.yp0 = mid0;
      Fa.yp1 = mid1;
      Fa.zm0 = za.x;
      Fa.zm1 = za.y;
      Fa.zp0 = face_beta(ra.x, ha_i.x);
      Fa.zp1 = face_beta(ra.y, ha_i.y);
      Fb.x0 = face_beta(rlb, rb.x);
      Fb.x1 = face_beta(rb.x, rb.y);
      Fb.x2 = face_beta(rb.y, rrb);
      Fb.ym0 = mid0;
      Fb.ym1 = mid1;
      Fb.yp0 = face_beta(rb.x, rup2.x);
      Fb.yp1 = face_beta(rb.y, rup2.y);
      Fb.zm0 = zb.x;
      Fb.zm1 = zb.y;
      Fb.zp0 = face_beta(rb.x, hb_i.x);
      Fb.zp1 = face_beta(rb.y, hb_i.y);
      za_next = V2{Fa.zp0, Fa.zp1};
      zb_next = V2{Fb.zp0, Fb.zp1};
      ra = ha;
      rb = hb;
    } else {
      const Rsrc xk = plane_rsrc(a.bx, k, q), yk = plane_rsrc(a.by, k, q), zu = plane_rsrc(a.bz, k + 1, q);
      const V2 bxa = ld2(xk, oa, zero), bxb = ld2(xk, ob, zero);
      const T bxra = ld1(xk, ora, zero), bxrb = ld1(xk, orb, zero);
      const V2 bya = ld2(yk, oa, zero), byb = ld2(yk, ob, zero), byu = ld2(yk, ou, zero);
      za_next = ld2(zu, oa, zero);   // 0 above the grid (top wall)
      zb_next = ld2(zu, ob, zero);
      Fa = PF<T>{bxa.x, bxa.y, bxra, bya.x, bya.y, byb.x, byb.y, za.x, za.y, za_next.x, za_next.y};
      Fb = PF<T>{bxb.x, bxb.y, bxrb, byb.x, byb.y, byu.x, byu.y, zb.x, zb.y, zb_next.x, zb_next.y};
    }
    T r0a, r1a, r0b, r1b;
    pair_r(Fa, pa, pla, pra, pd, pb, pa_lo, pa_hi, fa, fs, a.inv_h2, r0a, r1a);
    pair_r(Fb, pb, plb, prb, pa, pup, pb_lo, pb_hi, fb, fs, a.inv_h2, r0b, r1b);
    const long long plane = static_cast<long long>(k) << (2 * q);
    const long long ca = plane + oa / sizeof(T), cb = plane + ob / sizeof(T);
    if constexpr (NORM) {
      if constexpr (UPD) {   // read again only after the next FP32 cycle: streaming stores
        stream_store(a.pout + ca, pa);
        stream_store(a.pout + cb, pb);
      }
      acc = fmad(r1a, r1a, fmad(r0a, r0a, acc));
      acc = fmad(r1b, r1b, fmad(r0b, r0b, acc));
      if (a.r32) {
        *reinterpret_cast<float2*>(a.r32 + ca) = float2{static_cast<float>(r0a), static_cast<float>(r1a)};
        *reinterpret_cast<float2*>(a.r32 + cb) = float2{static_cast<float>(r0b), static_cast<float>(r1b)};
      }
      if (a.e32) {
        *reinterpret_cast<float2*>(a.e32 + ca) = float2{0.0f, 0.0f};
        *reinterpret_cast<float2*>(a.e32 + cb) = float2{0.0f, 0.0f};
      }
      if (a.r64) {
        *reinterpret_cast<double2*>(a.r64 + ca) = double2{r0a, r1a};
        *reinterpret_cast<double2*>(a.r64 + cb) = double2{r0b, r1b};
      }
      if (a.z64) {
        *reinterpret_cast<double2*>(a.z64 + ca) = double2{0.0, 0.0};
        *reinterpret_cast<double2*>(a.z64 + cb) = double2{0.0, 0.0};
      }
    } else if constexpr (MODE == kModeRestrict) {
      // children in the order of every other restriction: (row a, plane 2K),
      // (row b, plane 2K), (row a, plane 2K+1), (row b, plane 2K+1)
      if ((k & 1) == 0) csum = zero;
      csum += r0a + r1a;
      csum += r0b + r1b;
      if (k & 1) {
        const int qc = q - 1;
        const int C = ((((k >> 1) << qc) | (ja >> 1)) << qc) | (ip >> 1);
        a.fc[C] = csum * T(0.125);
        a.ec[C] = zero;
      }
    } else {
      // the residual of f = 0 is -A d
      const double2 wa{-r0a, -r1a}, wb{-r0b, -r1b};
      stream_store(a.w + ca, wa);   // read again only by the update pass
      stream_store(a.w + cb, wb);
      if constexpr (FX) {
        // the new direction (read again after the next cycle), and the previous step's
        // update of p with the old direction
        stream_store(a.dn + ca, pa);
        stream_store(a.dn + cb, pb);
        if (a.pp) {
          const double alpha = *a.s_alpha;
          const double2 xa = *reinterpret_cast<const double2*>(a.pp + ca);
          const double2 xb = *reinterpret_cast<const double2*>(a.pp + cb);
          stream_store(a.pp + ca, double2{__builtin_fma(alpha, dca.x, xa.x), __builtin_fma(alpha, dca.y, xa.y)});
          stream_store(a.pp + cb, double2{__builtin_fma(alpha, dcb.x, xb.x), __builtin_fma(alpha, dcb.y, xb.y)});
        }
      }
      const double2 rva = ld2(plane_rsrc(a.r, k, q), oa, 0.0), rvb = ld2(plane_rsrc(a.r, k, q), ob, 0.0);
      acc = fmad(pa.y, wa.y, fmad(pa.x, wa.x, acc));
      acc = fmad(pb.y, wb.y, fmad(pb.x, wb.x, acc));
      acc2 = fmad(pa.y, rva.y, fmad(pa.x, rva.x, acc2));
      acc2 = fmad(pb.y, rvb.y, fmad(pb.x, rvb.x, acc2));
    }
    pa_lo = pa;
    pb_lo = pb;
    pa = pa_hi;
    pb = pb_hi;
    za = za_next;
    zb = zb_next;
    if constexpr (FX) {
      dca = dha;
      dcb = dhb;
    }
  }
  if constexpr (NORM) {
    const double s = block_sum(acc);
    if (tid == 0) a.partials[bid] = s;
  } else if constexpr (PROD) {
    const double s1 = block_sum(acc);
    __syncthreads();
    const double s2 = block_sum(acc2);
    if (tid == 0) {
      a.partials[bid] = s1;
      a.partials2[bid] = s2;
    }
  }
}

// RESTRICT on the density form (128 x 8 tiles), with the in-plane neighbours of every
// plane exchanged through LDS instead of read again from the caches.  A thread loads its
// pair's two rows of p and rt, plus its share of the plane's halo (the rows j0-1 and
// j0+8 and the x neighbours of the tile rows), one plane before they are needed (f in
// the step that uses it); at the
// start of step k it puts plane k+1 into one of two LDS planes, and after that step's
// barrier everyone reads plane k from the other.  Each line of p and rt is then fetched
// once per tile plane, the halo once more, however little of one step stays in L2.
// The faces, sums and restriction are those of k_residual_march, so the bits are too.
template <typename T>
__global__ __launch_bounds__(kMarchThreads) void k_restrict_lds(MarchArgs<T> a) {
  using V2 = typename Vec2<T>::type;
  constexpr int TX = 128, PAIRS = TX / 2, RP = kMarchThreads / PAIRS, TY = 2 * RP;
  constexpr int LW = TX + 2, LH = TY + 2;   // a staged plane: the tile and a 1-cell halo
  __shared__ T Lp[2][LH][LW];
  __shared__ T Lr[2][LH][LW];
  const int q = a.q, n = 1 << q;
  const T inf = __builtin_huge_val();
  const T zero = T(0);
  const int tid = threadIdx.x;
  const int G = gridDim.x, bid = blockIdx.x;
  const int lid = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;   // neighbours on one XCD
  const int ntx = n / TX, nty = n / TY;
  const int i0 = (lid % ntx) * TX;
  const int j0 = ((lid / ntx) % nty) * TY;
  const int k0 = (lid / (ntx * nty)) * a.kc;
  const int xt = tid % PAIRS, rp = tid / PAIRS;
  const int ip = i0 + 2 * xt;
  const int ja = j0 + 2 * rp, jb = ja + 1;
  const unsigned oa = off_of<T>(ip, ja, q), ob = off_of<T>(ip, jb, q);
  const int ra_ = 1 + 2 * rp, rb_ = ra_ + 1, cc = 1 + 2 * xt;   // the pair in a staged plane
  const T fs = a.fshift ? static_cast<T>(*a.fshift) : zero;
  // halo share: threads 0 .. 63 a pair of row j0-1, 64 .. 127 a pair of row j0+TY,
  // 128 .. 128+2TY-1 the cell left or right of a tile row
  int hr = -1, hc = 0;
  bool hpair = false;
  unsigned ho = 0;
  if (tid < 2 * PAIRS) {
    hpair = true;
    hr = tid < PAIRS ? 0 : LH - 1;
    hc = 1 + 2 * (tid % PAIRS);
    ho = off_of<T>(i0 + 2 * (tid % PAIRS), j0 - 1 + hr, q);
  } else if (tid < 2 * PAIRS + 2 * TY) {
    const int e = tid - 2 * PAIRS;
    hr = 1 + e / 2;
    hc = (e & 1) ? LW - 1 : 0;
    ho = off_of<T>((e & 1) ? i0 + TX : i0 - 1, j0 - 1 + hr, q);
  }
  // one plane's loads: the pair's rows of p and rt, and the halo share
  struct Plane {
    V2 pa, pb, ra, rb, hp, hrt;
  };
  auto load = [&](int kk) {
    const Rsrc pk = plane_rsrc(a.p, kk, q), rk = plane_rsrc(a.rt, kk, q);
    Plane L;
    L.pa = ld2(pk, oa, zero);
    L.pb = ld2(pk, ob, zero);
    L.ra = ld2(rk, oa, zero);
    L.rb = ld2(rk, ob, zero);
    L.hp = V2{zero, zero};
    L.hrt = V2{zero, zero};
    if (hpair) {
      L.hp = ld2(pk, ho, zero);
      L.hrt = ld2(rk, ho, zero);
    } else if (hr >= 0) {
      L.hp.x = ld1(pk, ho, zero);
      L.hrt.x = ld1(rk, ho, zero);
    }
    return L;
  };
  auto put = [&](int b, const Plane& L) {
    Lp[b][ra_][cc] = L.pa.x;
    Lp[b][ra_][cc + 1] = L.pa.y;
    Lp[b][rb_][cc] = L.pb.x;
    Lp[b][rb_][cc + 1] = L.pb.y;
    Lr[b][ra_][cc] = L.ra.x;
    Lr[b][ra_][cc + 1] = L.ra.y;
    Lr[b][rb_][cc] = L.rb.x;
    Lr[b][rb_][cc + 1] = L.rb.y;
    if (hpair) {
      Lp[b][hr][hc] = L.hp.x;
      Lp[b][hr][hc + 1] = L.hp.y;
      Lr[b][hr][hc] = L.hrt.x;
      Lr[b][hr][hc + 1] = L.hrt.y;
    } else if (hr >= 0) {
      Lp[b][hr][hc] = L.hp.x;
      Lr[b][hr][hc] = L.hrt.x;
    }
  };
  auto load_f = [&](int kk, V2& fa, V2& fb) {
    const Rsrc fk = plane_rsrc(a.f, kk, q);
    fa = ld2(fk, oa, zero);
    fb = ld2(fk, ob, zero);
  };

  // prologue: plane k0 staged; the pair's p on k0-1, rt faces to plane k0-1; plane k0+1
  // and f of k0 loaded
  Plane cur = load(k0);
  const Rsrc p_lo = plane_rsrc(a.p, k0 - 1, q), r_lo = plane_rsrc(a.rt, k0 - 1, q);
  V2 pa_lo = ld2(p_lo, oa, zero), pb_lo = ld2(p_lo, ob, zero);
  const V2 la = ld2(r_lo, oa, zero), lb = ld2(r_lo, ob, zero);
  Plane nxt = load(k0 + 1);
  put(k0 & 1, cur);
  const bool in_lo = k0 >= 1;
  V2 za = in_lo ? V2{face_beta(la.x, cur.ra.x), face_beta(la.y, cur.ra.y)} : V2{zero, zero};
  V2 zb = in_lo ? V2{face_beta(lb.x, cur.rb.x), face_beta(lb.y, cur.rb.y)} : V2{zero, zero};
  T csum = zero;
  for (int k = k0; k < k0 + a.kc; ++k) {
    __syncthreads();   // plane k staged; the other LDS plane no longer read
    put((k + 1) & 1, nxt);
    const Plane hi = nxt;   // the pair's p and rt on plane k+1
    nxt = load(k + 2);
    V2 fa, fb;
    load_f(k, fa, fb);
    // plane k's neighbours of the pair, from LDS
    const int b = k & 1;
    const V2 pd{Lp[b][ra_ - 1][cc], Lp[b][ra_ - 1][cc + 1]}, pup{Lp[b][rb_ + 1][cc], Lp[b][rb_ + 1][cc + 1]};
    const T pla = Lp[b][ra_][cc - 1], pra = Lp[b][ra_][cc + 2];
    const T plb = Lp[b][rb_][cc - 1], prb = Lp[b][rb_][cc + 2];
    const V2 rd{Lr[b][ra_ - 1][cc], Lr[b][ra_ - 1][cc + 1]}, rup2{Lr[b][rb_ + 1][cc], Lr[b][rb_ + 1][cc + 1]};
    const T rla = Lr[b][ra_][cc - 1], rra = Lr[b][ra_][cc + 2];
    const T rlb = Lr[b][rb_][cc - 1], rrb = Lr[b][rb_][cc + 2];
    const bool in_hi = k + 1 < n;
    const V2 ha_i{in_hi ? hi.ra.x : inf, in_hi ? hi.ra.y : inf}, hb_i{in_hi ? hi.rb.x : inf, in_hi ? hi.rb.y : inf};
    const V2 ra = cur.ra, rb = cur.rb;
    PF<T> Fa, Fb;
    const T mid0 = face_beta(ra.x, rb.x), mid1 = face_beta(ra.y, rb.y);   // between rows a and b
    Fa.x0 = face_beta(rla, ra.x);
    Fa.x1 = face_beta(ra.x, ra.y);
    Fa.x2 = face_beta(ra.y, rra);
    Fa.ym0 = face_beta(rd.x, ra.x);
    Fa.ym1 = face_beta(rd.y, ra.y);
    Fa.yp0 = mid0;
    Fa.yp1 = mid1;
    Fa.zm0 = za.x;
    Fa.zm1 = za.y;
    Fa.zp0 = face_beta(ra.x, ha_i.x);
    Fa.zp1 = face_beta(ra.y, ha_i.y);
    Fb.x0 = face_beta(rlb, rb.x);
    Fb.x1 = face_beta(rb.x, rb.y);
    Fb.x2 = face_beta(rb.y, rrb);
    Fb.ym0 = mid0;
    Fb.ym1 = mid1;
    Fb.yp0 = face_beta(rb.x, rup2.x);
    Fb.yp1 = face_beta(rb.y, rup2.y);
    Fb.zm0 = zb.x;
    Fb.zm1 = zb.y;
    Fb.zp0 = face_beta(rb.x, hb_i.x);
    Fb.zp1 = face_beta(rb.y, hb_i.y);
    T r0a, r1a, r0b, r1b;
    pair_r(Fa, cur.pa, pla, pra, pd, cur.pb, pa_lo, hi.pa, fa, fs, a.inv_h2, r0a, r1a);
    pair_r(Fb, cur.pb, plb, prb, cur.pa, pup, pb_lo, hi.pb, fb, fs, a.inv_h2, r0b, r1b);
    // children in the order of every other restriction: (row a, plane 2K),
    // (row b, plane 2K), (row a, plane 2K+1), (row b, plane 2K+1)
    if ((k & 1) == 0) csum = zero;
    csum += r0a + r1a;
    csum += r0b + r1b;
    if (k & 1) {
      const int qc = q - 1;
      const int C = ((((k >> 1) << qc) | (ja >> 1)) << qc) | (ip >> 1);
      a.fc[C] = csum * T(0.125);
      a.ec[C] = zero;
    }
    pa_lo = cur.pa;
    pb_lo = cur.pb;
    za = V2{Fa.zp0, Fa.zp1};
    zb = V2{Fb.zp0, Fb.zp1};
    cur = hi;
  }
}

// The flexible-CG pass of k_residual_march's FCGX mode on the density form (128 x 8
// tiles), with the in-plane stencil exchanged through LDS as in k_restrict_lds.  A
// thread loads d_old, z and rt of its pair's rows and of its share of the halo a plane
// before they are needed, forms the new direction d = z + beta d_old there, and stages
// d and rt; after the step's barrier the pair's neighbours come from LDS.  Products,
// sums, the deferred p += alpha d_old and the per-workgroup partial sums are those of
// the FCGX mode, in the same order, so the bits are too.
__global__ __launch_bounds__(kMarchThreads) void k_fcgx_lds(MarchArgs<double> a) {
  using V2 = double2;
  using T = double;
  constexpr int TX = 128, PAIRS = TX / 2, RP = kMarchThreads / PAIRS, TY = 2 * RP;
  constexpr int LW = TX + 2, LH = TY + 2;
  __shared__ T Ld[2][LH][LW];
  __shared__ T Lr[2][LH][LW];
  const int q = a.q, n = 1 << q;
  const T inf = __builtin_huge_val();
  const T zero = T(0);
  const int tid = threadIdx.x;
  if (a.s_alpha_save && blockIdx.x == 0 && tid == 0) *a.s_alpha_save = *a.s_alpha;
  const int G = gridDim.x, bid = blockIdx.x;
  const int lid = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;   // neighbours on one XCD
  const int ntx = n / TX, nty = n / TY;
  const int i0 = (lid % ntx) * TX;
  const int j0 = ((lid / ntx) % nty) * TY;
  const int k0 = (lid / (ntx * nty)) * a.kc;
  const int xt = tid % PAIRS, rp = tid / PAIRS;
  const int ip = i0 + 2 * xt;
  const int ja = j0 + 2 * rp, jb = ja + 1;
  const unsigned oa = off_of<T>(ip, ja, q), ob = off_of<T>(ip, jb, q);
  const int ra_ = 1 + 2 * rp, rb_ = ra_ + 1, cc = 1 + 2 * xt;
  const bool first = a.s_zw == nullptr;
  const double beta = first ? 0.0 : -*a.s_zw / *a.s_dw;
  auto dn2 = [&](V2 d, V2 z) -> V2 {
    return first ? z : V2{__builtin_fma(beta, d.x, z.x), __builtin_fma(beta, d.y, z.y)};
  };
  auto dn1 = [&](T d, T z) -> T { return first ? z : __builtin_fma(beta, d, z); };
  auto zload2 = [&](int kk, unsigned off) -> V2 {
    if (a.zx64) return ld2(plane_rsrc(a.zx64, kk, q), off, 0.0);
    const float2 zf = ld2(plane_rsrc(a.zx32, kk, q), off >> 1, 0.0f);
    return V2{static_cast<double>(zf.x), static_cast<double>(zf.y)};
  };
  auto zload1 = [&](int kk, unsigned off) -> T {
    if (a.zx64) return ld1(plane_rsrc(a.zx64, kk, q), off, 0.0);
    return static_cast<double>(ld1(plane_rsrc(a.zx32, kk, q), off >> 1, 0.0f));
  };
  // halo share as in k_restrict_lds
  int hr = -1, hc = 0;
  bool hpair = false;
  unsigned ho = 0;
  if (tid < 2 * PAIRS) {
    hpair = true;
    hr = tid < PAIRS ? 0 : LH - 1;
    hc = 1 + 2 * (tid % PAIRS);
    ho = off_of<T>(i0 + 2 * (tid % PAIRS), j0 - 1 + hr, q);
  } else if (tid < 2 * PAIRS + 2 * TY) {
    const int e = tid - 2 * PAIRS;
    hr = 1 + e / 2;
    hc = (e & 1) ? LW - 1 : 0;
    ho = off_of<T>((e & 1) ? i0 + TX : i0 - 1, j0 - 1 + hr, q);
  }
  // one plane's loads, and the plane as used: the pair's d_old and new direction, rt
  struct Raw {
    V2 da, db, za, zb, ra, rb, hd, hz, hrt;
  };
  struct Plane {
    V2 pa, pb, da, db, ra, rb;
  };
  auto load = [&](int kk) {
    const Rsrc dk = plane_rsrc(a.p, kk, q), rk = plane_rsrc(a.rt, kk, q);
    Raw L;
    L.da = ld2(dk, oa, zero);
    L.db = ld2(dk, ob, zero);
    L.za = zload2(kk, oa);
    L.zb = zload2(kk, ob);
    L.ra = ld2(rk, oa, zero);
    L.rb = ld2(rk, ob, zero);
    L.hd = V2{zero, zero};
    L.hz = V2{zero, zero};
    L.hrt = V2{zero, zero};
    if (hpair) {
      L.hd = ld2(dk, ho, zero);
      L.hz = zload2(kk, ho);
      L.hrt = ld2(rk, ho, zero);
    } else if (hr >= 0) {
      L.hd.x = ld1(dk, ho, zero);
      L.hz.x = zload1(kk, ho);
      L.hrt.x = ld1(rk, ho, zero);
    }
    return L;
  };
  // the new direction of a loaded plane, staged in LDS plane b
  auto put = [&](int b, const Raw& L) {
    Plane P;
    P.pa = dn2(L.da, L.za);
    P.pb = dn2(L.db, L.zb);
    P.da = L.da;
    P.db = L.db;
    P.ra = L.ra;
    P.rb = L.rb;
    Ld[b][ra_][cc] = P.pa.x;
    Ld[b][ra_][cc + 1] = P.pa.y;
    Ld[b][rb_][cc] = P.pb.x;
    Ld[b][rb_][cc + 1] = P.pb.y;
    Lr[b][ra_][cc] = L.ra.x;
    Lr[b][ra_][cc + 1] = L.ra.y;
    Lr[b][rb_][cc] = L.rb.x;
    Lr[b][rb_][cc + 1] = L.rb.y;
    if (hpair) {
      const V2 h = dn2(L.hd, L.hz);
      Ld[b][hr][hc] = h.x;
      Ld[b][hr][hc + 1] = h.y;
      Lr[b][hr][hc] = L.hrt.x;
      Lr[b][hr][hc + 1] = L.hrt.y;
    } else if (hr >= 0) {
      Ld[b][hr][hc] = dn1(L.hd.x, L.hz.x);
      Lr[b][hr][hc] = L.hrt.x;
    }
    return P;
  };

  // prologue: plane k0 staged; the pair's direction on k0-1 and rt faces to plane k0-1;
  // plane k0+1 loaded
  Plane cur = put(k0 & 1, load(k0));
  const Rsrc d_lo = plane_rsrc(a.p, k0 - 1, q), r_lo = plane_rsrc(a.rt, k0 - 1, q);
  V2 pa_lo = dn2(ld2(d_lo, oa, zero), zload2(k0 - 1, oa));
  V2 pb_lo = dn2(ld2(d_lo, ob, zero), zload2(k0 - 1, ob));
  const V2 la = ld2(r_lo, oa, zero), lb = ld2(r_lo, ob, zero);
  Raw nxt = load(k0 + 1);
  const bool in_lo = k0 >= 1;
  V2 za = in_lo ? V2{face_beta(la.x, cur.ra.x), face_beta(la.y, cur.ra.y)} : V2{zero, zero};
  V2 zb = in_lo ? V2{face_beta(lb.x, cur.rb.x), face_beta(lb.y, cur.rb.y)} : V2{zero, zero};
  double acc = 0.0, acc2 = 0.0;
  for (int k = k0; k < k0 + a.kc; ++k) {
    __syncthreads();   // plane k staged; the other LDS plane no longer read
    const Plane hi = put((k + 1) & 1, nxt);
    nxt = load(k + 2);
    const int b = k & 1;
    const V2 pd{Ld[b][ra_ - 1][cc], Ld[b][ra_ - 1][cc + 1]}, pup{Ld[b][rb_ + 1][cc], Ld[b][rb_ + 1][cc + 1]};
    const T pla = Ld[b][ra_][cc - 1], pra = Ld[b][ra_][cc + 2];
    const T plb = Ld[b][rb_][cc - 1], prb = Ld[b][rb_][cc + 2];
    const V2 rd{Lr[b][ra_ - 1][cc], Lr[b][ra_ - 1][cc + 1]}, rup2{Lr[b][rb_ + 1][cc], Lr[b][rb_ + 1][cc + 1]};
    const T rla = Lr[b][ra_][cc - 1], rra = Lr[b][ra_][cc + 2];
    const T rlb = Lr[b][rb_][cc - 1], rrb = Lr[b][rb_][cc + 2];
    const bool in_hi = k + 1 < n;
    const V2 ha_i{in_hi ? hi.ra.x : inf, in_hi ? hi.ra.y : inf}, hb_i{in_hi ? hi.rb.x : inf, in_hi ? hi.rb.y : inf};
    const V2 ra = cur.ra, rb = cur.rb;
    PF<T> Fa, Fb;
    const T mid0 = face_beta(ra.x, rb.x), mid1 = face_beta(ra.y, rb.y);
    Fa.x0 = face_beta(rla, ra.x);
    Fa.x1 = face_beta(ra.x, ra.y);
    Fa.x2 = face_beta(ra.y, rra);
    Fa.ym0 = face_beta(rd.x, ra.x);
    Fa.ym1 = face_beta(rd.y, ra.y);
    Fa.yp0 = mid0;
    Fa.yp1 = mid1;
    Fa.zm0 = za.x;
    Fa.zm1 = za.y;
    Fa.zp0 = face_beta(ra.x, ha_i.x);
    Fa.zp1 = face_beta(ra.y, ha_i.y);
    Fb.x0 = face_beta(rlb, rb.x);
    Fb.x1 = face_beta(rb.x, rb.y);
    Fb.x2 = face_beta(rb.y, rrb);
    Fb.ym0 = mid0;
    Fb.ym1 = mid1;
    Fb.yp0 = face_beta(rb.x, rup2.x);
    Fb.yp1 = face_beta(rb.y, rup2.y);
    Fb.zm0 = zb.x;
    Fb.zm1 = zb.y;
    Fb.zp0 = face_beta(rb.x, hb_i.x);
    Fb.zp1 = face_beta(rb.y, hb_i.y);
    T r0a, r1a, r0b, r1b;
    const V2 f0{zero, zero};
    pair_r(Fa, cur.pa, pla, pra, pd, cur.pb, pa_lo, hi.pa, f0, zero, a.inv_h2, r0a, r1a);
    pair_r(Fb, cur.pb, plb, prb, cur.pa, pup, pb_lo, hi.pb, f0, zero, a.inv_h2, r0b, r1b);
    const long long plane = static_cast<long long>(k) << (2 * q);
    const long long ca = plane + oa / sizeof(T), cb = plane + ob / sizeof(T);
    // the residual of f = 0 is -A d
    const V2 wa{-r0a, -r1a}, wb{-r0b, -r1b};
    stream_store(a.w + ca, wa);   // read again only by the update pass
    stream_store(a.w + cb, wb);
    // the new direction (read again after the next cycle), and the previous step's
    // update of p with the old direction
    stream_store(a.dn + ca, cur.pa);
    stream_store(a.dn + cb, cur.pb);
    if (a.pp) {
      const double alpha = *a.s_alpha;
      V2 xa = *reinterpret_cast<const V2*>(a.pp + ca);
      V2 xb = *reinterpret_cast<const V2*>(a.pp + cb);
      if (a.dprev) {   // the step before's update first, as it would have been applied
        const double alpha0 = *a.s_alpha_prev;
        const V2 oa = *reinterpret_cast<const V2*>(a.dprev + ca), ob = *reinterpret_cast<const V2*>(a.dprev + cb);
        xa = V2{__builtin_fma(alpha0, oa.x, xa.x), __builtin_fma(alpha0, oa.y, xa.y)};
        xb = V2{__builtin_fma(alpha0, ob.x, xb.x), __builtin_fma(alpha0, ob.y, xb.y)};
      }
      stream_store(a.pp + ca, V2{__builtin_fma(alpha, cur.da.x, xa.x), __builtin_fma(alpha, cur.da.y, xa.y)});
      stream_store(a.pp + cb, V2{__builtin_fma(alpha, cur.db.x, xb.x), __builtin_fma(alpha, cur.db.y, xb.y)});
    }
    const V2 rva = ld2(plane_rsrc(a.r, k, q), oa, 0.0), rvb = ld2(plane_rsrc(a.r, k, q), ob, 0.0);
    acc = fmad(cur.pa.y, wa.y, fmad(cur.pa.x, wa.x, acc));
    acc = fmad(cur.pb.y, wb.y, fmad(cur.pb.x, wb.x, acc));
    acc2 = fmad(cur.pa.y, rva.y, fmad(cur.pa.x, rva.x, acc2));
    acc2 = fmad(cur.pb.y, rvb.y, fmad(cur.pb.x, rvb.x, acc2));
    pa_lo = cur.pa;
    pb_lo = cur.pb;
    za = V2{Fa.zp0, Fa.zp1};
    zb = V2{Fb.zp0, Fb.zp1};
    cur = hi;
  }
  const double s1 = block_sum(acc);
  __syncthreads();
  const double s2 = block_sum(acc2);
  if (tid == 0) {
    a.partials[bid] = s1;
    a.partials2[bid] = s2;
  }
}

template <typename T, bool RHO, int MODE>
hipError_t launch_mode(MarchArgs<T> a, int* nblocks, hipStream_t s) {
  const int n = 1 << a.q;
  const int TX = n >= 128 ? 128 : n;
  const int TY = 2 * (kMarchThreads / (TX / 2));
  if (n < 32 || TY > n) return hipErrorInvalidValue;
  const long long tiles = static_cast<long long>(n / TX) * (n / TY);
  int kc = 64;
  while (kc > 2 && tiles * (n / kc) < 1024) kc /= 2;
  if (kc > n) kc = n;
  while (tiles * (n / kc) > kNumPartials) kc *= 2;
  a.kc = kc;
  const int blocks = static_cast<int>(tiles * (n / kc));
  *nblocks = blocks;
  const dim3 grid(blocks), block(kMarchThreads);
  if (TX == 128)
    hipLaunchKernelGGL((k_residual_march<T, RHO, MODE, 128>), grid, block, 0, s, a);
  else if (TX == 64)
    hipLaunchKernelGGL((k_residual_march<T, RHO, MODE, 64>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k_residual_march<T, RHO, MODE, 32>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int MODE, typename T>
hipError_t launch_form(MarchArgs<T> a, int* nblocks, hipStream_t s) {
  return a.rt ? launch_mode<T, true, MODE>(a, nblocks, s) : launch_mode<T, false, MODE>(a, nblocks, s);
}

}  // namespace

int march_supported(int q) { return (1 << q) >= 32; }
int fcgx_defer_supported(const double* rt, int q) { return rt != nullptr && (1 << q) >= 128; }

hipError_t launch_residual_norm_march(const double* p, const double* f, const double* bx, const double* by,
                                      const double* bz, const double* rt, int q, double h, const double* fshift,
                                      float* r32, float* e32, double* r64, double* z64, double* partials,
                                      int* nblocks, hipStream_t s) {
  MarchArgs<double> a{};
  a.p = p;
  a.f = f;
  a.bx = bx;
  a.by = by;
  a.bz = bz;
  a.rt = rt;
  a.fshift = fshift;
  a.q = q;
  a.inv_h2 = 1.0 / (h * h);
  a.r32 = r32;
  a.e32 = e32;
  a.r64 = r64;
  a.z64 = z64;
  a.partials = partials;
  return launch_form<kModeNorm>(a, nblocks, s);
}

template <typename T>
hipError_t launch_residual_restrict_march(const T* p, const T* f, const T* bx, const T* by, const T* bz, const T* rt,
                                          int q, double h, const double* fshift, T* fc, T* ec, hipStream_t s) {
  MarchArgs<T> a{};
  a.p = p;
  a.f = f;
  a.bx = bx;
  a.by = by;
  a.bz = bz;
  a.rt = rt;
  a.fshift = fshift;
  a.q = q;
  a.inv_h2 = 1.0 / (h * h);
  a.fc = fc;
  a.ec = ec;
  int nb = 0;
  if (rt && (1 << q) >= 128) {   // the density form: neighbours through LDS
    const int n = 1 << q;
    const long long tiles = static_cast<long long>(n / 128) * (n / 8);
    int kc = 64;
    while (kc > 2 && tiles * (n / kc) < 1024) kc /= 2;
    if (kc > n) kc = n;
    a.kc = kc;
    hipLaunchKernelGGL(k_restrict_lds<T>, dim3(static_cast<unsigned>(tiles * (n / kc))), dim3(kMarchThreads), 0, s, a);
    return hipGetLastError();
  }
  return launch_form<kModeRestrict>(a, &nb, s);
}

hipError_t launch_residual_norm_update_march(const double* p, const float* e, double* pout, const double* f,
                                             const double* rt, int q, double h, const double* fshift, float* r32,
                                             float* e32, double* partials, int* nblocks, hipStream_t s) {
  if (!rt || p == pout || e == e32) return hipErrorInvalidValue;
  MarchArgs<double> a{};
  a.p = p;
  a.f = f;
  a.rt = rt;
  a.fshift = fshift;
  a.q = q;
  a.inv_h2 = 1.0 / (h * h);
  a.r32 = r32;
  a.e32 = e32;
  a.partials = partials;
  a.eu = e;
  a.pout = pout;
  return launch_mode<double, true, kModeNormUpdate>(a, nblocks, s);
}

template hipError_t launch_residual_restrict_march<double>(const double*, const double*, const double*, const double*,
                                                           const double*, const double*, int, double, const double*,
                                                           double*, double*, hipStream_t);
template hipError_t launch_residual_restrict_march<float>(const float*, const float*, const float*, const float*,
                                                          const float*, const float*, int, double, const double*,
                                                          float*, float*, hipStream_t);

hipError_t launch_fcg_aw_march(const double* d, const double* r, const double* bx, const double* by, const double* bz,
                               const double* rt, int q, double h, double* w, double* part_dw, double* part_dr,
                               int* nblocks, hipStream_t s) {
  MarchArgs<double> a{};
  a.p = d;
  a.bx = bx;
  a.by = by;
  a.bz = bz;
  a.rt = rt;
  a.q = q;
  a.inv_h2 = 1.0 / (h * h);
  a.r = r;
  a.w = w;
  a.partials = part_dw;
  a.partials2 = part_dr;
  return launch_form<kModeAw>(a, nblocks, s);
}

hipError_t launch_fcg_x_march(const double* z64, const float* z32, const double* d, double* dn, double* p,
                              const double* s_zw, const double* s_dw, const double* s_alpha, const double* r,
                              const double* bx, const double* by, const double* bz, const double* rt, int q, double h,
                              double* w, double* part_dw, double* part_dr, int* nblocks, hipStream_t s,
                              const FcgxDefer* df) {
  if ((z64 == nullptr) == (z32 == nullptr) || !d || !dn || dn == d || (s_zw == nullptr) != (s_dw == nullptr))
    return hipErrorInvalidValue;
  if (df && (!fcgx_defer_supported(rt, q) || !s_zw || (df->skip ? !df->s_alpha_save
                                                                : (!df->d_prev || !df->s_alpha_prev ||
                                                                   df->d_prev == dn || df->d_prev == d))))
    return hipErrorInvalidValue;
  MarchArgs<double> a{};
  a.p = d;
  a.bx = bx;
  a.by = by;
  a.bz = bz;
  a.rt = rt;
  a.q = q;
  a.inv_h2 = 1.0 / (h * h);
  a.r = r;
  a.w = w;
  a.partials = part_dw;
  a.partials2 = part_dr;
  a.zx64 = z64;
  a.zx32 = z32;
  a.s_zw = s_zw;
  a.s_dw = s_dw;
  a.s_alpha = s_alpha;
  a.dn = dn;
  a.pp = s_zw ? p : nullptr;
  if (df) {
    if (df->skip) {
      a.pp = nullptr;
      a.s_alpha_save = df->s_alpha_save;
    } else {
      a.dprev = df->d_prev;
      a.s_alpha_prev = df->s_alpha_prev;
    }
  }
  if (rt && (1 << q) >= 128) {   // the density form: the stencil through LDS
    const int n = 1 << q;
    const long long tiles = static_cast<long long>(n / 128) * (n / 8);
    int kc = 64;
    while (kc > 2 && tiles * (n / kc) < 1024) kc /= 2;
    if (kc > n) kc = n;
    while (tiles * (n / kc) > kNumPartials) kc *= 2;
    a.kc = kc;
    const int blocks = static_cast<int>(tiles * (n / kc));
    *nblocks = blocks;
    hipLaunchKernelGGL(k_fcgx_lds, dim3(blocks), dim3(kMarchThreads), 0, s, a);
    return hipGetLastError();
  }
  return launch_form<kModeFcgX>(a, nblocks, s);
}

}  // namespace mg
