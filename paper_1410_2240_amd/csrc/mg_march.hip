// Finest-grid residual passes that march up z (CDNA4, FP64).
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

constexpr int kMarchThreads = 256;
enum { kModeNorm = 0, kModeRestrict = 1, kModeAw = 2 };

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

struct MarchArgs {
  const double* p;    // p, or d in AW mode
  const double* f;    // NORM / RESTRICT
  const double* bx;
  const double* by;
  const double* bz;
  const double* rt;
  const double* fshift;
  int q, kc;
  double inv_h2;
  // NORM
  float* r32;
  float* e32;
  double* r64;
  double* z64;
  double* partials;   // NORM: r^2; AW: d.w
  // RESTRICT
  double* fc;
  double* ec;
  // AW
  const double* r;
  double* w;
  double* partials2;  // AW: d.r
};

// The six faces of the two cells of an x-pair
struct PF {
  double x0, x1, x2, ym0, ym1, yp0, yp1, zm0, zm1, zp0, zp1;
};

// r of the two cells of a pair from p at the cell, its x neighbours (pl, pr), the pair
// in the rows below / above and the planes below / above
__device__ __forceinline__ void pair_r(const PF& F, double2 pc, double pl, double pr, double2 pyd, double2 pyu,
                                       double2 pzd, double2 pzu, double2 fv, double fs, double inv_h2, double& r0,
                                       double& r1) {
  const double D0 = F.x0 + F.x1 + F.ym0 + F.yp0 + F.zm0 + F.zp0;
  const double D1 = F.x1 + F.x2 + F.ym1 + F.yp1 + F.zm1 + F.zp1;
  const double s0 = fmad(F.zp0, pzu.x - pc.x, fmad(F.zm0, pzd.x - pc.x, fmad(F.yp0, pyu.x - pc.x,
                    fmad(F.ym0, pyd.x - pc.x, fmad(F.x1, pc.y - pc.x, F.x0 * (pl - pc.x))))));
  const double s1 = fmad(F.zp1, pzu.y - pc.y, fmad(F.zm1, pzd.y - pc.y, fmad(F.yp1, pyu.y - pc.y,
                    fmad(F.ym1, pyd.y - pc.y, fmad(F.x2, pr - pc.y, F.x1 * (pc.x - pc.y))))));
  r0 = D0 > 0.0 ? fmad(-inv_h2, s0, fv.x - fs) : 0.0;
  r1 = D1 > 0.0 ? fmad(-inv_h2, s1, fv.y - fs) : 0.0;
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

template <bool RHO, int MODE, int TX>
__global__ __launch_bounds__(kMarchThreads) void k_residual_march(MarchArgs a) {
  constexpr int PAIRS = TX / 2;                 // x-pairs per tile row
  constexpr int RP = kMarchThreads / PAIRS;     // row pairs per tile
  constexpr int TY = 2 * RP;
  const int q = a.q, n = 1 << q;
  const double inf = __builtin_huge_val();
  const int tid = threadIdx.x;
  const int G = gridDim.x, bid = blockIdx.x;
  const int lid = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;   // neighbours on one XCD
  const int ntx = n / TX, nty = n / TY;
  const int i0 = (lid % ntx) * TX;
  const int j0 = ((lid / ntx) % nty) * TY;
  const int k0 = (lid / (ntx * nty)) * a.kc;
  const int ip = i0 + 2 * (tid % PAIRS);
  const int ja = j0 + 2 * (tid / PAIRS), jb = ja + 1;
  const unsigned oa = off_of<double>(ip, ja, q), ob = off_of<double>(ip, jb, q);
  const unsigned od = off_of<double>(ip, ja - 1, q), ou = off_of<double>(ip, jb + 1, q);
  const unsigned ola = off_of<double>(ip - 1, ja, q), ora = off_of<double>(ip + 2, ja, q);
  const unsigned olb = off_of<double>(ip - 1, jb, q), orb = off_of<double>(ip + 2, jb, q);
  const double fs = (MODE != kModeAw && a.fshift) ? *a.fshift : 0.0;

  // window: the pair's p on the planes below, at and above the current one (rows a, b)
  const Rsrc p_lo = plane_rsrc(a.p, k0 - 1, q), p_c = plane_rsrc(a.p, k0, q);
  double2 pa_lo = ld2(p_lo, oa, 0.0), pb_lo = ld2(p_lo, ob, 0.0);
  double2 pa = ld2(p_c, oa, 0.0), pb = ld2(p_c, ob, 0.0);
  // faces to the plane below (carried), and for the density form the pair's density
  double2 za, zb;                 // zm of rows a, b on the current plane
  double2 ra, rb;                 // density form: rt of the pair on the current plane
  if constexpr (RHO) {
    const bool in_lo = k0 >= 1;
    const double2 la = ld2(plane_rsrc(a.rt, k0 - 1, q), oa, 0.0), lb = ld2(plane_rsrc(a.rt, k0 - 1, q), ob, 0.0);
    ra = ld2(plane_rsrc(a.rt, k0, q), oa, 0.0);
    rb = ld2(plane_rsrc(a.rt, k0, q), ob, 0.0);
    za = in_lo ? double2{face_beta(la.x, ra.x), face_beta(la.y, ra.y)} : double2{0.0, 0.0};
    zb = in_lo ? double2{face_beta(lb.x, rb.x), face_beta(lb.y, rb.y)} : double2{0.0, 0.0};
  } else {
    const Rsrc zk = plane_rsrc(a.bz, k0, q);
    za = ld2(zk, oa, 0.0);   // 0 on the bottom wall (stored) and below the grid
    zb = ld2(zk, ob, 0.0);
  }
  double acc = 0.0, acc2 = 0.0, csum = 0.0;
  for (int k = k0; k < k0 + a.kc; ++k) {
    const Rsrc pk = plane_rsrc(a.p, k, q), pu = plane_rsrc(a.p, k + 1, q);
    const double2 pa_hi = ld2(pu, oa, 0.0), pb_hi = ld2(pu, ob, 0.0);   // 0 above the grid
    const double2 pd = ld2(pk, od, 0.0), pup = ld2(pk, ou, 0.0);
    const double pla = ld1(pk, ola, 0.0), pra = ld1(pk, ora, 0.0);
    const double plb = ld1(pk, olb, 0.0), prb = ld1(pk, orb, 0.0);
    double2 fa{0.0, 0.0}, fb{0.0, 0.0};
    if constexpr (MODE != kModeAw) {
      const Rsrc fk = plane_rsrc(a.f, k, q);
      fa = ld2(fk, oa, 0.0);
      fb = ld2(fk, ob, 0.0);
    }
    PF Fa, Fb;
    double2 za_next, zb_next;
    if constexpr (RHO) {
      const Rsrc rk = plane_rsrc(a.rt, k, q), rup = plane_rsrc(a.rt, k + 1, q);
      const bool in_hi = k + 1 < n;
      const double2 ha = ld2(rup, oa, 0.0), hb = ld2(rup, ob, 0.0);
      const double2 rd = ld2(rk, od, 0.0), rup2 = ld2(rk, ou, 0.0);
      const double rla = ld1(rk, ola, 0.0), rra = ld1(rk, ora, 0.0), rlb = ld1(rk, olb, 0.0), rrb = ld1(rk, orb, 0.0);
      const double2 ha_i{in_hi ? ha.x : inf, in_hi ? ha.y : inf}, hb_i{in_hi ? hb.x : inf, in_hi ? hb.y : inf};
      const double mid0 = face_beta(ra.x, rb.x), mid1 = face_beta(ra.y, rb.y);   // between rows a and b
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
      za_next = double2{Fa.zp0, Fa.zp1};
      zb_next = double2{Fb.zp0, Fb.zp1};
      ra = ha;
      rb = hb;
    } else {
      const Rsrc xk = plane_rsrc(a.bx, k, q), yk = plane_rsrc(a.by, k, q), zu = plane_rsrc(a.bz, k + 1, q);
      const double2 bxa = ld2(xk, oa, 0.0), bxb = ld2(xk, ob, 0.0);
      const double bxra = ld1(xk, ora, 0.0), bxrb = ld1(xk, orb, 0.0);
      const double2 bya = ld2(yk, oa, 0.0), byb = ld2(yk, ob, 0.0), byu = ld2(yk, ou, 0.0);
      za_next = ld2(zu, oa, 0.0);   // 0 above the grid (top wall)
      zb_next = ld2(zu, ob, 0.0);
      Fa = PF{bxa.x, bxa.y, bxra, bya.x, bya.y, byb.x, byb.y, za.x, za.y, za_next.x, za_next.y};
      Fb = PF{bxb.x, bxb.y, bxrb, byb.x, byb.y, byu.x, byu.y, zb.x, zb.y, zb_next.x, zb_next.y};
    }
    double r0a, r1a, r0b, r1b;
    pair_r(Fa, pa, pla, pra, pd, pb, pa_lo, pa_hi, fa, fs, a.inv_h2, r0a, r1a);
    pair_r(Fb, pb, plb, prb, pa, pup, pb_lo, pb_hi, fb, fs, a.inv_h2, r0b, r1b);
    const long long plane = static_cast<long long>(k) << (2 * q);
    const long long ca = plane + (oa >> 3), cb = plane + (ob >> 3);
    if constexpr (MODE == kModeNorm) {
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
      if ((k & 1) == 0) csum = 0.0;
      csum += r0a + r1a;
      csum += r0b + r1b;
      if (k & 1) {
        const int qc = q - 1;
        const int C = ((((k >> 1) << qc) | (ja >> 1)) << qc) | (ip >> 1);
        a.fc[C] = csum * 0.125;
        a.ec[C] = 0.0;
      }
    } else {
      // the residual of f = 0 is -A d
      const double2 wa{-r0a, -r1a}, wb{-r0b, -r1b};
      *reinterpret_cast<double2*>(a.w + ca) = wa;
      *reinterpret_cast<double2*>(a.w + cb) = wb;
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
  }
  if constexpr (MODE == kModeNorm) {
    const double s = block_sum(acc);
    if (tid == 0) a.partials[bid] = s;
  } else if constexpr (MODE == kModeAw) {
    const double s1 = block_sum(acc);
    __syncthreads();
    const double s2 = block_sum(acc2);
    if (tid == 0) {
      a.partials[bid] = s1;
      a.partials2[bid] = s2;
    }
  }
}

template <bool RHO, int MODE>
hipError_t launch_mode(MarchArgs a, int* nblocks, hipStream_t s) {
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
    hipLaunchKernelGGL((k_residual_march<RHO, MODE, 128>), grid, block, 0, s, a);
  else if (TX == 64)
    hipLaunchKernelGGL((k_residual_march<RHO, MODE, 64>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k_residual_march<RHO, MODE, 32>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_form(MarchArgs a, int* nblocks, hipStream_t s) {
  return a.rt ? launch_mode<true, MODE>(a, nblocks, s) : launch_mode<false, MODE>(a, nblocks, s);
}

}  // namespace

int march_supported(int q) { return (1 << q) >= 32; }

hipError_t launch_residual_norm_march(const double* p, const double* f, const double* bx, const double* by,
                                      const double* bz, const double* rt, int q, double h, const double* fshift,
                                      float* r32, float* e32, double* r64, double* z64, double* partials,
                                      int* nblocks, hipStream_t s) {
  MarchArgs a{};
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

hipError_t launch_residual_restrict_march(const double* p, const double* f, const double* bx, const double* by,
                                          const double* bz, const double* rt, int q, double h, const double* fshift,
                                          double* fc, double* ec, hipStream_t s) {
  MarchArgs a{};
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
  return launch_form<kModeRestrict>(a, &nb, s);
}

hipError_t launch_fcg_aw_march(const double* d, const double* r, const double* bx, const double* by, const double* bz,
                               const double* rt, int q, double h, double* w, double* part_dw, double* part_dr,
                               int* nblocks, hipStream_t s) {
  MarchArgs a{};
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

}  // namespace mg
