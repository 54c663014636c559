// Device kernels of the multigrid pressure solve for CDNA4 (gfx950).
//
// All kernels are memory-bound stencils on [k][j][i] arrays (x fastest) with
// 32-bit cell indices (N <= 1024).  Conventions shared by every kernel:
//   * periodic neighbours in x and y by masking with n-1 (n is a power of two);
//   * z walls: the bottom-wall face bz[0] is zero after setup, and the top wall has no
//     storage, so a z neighbour outside the grid is never read;
//   * a cell is active exactly when its diagonal D = sum of its six face coefficients
//     is positive: setup zeroes every face touching the body, and a coarse cell whose
//     children are all body cells inherits only zero faces.  The V-cycle kernels use
//     D > 0 instead of reading the mask.
#include "mg_kernels.h"
#include "mg_plan.h"

namespace mg {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int cell(int i, int j, int k, int q) { return (((k << q) + j) << q) + i; }

inline unsigned grid_for(long long work) {
  return static_cast<unsigned>((work + kBlock - 1) / kBlock);
}

// Six face coefficients and the matching neighbour offsets of cell (i, j, k).
template <typename T>
struct Faces {
  T xm, xp, ym, yp, zm, zp;   // beta on the low/high faces in x, y, z
  int cxm, cxp, cym, cyp, czm, czp;
};

template <typename T>
__device__ __forceinline__ Faces<T> load_faces(const T* __restrict__ bx, const T* __restrict__ by,
                                               const T* __restrict__ bz, int i, int j, int k, int q) {
  const int n = 1 << q, m = n - 1;
  const int c = cell(i, j, k, q);
  Faces<T> F;
  F.cxm = cell((i - 1) & m, j, k, q);
  F.cxp = cell((i + 1) & m, j, k, q);
  F.cym = cell(i, (j - 1) & m, k, q);
  F.cyp = cell(i, (j + 1) & m, k, q);
  F.czm = k > 0 ? c - (1 << (2 * q)) : c;
  F.czp = k < m ? c + (1 << (2 * q)) : c;
  F.xm = bx[c];
  F.xp = bx[F.cxp];
  F.ym = by[c];
  F.yp = by[F.cyp];
  F.zm = bz[c];                          // 0 on the bottom wall
  F.zp = k < m ? bz[F.czp] : T(0);       // top wall
  return F;
}

template <typename T>
__device__ __forceinline__ T diag(const Faces<T>& F) {
  return F.xm + F.xp + F.ym + F.yp + F.zm + F.zp;
}

// sum_f beta_f (p_nb - p_c): the flux balance of A p without the h^-2 factor
template <typename T>
__device__ __forceinline__ T flux_sum(const Faces<T>& F, const T* __restrict__ p, T pc) {
  return F.xm * (p[F.cxm] - pc) + F.xp * (p[F.cxp] - pc) + F.ym * (p[F.cym] - pc) +
         F.yp * (p[F.cyp] - pc) + F.zm * (p[F.czm] - pc) + F.zp * (p[F.czp] - pc);
}

template <typename T>
struct V2of;
template <>
struct V2of<double> {
  using type = double2;
};
template <>
struct V2of<float> {
  using type = float2;
};

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ typename V2of<T>::type ld2(const T* __restrict__ a, int c) {
  return *reinterpret_cast<const typename V2of<T>::type*>(a + c);
}

// Face coefficients around the x-neighbour pair (i, j, k), (i+1, j, k) with i even:
// the x faces at i, i+1, i+2 (low-face indexing, so x1 is the face between the two
// cells) and the low / high y and z faces of both cells.
template <typename T>
struct PairFaces {
  using V2 = typename V2of<T>::type;
  T x0, x1, x2;
  V2 ym, yp, zm, zp;
};

template <typename T>
__device__ __forceinline__ PairFaces<T> pair_faces(const T* __restrict__ bx, const T* __restrict__ by,
                                                   const T* __restrict__ bz, int i, int j, int k, int q) {
  using V2 = typename V2of<T>::type;
  const int m = (1 << q) - 1, nn = 1 << (2 * q);
  const int c = cell(i, j, k, q);
  PairFaces<T> F;
  const V2 bxv = ld2(bx, c);
  F.x0 = bxv.x;
  F.x1 = bxv.y;
  F.x2 = bx[cell((i + 2) & m, j, k, q)];
  F.ym = ld2(by, c);
  F.yp = ld2(by, cell(i, (j + 1) & m, k, q));
  F.zm = ld2(bz, c);   // 0 on the bottom wall
  F.zp = k < m ? ld2(bz, c + nn) : V2{T(0), T(0)};
  return F;
}

// The density form of the same coefficients, for the finest grid of a hierarchy built
// from the cell density: rt holds rho on active cells and +inf on every other cell,
// and a neighbour beyond a z wall counts as +inf too.  beta = 2 / (rt_L + rt_R) is then
// 0 on every face that touches an inactive cell or a wall, and on open faces it is bit
// for bit the stored coefficient (the sum is commutative, and both are formed by
// face_beta).  A sweep then reads one density instead of three face arrays.
template <typename T>
__device__ __forceinline__ T beta_rho(T a, T b) { return face_beta(a, b); }

template <typename T>
__device__ __forceinline__ PairFaces<T> pair_faces_rho(const T* __restrict__ rt, int i, int j, int k, int q) {
  using V2 = typename V2of<T>::type;
  const int m = (1 << q) - 1, nn = 1 << (2 * q);
  const int c = cell(i, j, k, q);
  const T inf = __builtin_huge_val();
  const V2 rc = ld2(rt, c);
  const T rl = rt[cell((i - 1) & m, j, k, q)], rr = rt[cell((i + 2) & m, j, k, q)];
  const V2 rs = ld2(rt, cell(i, (j - 1) & m, k, q)), rn = ld2(rt, cell(i, (j + 1) & m, k, q));
  const V2 rd = k > 0 ? ld2(rt, c - nn) : V2{inf, inf};
  const V2 ru = k < m ? ld2(rt, c + nn) : V2{inf, inf};
  PairFaces<T> F;
  F.x0 = beta_rho(rl, rc.x);
  F.x1 = beta_rho(rc.x, rc.y);
  F.x2 = beta_rho(rc.y, rr);
  F.ym = V2{beta_rho(rs.x, rc.x), beta_rho(rs.y, rc.y)};
  F.yp = V2{beta_rho(rc.x, rn.x), beta_rho(rc.y, rn.y)};
  F.zm = V2{beta_rho(rd.x, rc.x), beta_rho(rd.y, rc.y)};
  F.zp = V2{beta_rho(rc.x, ru.x), beta_rho(rc.y, ru.y)};
  return F;
}

// Where the face coefficients of a grid come from: the stored arrays bx, by, bz, or
// (finest grid of a hierarchy built from rho, FP64) the density form rt.
template <typename T>
struct Coefs {
  const T* bx;
  const T* by;
  const T* bz;
  const T* rt;
};

// Residuals r = (f - fs) - h^-2 sum_f beta_f (p_nb - p_c) of the x-neighbour pair
// (i, j, k), (i+1, j, k) with i even, 0 on inactive cells.  All loads but the two
// outer x neighbours are 2-wide and contiguous across adjacent threads.
template <typename T, bool RHO>
__device__ __forceinline__ void pair_residual(const T* __restrict__ p, const T* __restrict__ f, const Coefs<T>& K,
                                              int i, int j, int k, int q, T inv_h2, T fs, T& r0, T& r1) {
  using V2 = typename V2of<T>::type;
  const int m = (1 << q) - 1, nn = 1 << (2 * q);
  const int c = cell(i, j, k, q);
  const V2 pc = ld2(p, c);
  const T pl = p[cell((i - 1) & m, j, k, q)], pr = p[cell((i + 2) & m, j, k, q)];
  const V2 pyd = ld2(p, cell(i, (j - 1) & m, k, q)), pyu = ld2(p, cell(i, (j + 1) & m, k, q));
  const V2 pzd = k > 0 ? ld2(p, c - nn) : pc;
  const V2 pzu = k < m ? ld2(p, c + nn) : pc;
  const V2 fv = f ? ld2(f, c) : V2{T(0), T(0)};
  PairFaces<T> F;
  if constexpr (RHO)
    F = pair_faces_rho(K.rt, i, j, k, q);
  else
    F = pair_faces(K.bx, K.by, K.bz, i, j, k, q);
  const T D0 = F.x0 + F.x1 + F.ym.x + F.yp.x + F.zm.x + F.zp.x;
  const T D1 = F.x1 + F.x2 + F.ym.y + F.yp.y + F.zm.y + F.zp.y;
  // explicit fused multiply-adds: the rounding is fixed by the source, so both forms
  // of the coefficients give the same bits
  const T s0 = fmad(F.zp.x, pzu.x - pc.x, fmad(F.zm.x, pzd.x - pc.x, fmad(F.yp.x, pyu.x - pc.x,
               fmad(F.ym.x, pyd.x - pc.x, fmad(F.x1, pc.y - pc.x, F.x0 * (pl - pc.x))))));
  const T s1 = fmad(F.zp.y, pzu.y - pc.y, fmad(F.zm.y, pzd.y - pc.y, fmad(F.yp.y, pyu.y - pc.y,
               fmad(F.ym.y, pyd.y - pc.y, fmad(F.x2, pr - pc.y, F.x1 * (pc.x - pc.y))))));
  r0 = D0 > T(0) ? fmad(-inv_h2, s0, fv.x - fs) : T(0);
  r1 = D1 > T(0) ? fmad(-inv_h2, s1, fv.y - fs) : T(0);
}

// ----------------------------------------------------------------------------- setup

__global__ __launch_bounds__(kBlock) void k_coeffs_from_rho(const double* __restrict__ rho,
                                                            const uint8_t* __restrict__ mask, int q,
                                                            double* __restrict__ bx, double* __restrict__ by,
                                                            double* __restrict__ bz) {
  const int n = 1 << q, m = n - 1;
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
  const bool mc = mask[c] != 0;
  const int cx = cell((i - 1) & m, j, k, q), cy = cell(i, (j - 1) & m, k, q);
  const int cz = c - (1 << (2 * q));
  const bool ox = mc && mask[cx], oy = mc && mask[cy], oz = k > 0 && mc && mask[cz];
  if (!rho) {   // open-face areas only
    bx[c] = ox ? 1.0 : 0.0;
    by[c] = oy ? 1.0 : 0.0;
    bz[c] = oz ? 1.0 : 0.0;
    return;
  }
  bx[c] = ox ? face_beta(rho[c], rho[cx]) : 0.0;
  by[c] = oy ? face_beta(rho[c], rho[cy]) : 0.0;
  bz[c] = oz ? face_beta(rho[c], rho[cz]) : 0.0;
}

// Density moved cell centre to cell centre: mean over the active children, 1 when
// there is none (such a coarse cell has only closed faces).
// density form of the finest coefficients: rt = rho on active cells, +inf elsewhere
__global__ __launch_bounds__(kBlock) void k_rho_tilde(const double* __restrict__ rho, const uint8_t* __restrict__ mask,
                                                      int total, double* __restrict__ rt) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= total) return;
  rt[c] = mask[c] ? rho[c] : __builtin_huge_val();
}

__global__ __launch_bounds__(kBlock) void k_restrict_rho(const double* __restrict__ rho, const uint8_t* __restrict__ mask,
                                                         int qc, double* __restrict__ crho) {
  const int mc = (1 << qc) - 1, q = qc + 1;
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * qc))) return;
  const int C = static_cast<int>(t);
  const int I = C & mc, J = (C >> qc) & mc, K = C >> (2 * qc);
  double sum = 0.0;
  int cnt = 0;
  for (int d = 0; d < 8; ++d) {
    const int c = cell(2 * I + (d & 1), 2 * J + ((d >> 1) & 1), 2 * K + (d >> 2), q);
    if (mask[c]) {
      sum += rho[c];
      ++cnt;
    }
  }
  crho[C] = cnt ? sum / cnt : 1.0;
}

// beta = area * 2 / (rho_L + rho_R) in place (closed faces stay 0)
__global__ __launch_bounds__(kBlock) void k_area_to_beta(const double* __restrict__ rho, int q, double* __restrict__ bx,
                                                         double* __restrict__ by, double* __restrict__ bz) {
  const int m = (1 << q) - 1;
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
  const double ax = bx[c], ay = by[c], az = bz[c];
  if (ax != 0.0) bx[c] = ax * face_beta(rho[c], rho[cell((i - 1) & m, j, k, q)]);
  if (ay != 0.0) by[c] = ay * face_beta(rho[c], rho[cell(i, (j - 1) & m, k, q)]);
  if (az != 0.0) bz[c] = az * face_beta(rho[c], rho[c - (1 << (2 * q))]);
}

// Close the finest faces (copy unless bx is null), validate them, mark active cells.
// Grid-stride over cells with a bounded block count, so the three counters take few
// atomic adds.
__global__ __launch_bounds__(kBlock) void k_setup_fine(const double* __restrict__ ubx, const double* __restrict__ uby,
                                                       const double* __restrict__ ubz,
                                                       const uint8_t* __restrict__ umask, int q,
                                                       double* __restrict__ bx, double* __restrict__ by,
                                                       double* __restrict__ bz, uint8_t* __restrict__ mask,
                                                       long long* __restrict__ counters) {
  const int n = 1 << q, m = n - 1;
  const int total = 1 << (3 * q);
  const int nn = 1 << (2 * q);
  int bad = 0, active = 0, dropped = 0;
  for (int c = blockIdx.x * kBlock + threadIdx.x; c < total; c += gridDim.x * kBlock) {
    const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
    const bool mc = umask[c] != 0;
    const int cxm = cell((i - 1) & m, j, k, q), cxp = cell((i + 1) & m, j, k, q);
    const int cym = cell(i, (j - 1) & m, k, q), cyp = cell(i, (j + 1) & m, k, q);
    const double vx = ubx[c], vy = uby[c], vz = ubz[c];
    bad += !(vx >= 0.0 && vx <= 1.7976931348623157e308) + !(vy >= 0.0 && vy <= 1.7976931348623157e308) +
           !(vz >= 0.0 && vz <= 1.7976931348623157e308);
    const double xm = (mc && umask[cxm]) ? vx : 0.0;
    const double ym = (mc && umask[cym]) ? vy : 0.0;
    const double zm = (k > 0 && mc && umask[c - nn]) ? vz : 0.0;
    const double xp = (mc && umask[cxp]) ? ubx[cxp] : 0.0;
    const double yp = (mc && umask[cyp]) ? uby[cyp] : 0.0;
    const double zp = (k < m && mc && umask[c + nn]) ? ubz[c + nn] : 0.0;
    if (bx) {
      bx[c] = xm;
      by[c] = ym;
      bz[c] = zm;
    }
    const bool act = mc && (xm + xp + ym + yp + zm + zp) > 0.0;
    mask[c] = act ? 1 : 0;
    active += act;
    dropped += mc && !act;
  }
  __shared__ int red[3][kBlock / 64];
  int v[3] = {bad, active, dropped};
  for (int x = 0; x < 3; ++x)
    for (int off = 32; off > 0; off >>= 1) v[x] += __shfl_xor(v[x], off, 64);
  if ((threadIdx.x & 63) == 0)
    for (int x = 0; x < 3; ++x) red[x][threadIdx.x >> 6] = v[x];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int x = 0; x < 3; ++x) {
      long long sum = 0;
      for (int w = 0; w < kBlock / 64; ++w) sum += red[x][w];
      if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(&counters[x]), static_cast<unsigned long long>(sum));
    }
  }
}

// The finest grid of a hierarchy built from rho in one pass: the face products
// beta = 2 / (rho_L + rho_R) on faces between fluid cells (0 elsewhere and on the
// bottom wall), their validation, the active cells (fluid with an open face) and the
// density form rt (rho on active cells, +inf elsewhere).  The same values as
// k_coeffs_from_rho, then k_setup_fine and k_rho_tilde: each face, the low ones stored
// and the high ones summed into the diagonal, is face_beta of the same two densities.
__global__ __launch_bounds__(kBlock) void k_setup_from_rho(const double* __restrict__ rho,
                                                           const uint8_t* __restrict__ umask, int q,
                                                           double* __restrict__ bx, double* __restrict__ by,
                                                           double* __restrict__ bz, uint8_t* __restrict__ mask,
                                                           double* __restrict__ rt, long long* __restrict__ counters) {
  const int n = 1 << q, m = n - 1;
  const int total = 1 << (3 * q);
  const int nn = 1 << (2 * q);
  int bad = 0, active = 0, dropped = 0;
  auto ok = [](double v) { return v >= 0.0 && v <= 1.7976931348623157e308; };
  for (int c = blockIdx.x * kBlock + threadIdx.x; c < total; c += gridDim.x * kBlock) {
    const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
    const bool mc = umask[c] != 0;
    const int cxm = cell((i - 1) & m, j, k, q), cxp = cell((i + 1) & m, j, k, q);
    const int cym = cell(i, (j - 1) & m, k, q), cyp = cell(i, (j + 1) & m, k, q);
    const double rc = rho[c];
    const double xm = (mc && umask[cxm]) ? face_beta(rc, rho[cxm]) : 0.0;
    const double ym = (mc && umask[cym]) ? face_beta(rc, rho[cym]) : 0.0;
    const double zm = (k > 0 && mc && umask[c - nn]) ? face_beta(rc, rho[c - nn]) : 0.0;
    const double xp = (mc && umask[cxp]) ? face_beta(rho[cxp], rc) : 0.0;
    const double yp = (mc && umask[cyp]) ? face_beta(rho[cyp], rc) : 0.0;
    const double zp = (k < m && mc && umask[c + nn]) ? face_beta(rho[c + nn], rc) : 0.0;
    bad += !ok(xm) + !ok(ym) + !ok(zm);
    bx[c] = xm;
    by[c] = ym;
    bz[c] = zm;
    const bool act = mc && (xm + xp + ym + yp + zm + zp) > 0.0;
    mask[c] = act ? 1 : 0;
    rt[c] = act ? rc : __builtin_huge_val();
    active += act;
    dropped += mc && !act;
  }
  __shared__ int red[3][kBlock / 64];
  int v[3] = {bad, active, dropped};
  for (int x = 0; x < 3; ++x)
    for (int off = 32; off > 0; off >>= 1) v[x] += __shfl_xor(v[x], off, 64);
  if ((threadIdx.x & 63) == 0)
    for (int x = 0; x < 3; ++x) red[x][threadIdx.x >> 6] = v[x];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int x = 0; x < 3; ++x) {
      long long sum = 0;
      for (int w = 0; w < kBlock / 64; ++w) sum += red[x][w];
      if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(&counters[x]), static_cast<unsigned long long>(sum));
    }
  }
}

// Coarse face = mean of the 4 fine faces it covers; coarse cell active if any child is
// active and it keeps an open face.  One thread per coarse cell.
__global__ __launch_bounds__(kBlock) void k_coarsen(const double* __restrict__ bx, const double* __restrict__ by,
                                                    const double* __restrict__ bz, const uint8_t* __restrict__ mask,
                                                    int qc, double* __restrict__ cbx, double* __restrict__ cby,
                                                    double* __restrict__ cbz, uint8_t* __restrict__ cmask) {
  const int nc = 1 << qc, mc = nc - 1, q = qc + 1, mf = (1 << q) - 1;
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * qc))) return;
  const int C = static_cast<int>(t);
  const int I = C & mc, J = (C >> qc) & mc, K = C >> (2 * qc);
  const int i = 2 * I, j = 2 * J, k = 2 * K;
  auto fx = [&](int ii) {   // x face at fine column ii (wrapped), 2 x 2 in (j, k)
    ii &= mf;
    return 0.25 * (bx[cell(ii, j, k, q)] + bx[cell(ii, j + 1, k, q)] + bx[cell(ii, j, k + 1, q)] +
                   bx[cell(ii, j + 1, k + 1, q)]);
  };
  auto fy = [&](int jj) {
    jj &= mf;
    return 0.25 * (by[cell(i, jj, k, q)] + by[cell(i + 1, jj, k, q)] + by[cell(i, jj, k + 1, q)] +
                   by[cell(i + 1, jj, k + 1, q)]);
  };
  auto fz = [&](int kk) {
    return 0.25 * (bz[cell(i, j, kk, q)] + bz[cell(i + 1, j, kk, q)] + bz[cell(i, j + 1, kk, q)] +
                   bz[cell(i + 1, j + 1, kk, q)]);
  };
  const double xm = fx(i), ym = fy(j), zm = fz(k);
  const double xp = fx(i + 2), yp = fy(j + 2), zp = K < mc ? fz(k + 2) : 0.0;
  cbx[C] = xm;
  cby[C] = ym;
  cbz[C] = zm;
  bool any = false;
  for (int d = 0; d < 8; ++d) any |= mask[cell(i + (d & 1), j + ((d >> 1) & 1), k + (d >> 2), q)] != 0;
  cmask[C] = (any && (xm + xp + ym + yp + zm + zp) > 0.0) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_to_f32(const double* __restrict__ src, float* __restrict__ dst,
                                                   long long count) {
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t < count) dst[t] = static_cast<float>(src[t]);
}

// --------------------------------------------------------------------------- V-cycle

// Gauss-Seidel on one colour, in place: each cell of that colour only reads cells of
// the other colour, so the update order inside the launch does not matter.
// One thread per pair of x-neighbours (one cell of each colour).
template <typename T>
__device__ __forceinline__ void gs_pair(T* __restrict__ p, const T* __restrict__ f, const T* __restrict__ bx,
                                        const T* __restrict__ by, const T* __restrict__ bz, int q, T h2, int colour,
                                        T fs, int pr) {
  const int m = (1 << q) - 1;
  const int ip = pr & (m >> 1), j = (pr >> (q - 1)) & m, k = pr >> (2 * q - 1);
  const int i = 2 * ip + ((colour + j + k) & 1);
  const Faces<T> F = load_faces(bx, by, bz, i, j, k, q);
  const int c = cell(i, j, k, q);
  // every load issued before the activity test, so they are in flight together
  const T pxm = p[F.cxm], pxp = p[F.cxp], pym = p[F.cym], pyp = p[F.cyp], pzm = p[F.czm], pzp = p[F.czp];
  const T fc = f[c];
  const T D = diag(F);
  if (!(D > T(0))) return;
  const T S = F.xm * pxm + F.xp * pxp + F.ym * pym + F.yp * pyp + F.zm * pzm + F.zp * pzp;
  p[c] = gs_quotient(S - h2 * (fc - fs), D);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rbgs_half(T* __restrict__ p, const T* __restrict__ f,
                                                      const T* __restrict__ bx, const T* __restrict__ by,
                                                      const T* __restrict__ bz, int q, T h2, int colour,
                                                      const double* __restrict__ fshift) {
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * q - 1))) return;
  const T fs = fshift ? static_cast<T>(*fshift) : T(0);
  gs_pair(p, f, bx, by, bz, q, h2, colour, fs, static_cast<int>(t));
}

// fc = mean over the 8 children of r = (f - fshift) - A p; ec = 0.  One thread per
// coarse cell: its children are two x-pairs on each of two rows and two planes.
template <typename T, bool RHO>
__device__ __forceinline__ void restrict_cell(const T* __restrict__ p, const T* __restrict__ f, const Coefs<T>& K,
                                              int q, T inv_h2, T fs, T* __restrict__ fc, T* __restrict__ ec, int C) {
  const int qc = q - 1, mc = (1 << qc) - 1;
  const int I = C & mc, J = (C >> qc) & mc, Kz = C >> (2 * qc);
  T sum = T(0);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    T r0, r1;
    pair_residual<T, RHO>(p, f, K, 2 * I, 2 * J + (d & 1), 2 * Kz + (d >> 1), q, inv_h2, fs, r0, r1);
    sum += r0 + r1;
  }
  fc[C] = sum * T(0.125);
  ec[C] = T(0);
}

template <typename T, bool RHO>
__global__ __launch_bounds__(kBlock) void k_residual_restrict(const T* __restrict__ p, const T* __restrict__ f,
                                                              Coefs<T> K, int q, T inv_h2,
                                                              const double* __restrict__ fshift,
                                                              T* __restrict__ fc, T* __restrict__ ec) {
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * (q - 1)))) return;
  const T fs = fshift ? static_cast<T>(*fshift) : T(0);
  restrict_cell<T, RHO>(p, f, K, q, inv_h2, fs, fc, ec, static_cast<int>(t));
}

// p += mask * trilinear(ec); 1-D weights 3/4 (parent) and 1/4 (nearer neighbour),
// periodic in x and y, parent reused for a z neighbour outside the grid.  One thread
// per coarse cell updates its 8 children (x-pairs on two rows of two planes), applying
// the 1-D weights in x, then y, then z, each as one fused multiply-add (3/4 a + (1/4 b),
// the second product exact), so that the rounding is fixed by the source.
template <typename T>
__device__ __forceinline__ void prolong_cell(const T* __restrict__ ec, T* __restrict__ p,
                                             const uint8_t* __restrict__ mask, int q, int C) {
  using V2 = typename V2of<T>::type;
  const int qc = q - 1, mc = (1 << qc) - 1;
  const int I = C & mc, J = (C >> qc) & mc, K = C >> (2 * qc);
  const int Ix[3] = {(I - 1) & mc, I, (I + 1) & mc};
  const int Jy[3] = {(J - 1) & mc, J, (J + 1) & mc};
  const int Kz[3] = {K > 0 ? K - 1 : K, K, K < mc ? K + 1 : K};
  const T w3 = T(0.75), w1 = T(0.25);
  // x interpolation on the 3 x 3 coarse rows around (J, K): even child uses I-1, odd I+1
  T ax[3][3][2];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int row = cell(0, Jy[a], Kz[b], qc);
      const T e0 = ec[row + Ix[0]], e1 = ec[row + Ix[1]], e2 = ec[row + Ix[2]];
      ax[b][a][0] = fmad(w3, e1, w1 * e0);
      ax[b][a][1] = fmad(w3, e1, w1 * e2);
    }
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int kk = 2 * K + dz, jj = 2 * J + dy;
      const int c = cell(2 * I, jj, kk, q);
      const uchar2 mk = *reinterpret_cast<const uchar2*>(mask + c);
      if (!(mk.x | mk.y)) continue;
      V2 v = *reinterpret_cast<const V2*>(p + c);
      T out[2];
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int ay = dy ? 2 : 0, bz_ = dz ? 2 : 0;   // nearer neighbour row / plane
        const T lo = fmad(w3, ax[1][1][dx], w1 * ax[1][ay][dx]);
        const T hi = fmad(w3, ax[bz_][1][dx], w1 * ax[bz_][ay][dx]);
        out[dx] = fmad(w3, lo, w1 * hi);
      }
      if (mk.x) v.x += out[0];
      if (mk.y) v.y += out[1];
      *reinterpret_cast<V2*>(p + c) = v;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(const T* __restrict__ ec, T* __restrict__ p,
                                                        const uint8_t* __restrict__ mask, int q) {
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * (q - 1)))) return;
  prolong_cell(ec, p, mask, q, static_cast<int>(t));
}

// e = A_c^+ (f - active mean of f) on the 4^3 grid, in FP64, by the first wavefront
// (64 lanes) of the calling block; fh is a 64-double shared buffer.
template <typename T>
__device__ __forceinline__ void coarse_solve_wave(const T* __restrict__ f, T* __restrict__ e,
                                                  const double* __restrict__ pinv, const uint8_t* __restrict__ mask,
                                                  double* fh) {
  const int t = threadIdx.x;
  if (t < 64) {
    const bool act = mask[t] != 0;
    const double v = act ? static_cast<double>(f[t]) : 0.0;
    double s = v, cnt = act ? 1.0 : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
      s += __shfl_xor(s, off, 64);
      cnt += __shfl_xor(cnt, off, 64);
    }
    const double mean = cnt > 0.0 ? s / cnt : 0.0;
    fh[t] = act ? v - mean : 0.0;
  }
  __syncthreads();
  if (t < 64) {
    double acc = 0.0;
    for (int c = 0; c < 64; ++c) acc += pinv[t * 64 + c] * fh[c];
    e[t] = static_cast<T>(acc);
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_coarse_solve(const T* __restrict__ f, T* __restrict__ e,
                                                     const double* __restrict__ pinv,
                                                     const uint8_t* __restrict__ mask) {
  __shared__ double fh[64];
  coarse_solve_wave(f, e, pinv, mask, fh);
}

// The whole V(2,2) sub-cycle on grids of 16^3 and smaller, by one workgroup: the same
// per-cell steps as the multi-block kernels, separated by workgroup barriers instead of
// kernel launches.  The corrections and right-hand sides of every grid live in LDS
// (75 KB in FP64 for 16^3 + 8^3 + 4^3); only the coefficients and masks are read from
// memory.  Level 0 of `a` enters with its right-hand side and its correction (zero, or
// the current iterate when it is the finest grid) and gets the result back.  The level
// loops are unrolled over the at most three grids so every field of `a` is read with a
// constant index.
constexpr int kCoarseThreads = 512;
constexpr int kCoarseCells = 4096 + 512 + 64;

// e = A_c^+ (f - active mean of f) on the 4^3 grid in FP64 by the whole block: the mean
// by the first wavefront, then each row of the pseudo-inverse product by 8 threads.
template <typename T>
__device__ __forceinline__ void coarse_solve_block(const T* f, T* e, const double* __restrict__ pinv,
                                                   const uint8_t* __restrict__ mask, double* fh) {
  const int t = threadIdx.x;
  if (t < 64) {
    const bool act = mask[t] != 0;
    const double v = act ? static_cast<double>(f[t]) : 0.0;
    double s = v, cnt = act ? 1.0 : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
      s += __shfl_xor(s, off, 64);
      cnt += __shfl_xor(cnt, off, 64);
    }
    const double mean = cnt > 0.0 ? s / cnt : 0.0;
    fh[t] = act ? v - mean : 0.0;
  }
  const int row = t >> 3, part = t & 7;
  double pv[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) pv[c] = pinv[row * 64 + part * 8 + c];   // issued before the barrier
  __syncthreads();
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) acc = __builtin_fma(pv[c], fh[part * 8 + c], acc);
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  acc += __shfl_xor(acc, 4, 64);
  if (part == 0) e[row] = static_cast<T>(acc);
}

template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_cycle(CoarseCycle<T> a) {
  static_assert(kCoarseThreads == 512, "the pseudo-inverse product maps 64 rows x 8 threads");
  __shared__ double fh[64];
  __shared__ T se[kCoarseCells];
  __shared__ T sf[kCoarseCells];
  const int tid = threadIdx.x;
  const int last = a.nlev - 1;
  // LDS arrays of each grid
  T* e[3];
  T* f[3];
  {
    int off = 0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      e[l] = se + off;
      f[l] = sf + off;
      if (l < a.nlev) off += 1 << (3 * a.q[l]);
    }
  }
  const int n0 = 1 << (3 * a.q[0]);
  for (int c = tid; c < n0; c += kCoarseThreads) {
    e[0][c] = a.e[0][c];
    f[0][c] = a.f[0][c];
  }
  __syncthreads();
  // The face coefficients of the cells this thread updates on the grids that are
  // smoothed, loaded once (every half-sweep would otherwise wait for them from L2 again):
  // on the first grid in FP32, on the second in both precisions.  Pair slot u of grid l
  // is pair tid + u x 512 (at most 4 on a 16^3 grid), colour 0 / 1 its red / black cell.
  // FP64 reads the first grid's from L2 in each half-sweep, all of a thread's pairs at
  // once: held in registers they would spill.
  constexpr bool PRE = sizeof(T) == 4;
  constexpr int U0 = (kCoarseCycleMaxN * kCoarseCycleMaxN * kCoarseCycleMaxN / 2) / kCoarseThreads;
  struct CF {
    T xm, xp, ym, yp, zm, zp;
  };
  CF cf0[U0][2], cf1[2];
  auto pair_cell = [&](int l, int pr, int colour, int& i, int& j, int& k) {
    const int q = a.q[l], m = (1 << q) - 1;
    const int ip = pr & (m >> 1);
    j = (pr >> (q - 1)) & m;
    k = pr >> (2 * q - 1);
    i = 2 * ip + ((colour + j + k) & 1);
  };
  auto load_cf = [&](int l, int pr, int colour) {
    int i, j, k;
    pair_cell(l, pr, colour, i, j, k);
    const Faces<T> F = load_faces(a.bx[l], a.by[l], a.bz[l], i, j, k, a.q[l]);
    return CF{F.xm, F.xp, F.ym, F.yp, F.zm, F.zp};
  };
  auto preload0 = [&]() {
    if constexpr (!PRE) return;
#pragma unroll
    for (int u = 0; u < U0; ++u) {
      const int pr = tid + u * kCoarseThreads;
      if (last > 0 && pr < (1 << (3 * a.q[0] - 1))) {
        cf0[u][0] = load_cf(0, pr, 0);
        cf0[u][1] = load_cf(0, pr, 1);
      }
    }
  };
  preload0();
  if (last > 1 && tid < (1 << (3 * a.q[1] - 1))) {   // the second grid's: both precisions
    cf1[0] = load_cf(1, tid, 0);
    cf1[1] = load_cf(1, tid, 1);
  }
  // the update of gs_pair with preloaded coefficients (same operations, same order)
  auto gs_pre = [&](int l, int pr, int colour, const CF& C, T fs) {
    const int q = a.q[l], n = 1 << q, m = n - 1;
    int i, j, k;
    pair_cell(l, pr, colour, i, j, k);
    const int c = cell(i, j, k, q);
    const int cxm = cell((i - 1) & m, j, k, q), cxp = cell((i + 1) & m, j, k, q);
    const int cym = cell(i, (j - 1) & m, k, q), cyp = cell(i, (j + 1) & m, k, q);
    const int czm = k > 0 ? c - (1 << (2 * q)) : c, czp = k < m ? c + (1 << (2 * q)) : c;
    T* p = e[l];
    const T pxm = p[cxm], pxp = p[cxp], pym = p[cym], pyp = p[cyp], pzm = p[czm], pzp = p[czp];
    const T fc = f[l][c];
    const T D = C.xm + C.xp + C.ym + C.yp + C.zm + C.zp;
    if (!(D > T(0))) return;
    const T S = C.xm * pxm + C.xp * pxp + C.ym * pym + C.yp * pyp + C.zm * pzm + C.zp * pzp;
    p[c] = gs_quotient(S - a.h2[l] * (fc - fs), D);
  };
  auto sweep = [&](int l, int colour, const T* bx, const T* by, const T* bz) {
    const T fs = (l == 0 && a.fshift) ? static_cast<T>(*a.fshift) : T(0);
    if (l == 1) {
      if (tid < (1 << (3 * a.q[1] - 1))) gs_pre(1, tid, colour, cf1[colour], fs);
    } else if constexpr (!PRE) {
      // a fixed trip count, unrolled, so that the coefficient loads of all of a thread's
      // pairs are in flight together
#pragma unroll
      for (int u = 0; u < U0; ++u) {
        const int pr = tid + u * kCoarseThreads;
        if (pr < (1 << (3 * a.q[0] - 1))) gs_pair(e[0], f[0], bx, by, bz, a.q[0], a.h2[0], colour, fs, pr);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U0; ++u) {
        const int pr = tid + u * kCoarseThreads;
        if (pr < (1 << (3 * a.q[0] - 1))) gs_pre(0, pr, colour, cf0[u][colour], fs);
      }
    }
    __syncthreads();
  };
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    if (l < last) {
      for (int s = 0; s < 2; ++s) {
        sweep(l, 0, a.bx[l], a.by[l], a.bz[l]);
        sweep(l, 1, a.bx[l], a.by[l], a.bz[l]);
      }
      const T fs = (l == 0 && a.fshift) ? static_cast<T>(*a.fshift) : T(0);
      for (int C = tid; C < (1 << (3 * (a.q[l] - 1))); C += kCoarseThreads)
        restrict_cell<T, false>(e[l], f[l], Coefs<T>{a.bx[l], a.by[l], a.bz[l], nullptr}, a.q[l], a.inv_h2[l], fs,
                                f[l + 1], e[l + 1], C);
      __syncthreads();
    }
  }
  const uint8_t* ml = last == 0 ? a.mask[0] : (last == 1 ? a.mask[1] : a.mask[2]);
  coarse_solve_block(f[last], e[last], a.pinv, ml, fh);
  __syncthreads();
#pragma unroll
  for (int l = 1; l >= 0; --l) {
    if (l < last) {
      // the first grid's coefficients again for its post-smoothing (not kept in
      // registers through the coarser grids), in flight during the prolongation
      if (l == 0) preload0();
      for (int C = tid; C < (1 << (3 * (a.q[l] - 1))); C += kCoarseThreads)
        prolong_cell(e[l + 1], e[l], a.mask[l], a.q[l], C);
      __syncthreads();
      for (int s = 0; s < 2; ++s) {
        sweep(l, 1, a.bx[l], a.by[l], a.bz[l]);
        sweep(l, 0, a.bx[l], a.by[l], a.bz[l]);
      }
    }
  }
  for (int c = tid; c < n0; c += kCoarseThreads) a.e[0][c] = e[0][c];
}

// ------------------------------------------------------------------ FP64 finest passes

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
  return s;   // valid in thread 0
}

template <bool RHO>
__global__ __launch_bounds__(kBlock) void k_residual_norm(const double* __restrict__ p, const double* __restrict__ f,
                                                          Coefs<double> K, int q, double inv_h2,
                                                          const double* __restrict__ fshift,
                                                          float* __restrict__ r32, float* __restrict__ e32,
                                                          double* __restrict__ r64, double* __restrict__ z64,
                                                          double* __restrict__ partials) {
  const int m = (1 << q) - 1;
  const int pairs = 1 << (3 * q - 1);
  const double fs = fshift ? *fshift : 0.0;
  double acc = 0.0;
  for (int t = blockIdx.x * kBlock + threadIdx.x; t < pairs; t += gridDim.x * kBlock) {
    const int i = 2 * (t & (m >> 1)), j = (t >> (q - 1)) & m, k = t >> (2 * q - 1);
    double r0, r1;
    pair_residual<double, RHO>(p, f, K, i, j, k, q, inv_h2, fs, r0, r1);
    acc = fmad(r1, r1, fmad(r0, r0, acc));
    const int c = cell(i, j, k, q);
    if (r32) *reinterpret_cast<float2*>(r32 + c) = float2{static_cast<float>(r0), static_cast<float>(r1)};
    if (e32) *reinterpret_cast<float2*>(e32 + c) = float2{0.0f, 0.0f};
    if (r64) *reinterpret_cast<double2*>(r64 + c) = double2{r0, r1};
    if (z64) *reinterpret_cast<double2*>(z64 + c) = double2{0.0, 0.0};
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_masked_sum(const double* __restrict__ x, const uint8_t* __restrict__ mask,
                                                       int total, int mode, const double* __restrict__ shift,
                                                       double* __restrict__ partials) {
  const double sh = (mode == 1 && shift) ? *shift : 0.0;
  double acc = 0.0;
  for (int c = blockIdx.x * kBlock + threadIdx.x; c < total; c += gridDim.x * kBlock) {
    if (mask[c]) {
      const double v = x[c] - sh;
      acc += mode == 1 ? v * v : v;
    }
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_reduce_final(const double* __restrict__ partials, int nparts,
                                                       double scale, double* __restrict__ out) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int t = threadIdx.x; t < nparts; t += 1024) s += partials[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

__global__ __launch_bounds__(kBlock) void k_gauge(double* __restrict__ p, const uint8_t* __restrict__ mask, int total,
                                                  const double* __restrict__ mean) {
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= total) return;
  const double mu = mean ? *mean : 0.0;
  p[t] = mask[t] ? p[t] - mu : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_update_p(double* __restrict__ p, const float* __restrict__ e32,
                                                     const uint8_t* __restrict__ mask, int total) {
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= total) return;
  if (mask[t]) p[t] += static_cast<double>(e32[t]);
}

__global__ __launch_bounds__(kBlock) void k_apply(const double* __restrict__ p, const double* __restrict__ bx,
                                                  const double* __restrict__ by, const double* __restrict__ bz,
                                                  int q, double inv_h2, double* __restrict__ Ap) {
  const int m = (1 << q) - 1;
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const Faces<double> F = load_faces(bx, by, bz, c & m, (c >> q) & m, c >> (2 * q), q);
  Ap[c] = inv_h2 * flux_sum(F, p, p[c]);
}

// dL/dbeta on the low faces of each cell and dL/drho_c = -1/2 sum_f beta_f^2 dL/dbeta_f;
// high faces are recomputed from the neighbours so no thread waits on another.
__global__ __launch_bounds__(kBlock) void k_coeff_grad(const double* __restrict__ mu, const double* __restrict__ p,
                                                       int batch, const double* __restrict__ bx,
                                                       const double* __restrict__ by,
                                                       const double* __restrict__ bz,
                                                       const uint8_t* __restrict__ mask, int q, double inv_h2,
                                                       double* __restrict__ gbx, double* __restrict__ gby,
                                                       double* __restrict__ gbz, double* __restrict__ grho) {
  const int m = (1 << q) - 1;
  const long long total = 1LL << (3 * q);
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= total) return;
  const int c = static_cast<int>(t);
  const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
  const int nb[6] = {cell((i - 1) & m, j, k, q), cell((i + 1) & m, j, k, q), cell(i, (j - 1) & m, k, q),
                     cell(i, (j + 1) & m, k, q), k > 0 ? c - (1 << (2 * q)) : c,
                     k < m ? c + (1 << (2 * q)) : c};
  const bool mc = mask[c] != 0;
  bool open[6];
  for (int f = 0; f < 6; ++f) open[f] = mc && mask[nb[f]] != 0;
  open[4] = open[4] && k > 0;
  open[5] = open[5] && k < m;
  double g[6] = {0, 0, 0, 0, 0, 0};
  for (int b = 0; b < batch; ++b) {
    const double* mb = mu + static_cast<long long>(b) * total;
    const double* pb = p + static_cast<long long>(b) * total;
    const double mcv = mb[c], pcv = pb[c];
    for (int f = 0; f < 6; ++f)
      if (open[f]) g[f] += (mb[nb[f]] - mcv) * (pb[nb[f]] - pcv);
  }
  for (int f = 0; f < 6; ++f) g[f] *= inv_h2;
  if (gbx) gbx[c] = g[0];
  if (gby) gby[c] = g[2];
  if (gbz) gbz[c] = g[4];
  if (grho) {
    const double b[6] = {bx[c], bx[nb[1]], by[c], by[nb[3]], bz[c], k < m ? bz[nb[5]] : 0.0};
    double s = 0.0;
    for (int f = 0; f < 6; ++f) s += b[f] * b[f] * g[f];
    grho[c] = -0.5 * s;
  }
}

// ---------------------------------------------------------- flexible CG (finest grid, FP64)
// Vectors are zero on inactive cells.  All loops run over x-pairs with 2-wide loads
// and end in the fixed-order two-pass block sums.

// w = A d, partial sums of d.w and d.r
template <bool RHO>
__global__ __launch_bounds__(kBlock) void k_fcg_aw(const double* __restrict__ d, const double* __restrict__ r,
                                                   Coefs<double> K, int q, double inv_h2,
                                                   double* __restrict__ w, double* __restrict__ part_dw,
                                                   double* __restrict__ part_dr) {
  const int m = (1 << q) - 1;
  const int pairs = 1 << (3 * q - 1);
  double dw = 0.0, dr = 0.0;
  for (int t = blockIdx.x * kBlock + threadIdx.x; t < pairs; t += gridDim.x * kBlock) {
    const int i = 2 * (t & (m >> 1)), j = (t >> (q - 1)) & m, k = t >> (2 * q - 1);
    double a0, a1;
    // the residual of f = 0 is -A d
    pair_residual<double, RHO>(d, nullptr, K, i, j, k, q, inv_h2, 0.0, a0, a1);
    const int c = cell(i, j, k, q);
    const double2 dv = ld2(d, c), rv = ld2(r, c);
    const double2 wv = double2{-a0, -a1};
    *reinterpret_cast<double2*>(w + c) = wv;
    dw = fmad(dv.y, wv.y, fmad(dv.x, wv.x, dw));
    dr = fmad(dv.y, rv.y, fmad(dv.x, rv.x, dr));
  }
  const double s1 = block_sum(dw);
  const double s2 = block_sum(dr);
  if (threadIdx.x == 0) {
    part_dw[blockIdx.x] = s1;
    part_dr[blockIdx.x] = s2;
  }
}

// alpha = dr / dw (kept in *s_alpha for the deferred update of p);  r -= alpha w;
// partial ||r||^2.  Leaves the next preconditioner input ready: FP64 z = 0, or FP32
// r32 = r and e32 = 0.
__global__ __launch_bounds__(kBlock) void k_fcg_rupdate(double* __restrict__ r, const double* __restrict__ w,
                                                        const double* __restrict__ s_dr,
                                                        const double* __restrict__ s_dw,
                                                        double* __restrict__ s_alpha, int total,
                                                        double* __restrict__ z_zero, float* __restrict__ r32,
                                                        float* __restrict__ e32_zero, double* __restrict__ part_rr) {
  const double alpha = *s_dr / *s_dw;
  if (blockIdx.x == 0 && threadIdx.x == 0) *s_alpha = alpha;
  double rr = 0.0;
  for (int c = 2 * (blockIdx.x * kBlock + threadIdx.x); c < total; c += 2 * gridDim.x * kBlock) {
    double2 rv = ld2(r, c);
    const double2 wv = ld2(w, c);
    rv.x -= alpha * wv.x;
    rv.y -= alpha * wv.y;
    *reinterpret_cast<double2*>(r + c) = rv;
    rr += rv.x * rv.x + rv.y * rv.y;
    if (r32) *reinterpret_cast<float2*>(r32 + c) = float2{static_cast<float>(rv.x), static_cast<float>(rv.y)};
    if (e32_zero) *reinterpret_cast<float2*>(e32_zero + c) = float2{0.0f, 0.0f};
    if (z_zero) *reinterpret_cast<double2*>(z_zero + c) = double2{0.0, 0.0};
  }
  const double s = block_sum(rr);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
}

// p += alpha d (the last step's update of the solution)
__global__ __launch_bounds__(kBlock) void k_fcg_padd(double* __restrict__ p, const double* __restrict__ d,
                                                     const double* __restrict__ s_alpha, int total) {
  const double alpha = *s_alpha;
  const long long c = 2 * (static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x);
  if (c >= total) return;
  const double2 pv = ld2(p, static_cast<int>(c)), dv = ld2(d, static_cast<int>(c));
  *reinterpret_cast<double2*>(p + c) = double2{fmad(alpha, dv.x, pv.x), fmad(alpha, dv.y, pv.y)};
}

__global__ __launch_bounds__(kBlock) void k_fcg_padd2(double* __restrict__ p, const double* __restrict__ d0,
                                                      const double* __restrict__ s_alpha0, const double* __restrict__ d,
                                                      const double* __restrict__ s_alpha, int total) {
  const double alpha0 = *s_alpha0, alpha = *s_alpha;
  const long long c = 2 * (static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x);
  if (c >= total) return;
  const double2 pv = ld2(p, static_cast<int>(c)), ov = ld2(d0, static_cast<int>(c)), dv = ld2(d, static_cast<int>(c));
  *reinterpret_cast<double2*>(p + c) =
      double2{fmad(alpha, dv.x, fmad(alpha0, ov.x, pv.x)), fmad(alpha, dv.y, fmad(alpha0, ov.y, pv.y))};
}

// partial sums of z.w, z in FP64 (z64) or FP32 (z32)
__global__ __launch_bounds__(kBlock) void k_fcg_zw(const double* __restrict__ z64, const float* __restrict__ z32,
                                                   const double* __restrict__ w, int total,
                                                   double* __restrict__ part) {
  double acc = 0.0;
  for (int c = 2 * (blockIdx.x * kBlock + threadIdx.x); c < total; c += 2 * gridDim.x * kBlock) {
    const double2 wv = ld2(w, c);
    double2 zv;
    if (z64) {
      zv = ld2(z64, c);
    } else {
      const float2 zf = *reinterpret_cast<const float2*>(z32 + c);
      zv = double2{static_cast<double>(zf.x), static_cast<double>(zf.y)};
    }
    acc += zv.x * wv.x + zv.y * wv.y;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// d = z + beta d with beta = -zw / dw (beta = 0 when s_zw is null: the first direction)
__global__ __launch_bounds__(kBlock) void k_fcg_dir(const double* __restrict__ z64, const float* __restrict__ z32,
                                                    const double* d, double* dn, double* p,
                                                    const double* __restrict__ s_zw, const double* __restrict__ s_dw,
                                                    const double* __restrict__ s_alpha, int total) {
  const double beta = s_zw ? -*s_zw / *s_dw : 0.0;
  const long long c = 2 * (static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x);
  if (c >= total) return;
  double2 zv;
  if (z64) {
    zv = ld2(z64, static_cast<int>(c));
  } else {
    const float2 zf = *reinterpret_cast<const float2*>(z32 + c);
    zv = double2{static_cast<double>(zf.x), static_cast<double>(zf.y)};
  }
  if (!s_zw) {   // the first direction (d is not read)
    *reinterpret_cast<double2*>(dn + c) = zv;
    return;
  }
  const double2 dv = *reinterpret_cast<const double2*>(d + c);
  if (p) {
    const double alpha = *s_alpha;
    const double2 pv = *reinterpret_cast<const double2*>(p + c);
    *reinterpret_cast<double2*>(p + c) = double2{fmad(alpha, dv.x, pv.x), fmad(alpha, dv.y, pv.y)};
  }
  *reinterpret_cast<double2*>(dn + c) = double2{fmad(beta, dv.x, zv.x), fmad(beta, dv.y, zv.y)};
}

// ------------------------------------------- Runge-Kutta stage around the solve (FP64)
// Face velocities use the low-face storage of the face coefficients.  A face is open
// when both cells are active (and it is not a z wall); closed faces carry no flux.

// f_c = div(U + dt R)_c / dt on active cells (R may be null)
__global__ __launch_bounds__(kBlock) void k_divergence(const double* __restrict__ ux, const double* __restrict__ uy,
                                                       const double* __restrict__ uz, const double* __restrict__ rx,
                                                       const double* __restrict__ ry, const double* __restrict__ rz,
                                                       double dt, const uint8_t* __restrict__ mask, int q,
                                                       double inv_hdt, double* __restrict__ f) {
  const int n = 1 << q, m = n - 1, nn = 1 << (2 * q);
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
  if (!mask[c]) {
    f[c] = 0.0;
    return;
  }
  const int cxp = cell((i + 1) & m, j, k, q), cxm = cell((i - 1) & m, j, k, q);
  const int cyp = cell(i, (j + 1) & m, k, q), cym = cell(i, (j - 1) & m, k, q);
  auto U = [&](const double* a, const double* r, int at) { return r ? a[at] + dt * r[at] : a[at]; };
  double div = 0.0;
  if (mask[cxp]) div += U(ux, rx, cxp);
  if (mask[cxm]) div -= U(ux, rx, c);
  if (mask[cyp]) div += U(uy, ry, cyp);
  if (mask[cym]) div -= U(uy, ry, c);
  if (k < m && mask[c + nn]) div += U(uz, rz, c + nn);
  if (k > 0 && mask[c - nn]) div -= U(uz, rz, c);
  f[c] = div * inv_hdt;
}

// U_f <- o_f (U_f + dt R_f - dt beta_f (p_hi - p_lo) / h) on the low faces of each cell
__global__ __launch_bounds__(kBlock) void k_project(double* __restrict__ ux, double* __restrict__ uy,
                                                    double* __restrict__ uz, const double* __restrict__ rx,
                                                    const double* __restrict__ ry, const double* __restrict__ rz,
                                                    double dt, const double* __restrict__ p,
                                                    const double* __restrict__ bx, const double* __restrict__ by,
                                                    const double* __restrict__ bz, const uint8_t* __restrict__ mask,
                                                    int q, double dt_over_h) {
  const int n = 1 << q, m = n - 1, nn = 1 << (2 * q);
  const long long t = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
  const bool mc = mask[c] != 0;
  const int cxm = cell((i - 1) & m, j, k, q), cym = cell(i, (j - 1) & m, k, q);
  const double pc = p[c];
  auto upd = [&](double* a, const double* r, const double* b, int lo, bool open) {
    a[c] = open ? (r ? a[c] + dt * r[c] : a[c]) - dt_over_h * b[c] * (pc - p[lo]) : 0.0;
  };
  upd(ux, rx, bx, cxm, mc && mask[cxm]);
  upd(uy, ry, by, cym, mc && mask[cym]);
  upd(uz, rz, bz, k > 0 ? c - nn : c, k > 0 && mc && mask[c - nn]);
}

int reduction_blocks(long long work) {
  long long b = (work + kBlock - 1) / kBlock;
  return static_cast<int>(b < kNumPartials ? b : kNumPartials);
}

}  // namespace

// ------------------------------------------------------------------------- launchers

hipError_t launch_coeffs_from_rho(const double* rho, const uint8_t* mask, int q, double* bx, double* by,
                                  double* bz, hipStream_t s) {
  hipLaunchKernelGGL(k_coeffs_from_rho, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, rho, mask, q, bx, by, bz);
  return hipGetLastError();
}

hipError_t launch_setup_fine(const double* ubx, const double* uby, const double* ubz, const uint8_t* umask, int q,
                             double* bx, double* by, double* bz, uint8_t* mask, long long* counters,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_setup_fine, dim3(reduction_blocks(1LL << (3 * q))), dim3(kBlock), 0, s, ubx, uby, ubz, umask, q,
                     bx, by, bz, mask, counters);
  return hipGetLastError();
}

hipError_t launch_setup_from_rho(const double* rho, const uint8_t* umask, int q, double* bx, double* by, double* bz,
                                 uint8_t* mask, double* rt, long long* counters, hipStream_t s) {
  hipLaunchKernelGGL(k_setup_from_rho, dim3(reduction_blocks(1LL << (3 * q))), dim3(kBlock), 0, s, rho, umask, q, bx,
                     by, bz, mask, rt, counters);
  return hipGetLastError();
}

hipError_t launch_rho_tilde(const double* rho, const uint8_t* mask, int q, double* rt, hipStream_t s) {
  hipLaunchKernelGGL(k_rho_tilde, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, rho, mask, 1 << (3 * q), rt);
  return hipGetLastError();
}

hipError_t launch_restrict_rho(const double* rho, const uint8_t* mask, int qc, double* crho, hipStream_t s) {
  hipLaunchKernelGGL(k_restrict_rho, dim3(grid_for(1LL << (3 * qc))), dim3(kBlock), 0, s, rho, mask, qc, crho);
  return hipGetLastError();
}

hipError_t launch_area_to_beta(const double* rho, int q, double* bx, double* by, double* bz, hipStream_t s) {
  hipLaunchKernelGGL(k_area_to_beta, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, rho, q, bx, by, bz);
  return hipGetLastError();
}

hipError_t launch_coarsen(const double* bx, const double* by, const double* bz, const uint8_t* mask, int qc,
                          double* cbx, double* cby, double* cbz, uint8_t* cmask, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsen, dim3(grid_for(1LL << (3 * qc))), dim3(kBlock), 0, s, bx, by, bz, mask, qc, cbx, cby,
                     cbz, cmask);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, long long count, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(count)), dim3(kBlock), 0, s, src, dst, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rbgs_half(T* p, const T* f, const T* bx, const T* by, const T* bz, int q, double h, int colour,
                            const double* fshift, hipStream_t s) {
  const T h2 = static_cast<T>(h * h);
  hipLaunchKernelGGL(k_rbgs_half<T>, dim3(grid_for(1LL << (3 * q - 1))), dim3(kBlock), 0, s, p, f, bx, by, bz, q,
                     h2, colour, fshift);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_residual_restrict(const T* p, const T* f, const T* bx, const T* by, const T* bz, const T* rt, int q,
                                    double h, const double* fshift, T* fc, T* ec, hipStream_t s) {
  const T inv_h2 = static_cast<T>(1.0 / (h * h));
  const Coefs<T> K{bx, by, bz, rt};
  const dim3 grid(grid_for(1LL << (3 * (q - 1))));
  if (rt)
    hipLaunchKernelGGL((k_residual_restrict<T, true>), grid, dim3(kBlock), 0, s, p, f, K, q, inv_h2, fshift, fc, ec);
  else
    hipLaunchKernelGGL((k_residual_restrict<T, false>), grid, dim3(kBlock), 0, s, p, f, K, q, inv_h2, fshift, fc, ec);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const T* ec, T* p, const uint8_t* mask, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_prolong_add<T>, dim3(grid_for(1LL << (3 * (q - 1)))), dim3(kBlock), 0, s, ec, p, mask, q);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve(const T* f, T* e, const double* pinv, const uint8_t* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(64), 0, s, f, e, pinv, mask);
  return hipGetLastError();
}

hipError_t launch_residual_norm(const double* p, const double* f, const double* bx, const double* by,
                                const double* bz, const double* rt, int q, double h, const double* fshift, float* r32,
                                float* e32, double* r64, double* z64, double* partials, int* nblocks,
                                hipStream_t s) {
  const int nb = reduction_blocks(1LL << (3 * q - 1));
  const Coefs<double> K{bx, by, bz, rt};
  if (rt)
    hipLaunchKernelGGL(k_residual_norm<true>, dim3(nb), dim3(kBlock), 0, s, p, f, K, q, 1.0 / (h * h), fshift, r32,
                       e32, r64, z64, partials);
  else
    hipLaunchKernelGGL(k_residual_norm<false>, dim3(nb), dim3(kBlock), 0, s, p, f, K, q, 1.0 / (h * h), fshift, r32,
                       e32, r64, z64, partials);
  *nblocks = nb;
  return hipGetLastError();
}

hipError_t launch_masked_sum(const double* x, const uint8_t* mask, int q, int mode, const double* shift,
                             double* partials, int* nblocks, hipStream_t s) {
  const int nb = reduction_blocks(1LL << (3 * q));
  hipLaunchKernelGGL(k_masked_sum, dim3(nb), dim3(kBlock), 0, s, x, mask, 1 << (3 * q), mode, shift, partials);
  *nblocks = nb;
  return hipGetLastError();
}

hipError_t launch_reduce_final(const double* partials, int nparts, double scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, s, partials, nparts, scale, out);
  return hipGetLastError();
}

hipError_t launch_gauge(double* p, const uint8_t* mask, int q, const double* mean, hipStream_t s) {
  hipLaunchKernelGGL(k_gauge, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, p, mask, 1 << (3 * q), mean);
  return hipGetLastError();
}

hipError_t launch_update_p(double* p, const float* e32, const uint8_t* mask, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, p, e32, mask, 1 << (3 * q));
  return hipGetLastError();
}

hipError_t launch_apply(const double* p, const double* bx, const double* by, const double* bz, int q, double h,
                        double* Ap, hipStream_t s) {
  hipLaunchKernelGGL(k_apply, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, p, bx, by, bz, q, 1.0 / (h * h), Ap);
  return hipGetLastError();
}

hipError_t launch_coeff_grad(const double* mu, const double* p, int batch, const double* bx, const double* by,
                             const double* bz, const uint8_t* mask, int q, double h, double* gbx, double* gby,
                             double* gbz, double* grho, hipStream_t s) {
  hipLaunchKernelGGL(k_coeff_grad, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, mu, p, batch, bx, by, bz, mask,
                     q, 1.0 / (h * h), gbx, gby, gbz, grho);
  return hipGetLastError();
}


hipError_t launch_fcg_aw(const double* d, const double* r, const double* bx, const double* by, const double* bz,
                         const double* rt, int q, double h, double* w, double* part_dw, double* part_dr, int* nblocks,
                         hipStream_t s) {
  const int nb = reduction_blocks(1LL << (3 * q - 1));
  const Coefs<double> K{bx, by, bz, rt};
  if (rt)
    hipLaunchKernelGGL(k_fcg_aw<true>, dim3(nb), dim3(kBlock), 0, s, d, r, K, q, 1.0 / (h * h), w, part_dw, part_dr);
  else
    hipLaunchKernelGGL(k_fcg_aw<false>, dim3(nb), dim3(kBlock), 0, s, d, r, K, q, 1.0 / (h * h), w, part_dw, part_dr);
  *nblocks = nb;
  return hipGetLastError();
}

hipError_t launch_fcg_rupdate(double* r, const double* w, const double* s_dr, const double* s_dw, double* s_alpha,
                              int q, double* z_zero, float* r32, float* e32_zero, double* part_rr, int* nblocks,
                              hipStream_t s) {
  const int nb = reduction_blocks(1LL << (3 * q - 1));
  hipLaunchKernelGGL(k_fcg_rupdate, dim3(nb), dim3(kBlock), 0, s, r, w, s_dr, s_dw, s_alpha, 1 << (3 * q), z_zero, r32,
                     e32_zero, part_rr);
  *nblocks = nb;
  return hipGetLastError();
}

hipError_t launch_fcg_padd(double* p, const double* d, const double* s_alpha, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_padd, dim3(grid_for(1LL << (3 * q - 1))), dim3(kBlock), 0, s, p, d, s_alpha, 1 << (3 * q));
  return hipGetLastError();
}

hipError_t launch_fcg_padd2(double* p, const double* d0, const double* s_alpha0, const double* d, const double* s_alpha,
                            int q, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_padd2, dim3(grid_for(1LL << (3 * q - 1))), dim3(kBlock), 0, s, p, d0, s_alpha0, d, s_alpha,
                     1 << (3 * q));
  return hipGetLastError();
}

hipError_t launch_fcg_zw(const double* z64, const float* z32, const double* w, int q, double* part, int* nblocks,
                         hipStream_t s) {
  const int nb = reduction_blocks(1LL << (3 * q - 1));
  hipLaunchKernelGGL(k_fcg_zw, dim3(nb), dim3(kBlock), 0, s, z64, z32, w, 1 << (3 * q), part);
  *nblocks = nb;
  return hipGetLastError();
}

hipError_t launch_fcg_dir(const double* z64, const float* z32, const double* d, double* dn, double* p,
                          const double* s_zw, const double* s_dw, const double* s_alpha, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_dir, dim3(grid_for(1LL << (3 * q - 1))), dim3(kBlock), 0, s, z64, z32, d, dn, p, s_zw, s_dw,
                     s_alpha, 1 << (3 * q));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_cycle(const CoarseCycle<T>& a, hipStream_t s) {
  if (a.nlev < 1 || a.nlev > 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_coarse_cycle<T>, dim3(1), dim3(kCoarseThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_divergence(const double* ux, const double* uy, const double* uz, const double* rx, const double* ry,
                             const double* rz, double dt, const uint8_t* mask, int q, double h, double* f,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_divergence, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, ux, uy, uz, rx, ry, rz, dt, mask,
                     q, 1.0 / (h * dt), f);
  return hipGetLastError();
}

hipError_t launch_project(double* ux, double* uy, double* uz, const double* rx, const double* ry, const double* rz,
                          double dt, const double* p, const double* bx, const double* by, const double* bz,
                          const uint8_t* mask, int q, double h, hipStream_t s) {
  hipLaunchKernelGGL(k_project, dim3(grid_for(1LL << (3 * q))), dim3(kBlock), 0, s, ux, uy, uz, rx, ry, rz, dt, p, bx,
                     by, bz, mask, q, dt / h);
  return hipGetLastError();
}

#define MG_INSTANTIATE(T)                                                                                        \
  template hipError_t launch_rbgs_half<T>(T*, const T*, const T*, const T*, const T*, int, double, int,          \
                                          const double*, hipStream_t);                                           \
  template hipError_t launch_residual_restrict<T>(const T*, const T*, const T*, const T*, const T*, const T*, int, \
                                                  double, const double*, T*, T*, hipStream_t);                   \
  template hipError_t launch_prolong_add<T>(const T*, T*, const uint8_t*, int, hipStream_t);                     \
  template hipError_t launch_coarse_solve<T>(const T*, T*, const double*, const uint8_t*, hipStream_t);    \
  template hipError_t launch_coarse_cycle<T>(const CoarseCycle<T>&, hipStream_t);
MG_INSTANTIATE(double)
MG_INSTANTIATE(float)
#undef MG_INSTANTIATE

}  // namespace mg
