// Cut cells: open-area and fluid-volume fractions from the body's level set, merging of
// small cells, and the merged face coefficients (paper section 2.2, the method of
// fractional areas in eq. (integral2)).
//
// Setup-time kernels, one thread per cell.  Inside/outside is decided per sample of the
// bilinear (faces) or trilinear (cells) interpolant of psi at the corners.  Sample
// values are summed corner by corner in a fixed order with __dmul_rn / __dadd_rn (no
// fused multiply-adds; the weights are exact dyadic numbers), so every decision is
// reproducible bit for bit on any IEEE implementation.  A face or cell whose corners
// all have the same sign needs no samples: interpolation weights are positive, so every
// sample has that sign too.
#include "mg_kernels.h"

namespace mg {

namespace {

constexpr int kCutBlock = 256;

__device__ __forceinline__ double corner_psi(const double* __restrict__ psi, int i, int j, int k, int q) {
  const int m = (1 << q) - 1;
  return psi[(static_cast<long long>(k) << (2 * q)) + (((j & m) << q) | (i & m))];
}

// samples of the bilinear interpolant > 0; c_uv is the corner at (u, v) in {0, 1}^2
__device__ int face_count(double c00, double c10, double c01, double c11, int S) {
  if (c00 > 0.0 && c10 > 0.0 && c01 > 0.0 && c11 > 0.0) return S * S;
  if (!(c00 > 0.0) && !(c10 > 0.0) && !(c01 > 0.0) && !(c11 > 0.0)) return 0;
  const double inv = 1.0 / S;
  int count = 0;
  for (int iv = 0; iv < S; ++iv) {
    const double v = (iv + 0.5) * inv;
    for (int iu = 0; iu < S; ++iu) {
      const double u = (iu + 0.5) * inv;
      const double w00 = (1.0 - u) * (1.0 - v), w10 = u * (1.0 - v), w01 = (1.0 - u) * v, w11 = u * v;
      const double val =
          __dadd_rn(__dadd_rn(__dadd_rn(__dmul_rn(w00, c00), __dmul_rn(w10, c10)), __dmul_rn(w01, c01)),
                    __dmul_rn(w11, c11));
      count += val > 0.0;
    }
  }
  return count;
}

// samples of the trilinear interpolant > 0; c[a + 2b + 4c] is the corner (a, b, c)
__device__ int cell_count(const double* c, int S) {
  bool all_in = true, all_out = true;
  for (int q = 0; q < 8; ++q) {
    all_in = all_in && c[q] > 0.0;
    all_out = all_out && !(c[q] > 0.0);
  }
  if (all_in) return S * S * S;
  if (all_out) return 0;
  const double inv = 1.0 / S;
  int count = 0;
  for (int iw = 0; iw < S; ++iw) {
    const double w = (iw + 0.5) * inv;
    for (int iv = 0; iv < S; ++iv) {
      const double v = (iv + 0.5) * inv;
      for (int iu = 0; iu < S; ++iu) {
        const double u = (iu + 0.5) * inv;
        double val = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double wt = ((q & 1) ? u : 1.0 - u) * ((q & 2) ? v : 1.0 - v) * ((q & 4) ? w : 1.0 - w);
          val = q == 0 ? __dmul_rn(wt, c[0]) : __dadd_rn(val, __dmul_rn(wt, c[q]));
        }
        count += val > 0.0;
      }
    }
  }
  return count;
}

__global__ __launch_bounds__(kCutBlock) void k_cut_fractions(const double* __restrict__ psi, int q, int S,
                                                             double* __restrict__ ax, double* __restrict__ ay,
                                                             double* __restrict__ az, double* __restrict__ vol) {
  const int m = (1 << q) - 1;
  const long long t = static_cast<long long>(blockIdx.x) * kCutBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
  double p[8];
#pragma unroll
  for (int n = 0; n < 8; ++n) p[n] = corner_psi(psi, i + (n & 1), j + ((n >> 1) & 1), k + (n >> 2), q);
  const double s2 = static_cast<double>(S * S);
  // faces x = i h: (u, v) = (y, z); y = j h: (x, z); z = k h: (x, y)
  ax[c] = face_count(p[0], p[2], p[4], p[6], S) / s2;
  ay[c] = face_count(p[0], p[1], p[4], p[5], S) / s2;
  az[c] = k == 0 ? 0.0 : face_count(p[0], p[1], p[2], p[3], S) / s2;   // bottom wall closed
  vol[c] = cell_count(p, S) / (s2 * S);
}

__global__ __launch_bounds__(kCutBlock) void k_cut_merge(const double* __restrict__ psi,
                                                         const double* __restrict__ vol, int q,
                                                         int32_t* __restrict__ merge_to) {
  const int n = 1 << q, m = n - 1;
  const long long t = static_cast<long long>(blockIdx.x) * kCutBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const int i = c & m, j = (c >> q) & m, k = c >> (2 * q);
  int target = -1;
  const double V = vol[c];
  if (V > 0.0 && V < kMergeFraction) {
    double p[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) p[s] = corner_psi(psi, i + (s & 1), j + ((s >> 1) & 1), k + (s >> 2), q);
    // gradient of the trilinear psi at the centre: mean of the 4 edge differences per axis
    const double gx = __dadd_rn(__dadd_rn(__dadd_rn(__dsub_rn(p[1], p[0]), __dsub_rn(p[3], p[2])),
                                          __dsub_rn(p[5], p[4])), __dsub_rn(p[7], p[6])) * 0.25;
    const double gy = __dadd_rn(__dadd_rn(__dadd_rn(__dsub_rn(p[2], p[0]), __dsub_rn(p[3], p[1])),
                                          __dsub_rn(p[6], p[4])), __dsub_rn(p[7], p[5])) * 0.25;
    const double gz = __dadd_rn(__dadd_rn(__dadd_rn(__dsub_rn(p[4], p[0]), __dsub_rn(p[5], p[1])),
                                          __dsub_rn(p[6], p[2])), __dsub_rn(p[7], p[3])) * 0.25;
    const double fx = fabs(gx), fy = fabs(gy), fz = fabs(gz);
    const int d = (fx >= fy && fx >= fz) ? 0 : (fy >= fz ? 1 : 2);
    const double g = d == 0 ? gx : (d == 1 ? gy : gz);
    const int s = g > 0.0 ? 1 : -1;
    int ti = i, tj = j, tk = k;
    if (d == 0) ti = (i + s) & m;
    else if (d == 1) tj = (j + s) & m;
    else tk = k + s;
    if (tk >= 0 && tk < n) {
      const int tc = (((tk << q) | tj) << q) | ti;
      if (!(vol[tc] < kMergeFraction)) target = tc;
    }
  }
  merge_to[c] = target;
}

// neighbour of c one step along axis m (x, y periodic); -1 beyond a z wall
__device__ __forceinline__ int step_cell(int c, int m_axis, int s, int q) {
  const int n = 1 << q, msk = n - 1;
  const int i = c & msk, j = (c >> q) & msk, k = c >> (2 * q);
  if (m_axis == 0) return (((k << q) | j) << q) | ((i + s) & msk);
  if (m_axis == 1) return (((k << q) | ((j + s) & msk)) << q) | i;
  const int kk = k + s;
  return (kk < 0 || kk >= n) ? -1 : (((kk << q) | j) << q) | i;
}

__device__ __forceinline__ bool kept_cell(const double* __restrict__ vol, const int32_t* __restrict__ merge_to, int c) {
  return vol[c] > 0.0 && merge_to[c] < 0;
}

__global__ __launch_bounds__(kCutBlock) void k_cut_coeffs(const double* __restrict__ rho,
                                                          const double* __restrict__ ax,
                                                          const double* __restrict__ ay,
                                                          const double* __restrict__ az,
                                                          const double* __restrict__ vol,
                                                          const int32_t* __restrict__ merge_to, int q,
                                                          double* __restrict__ bx, double* __restrict__ by,
                                                          double* __restrict__ bz, uint8_t* __restrict__ mask) {
  const long long t = static_cast<long long>(blockIdx.x) * kCutBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const bool kc = kept_cell(vol, merge_to, c);
  mask[c] = kc ? 1 : 0;
  const double* area[3] = {ax, ay, az};
  double* out[3] = {bx, by, bz};
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int lo = step_cell(c, l, -1, q);
    double beta = 0.0;
    if (kc && lo >= 0 && kept_cell(vol, merge_to, lo)) {
      // own area, then faces between donors merging side by side into c and lo
      double a = area[l][c];
      for (int mm = 0; mm < 3; ++mm) {
        if (mm == l) continue;
        for (int s = -1; s <= 1; s += 2) {
          const int d = step_cell(c, mm, s, q), dl = step_cell(lo, mm, s, q);
          if (d >= 0 && dl >= 0 && merge_to[d] == c && merge_to[dl] == lo) a = a + area[l][d];
        }
      }
      beta = a * face_beta(rho[c], rho[lo]);
    }
    out[l][c] = beta;
  }
}

__global__ __launch_bounds__(kCutBlock) void k_merge_rhs(const int32_t* __restrict__ merge_to,
                                                         const double* __restrict__ f, int q,
                                                         double* __restrict__ g) {
  const long long t = static_cast<long long>(blockIdx.x) * kCutBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  if (merge_to[c] >= 0) {
    g[c] = 0.0;
    return;
  }
  double acc = f[c];
  for (int mm = 0; mm < 3; ++mm)
    for (int s = -1; s <= 1; s += 2) {
      const int d = step_cell(c, mm, s, q);
      if (d >= 0 && merge_to[d] == c) acc = acc + f[d];
    }
  g[c] = acc;
}

__global__ __launch_bounds__(kCutBlock) void k_merge_fill(const int32_t* __restrict__ merge_to, int q,
                                                          double* __restrict__ p) {
  const long long t = static_cast<long long>(blockIdx.x) * kCutBlock + threadIdx.x;
  if (t >= (1LL << (3 * q))) return;
  const int c = static_cast<int>(t);
  const int target = merge_to[c];
  if (target >= 0) p[c] = p[target];   // a target is never a donor
}

inline unsigned cut_grid(int q) { return static_cast<unsigned>(((1LL << (3 * q)) + kCutBlock - 1) / kCutBlock); }

}  // namespace

hipError_t launch_cut_cells(const double* psi, int q, int samples, double* ax, double* ay, double* az, double* vol,
                            int32_t* merge_to, hipStream_t s) {
  hipLaunchKernelGGL(k_cut_fractions, dim3(cut_grid(q)), dim3(kCutBlock), 0, s, psi, q, samples, ax, ay, az, vol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cut_merge, dim3(cut_grid(q)), dim3(kCutBlock), 0, s, psi, vol, q, merge_to);
  return hipGetLastError();
}

hipError_t launch_cut_coeffs(const double* rho, const double* ax, const double* ay, const double* az,
                             const double* vol, const int32_t* merge_to, int q, double* bx, double* by, double* bz,
                             uint8_t* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_cut_coeffs, dim3(cut_grid(q)), dim3(kCutBlock), 0, s, rho, ax, ay, az, vol, merge_to, q, bx,
                     by, bz, mask);
  return hipGetLastError();
}

hipError_t launch_merge_rhs(const int32_t* merge_to, const double* f, double* g, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_rhs, dim3(cut_grid(q)), dim3(kCutBlock), 0, s, merge_to, f, q, g);
  return hipGetLastError();
}

hipError_t launch_merge_fill(const int32_t* merge_to, double* p, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_fill, dim3(cut_grid(q)), dim3(kCutBlock), 0, s, merge_to, q, p);
  return hipGetLastError();
}

}  // namespace mg
