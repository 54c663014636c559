// Pseudo-inverse of a small symmetric matrix (pure host C++, FP64).
//
// The directly solved 4^3 grid of the hierarchy has a 64 x 64 symmetric operator
// whose null space holds the constant on each connected fluid region and one unit
// vector per body cell.  Its pseudo-inverse is formed once per setup from the
// eigendecomposition, computed here by cyclic Jacobi rotations: each rotation in the
// (p, q) plane is chosen to zero the (p, q) entry, and sweeps over all pairs repeat
// until the off-diagonal mass is negligible.  Eigenvalues below rtol * max|lambda|
// are treated as zero.
#include <cmath>
#include <vector>

namespace mg {

void jacobi_eigen(int n, std::vector<double>& a, std::vector<double>& v, std::vector<double>& lam) {
  v.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  auto A = [&](int r, int c) -> double& { return a[static_cast<size_t>(r) * n + c]; };
  auto V = [&](int r, int c) -> double& { return v[static_cast<size_t>(r) * n + c]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) (r == c ? diag : off) += A(r, c) * A(r, c);
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        if (apq == 0.0) continue;
        // angle phi with cot(2 phi) = (a_qq - a_pp) / (2 a_pq); t = tan(phi), smaller root
        const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0);
        const double s = t * c;
        for (int k = 0; k < n; ++k) {   // columns: A J
          const double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows: J^T (A J)
          const double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        A(p, q) = A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {   // eigenvectors: V J
          const double vkp = V(k, p), vkq = V(k, q);
          V(k, p) = c * vkp - s * vkq;
          V(k, q) = s * vkp + c * vkq;
        }
      }
    }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A(i, i);
}

// pinv (row-major n x n) of the symmetric matrix a (row-major, destroyed).
void symmetric_pinv(int n, std::vector<double>& a, double rtol, std::vector<double>& pinv) {
  std::vector<double> v, lam;
  jacobi_eigen(n, a, v, lam);
  double big = 0.0;
  for (double l : lam) big = std::fmax(big, std::fabs(l));
  std::vector<double> inv(n, 0.0);
  for (int i = 0; i < n; ++i)
    if (std::fabs(lam[i]) > rtol * big) inv[i] = 1.0 / lam[i];
  pinv.assign(static_cast<size_t>(n) * n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += v[r * n + k] * inv[k] * v[c * n + k];
      pinv[static_cast<size_t>(r) * n + c] = s;
    }
}

}  // namespace mg

namespace mg {

// Pseudo-inverse of a symmetric negative semi-definite graph operator whose null
// space is known: one normalised indicator vector per connected component of the
// active cells, and one unit vector per inactive cell (their rows and columns are
// zero).  With Z that orthonormal basis, B = A - Z Z^T is negative definite and
// A^+ = B^-1 + Z Z^T.  B^-1 comes from a Cholesky factorisation of -B, an O(n^3)
// direct method (about 100x cheaper than Jacobi sweeps at n = 64).  Returns false if
// the factorisation meets a non-positive pivot; the caller then falls back to the
// eigendecomposition.
bool graph_pinv(int n, const std::vector<double>& a, const std::vector<int>& component, double rtol,
                std::vector<double>& pinv) {
  // component[c] = id >= 0 for active cells, -1 for inactive ones
  int ncomp = 0;
  for (int c = 0; c < n; ++c) ncomp = component[c] + 1 > ncomp ? component[c] + 1 : ncomp;
  std::vector<double> zz(static_cast<size_t>(n) * n, 0.0);
  std::vector<int> size(ncomp, 0);
  for (int c = 0; c < n; ++c)
    if (component[c] >= 0) ++size[component[c]];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      double v = 0.0;
      if (component[r] < 0 || component[c] < 0)
        v = (r == c && component[r] < 0) ? 1.0 : 0.0;
      else if (component[r] == component[c])
        v = 1.0 / size[component[r]];
      zz[static_cast<size_t>(r) * n + c] = v;
    }
  // M = -(A - Z Z^T) = Z Z^T - A, symmetric positive definite
  std::vector<double> L(static_cast<size_t>(n) * n, 0.0);
  double big = 0.0;
  for (size_t i = 0; i < a.size(); ++i) big = std::fmax(big, std::fabs(a[i]));
  for (int j = 0; j < n; ++j) {
    double d = zz[static_cast<size_t>(j) * n + j] - a[static_cast<size_t>(j) * n + j];
    for (int k = 0; k < j; ++k) d -= L[static_cast<size_t>(j) * n + k] * L[static_cast<size_t>(j) * n + k];
    if (!(d > rtol * std::fmax(big, 1.0))) return false;
    const double ljj = std::sqrt(d);
    L[static_cast<size_t>(j) * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = zz[static_cast<size_t>(i) * n + j] - a[static_cast<size_t>(i) * n + j];
      for (int k = 0; k < j; ++k) s -= L[static_cast<size_t>(i) * n + k] * L[static_cast<size_t>(j) * n + k];
      L[static_cast<size_t>(i) * n + j] = s / ljj;
    }
  }
  // M^-1 column by column (forward then backward substitution), A^+ = -M^-1 + Z Z^T
  pinv.assign(static_cast<size_t>(n) * n, 0.0);
  std::vector<double> y(n), x(n);
  for (int col = 0; col < n; ++col) {
    for (int i = 0; i < n; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[static_cast<size_t>(i) * n + k] * y[k];
      y[i] = s / L[static_cast<size_t>(i) * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= L[static_cast<size_t>(k) * n + i] * x[k];
      x[i] = s / L[static_cast<size_t>(i) * n + i];
    }
    for (int r = 0; r < n; ++r) pinv[static_cast<size_t>(r) * n + col] = -x[r] + zz[static_cast<size_t>(r) * n + col];
  }
  return true;
}

}  // namespace mg
