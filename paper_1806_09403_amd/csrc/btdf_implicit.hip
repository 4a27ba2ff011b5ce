// btdf_implicit.hip -- host set-up of the comparison forcing methods of
// Section 3: the implicit direct forcing (eq 17; the implicit velocity
// correction of eqs 32-35 is the same method, Appendix A) and RKPM (eq 36 /
// B54). Both need, per body, the matrix A of eq 22 (drs = dh):
//   A_lm = ds sum_k W_lk W_mk     (dh = 1),
// the node sum of the delta weights of markers l and m. For the implicit
// method the library keeps (D_I D_E)^-1 = (drs A)^-1 per body and applies
// it to the direct force each step; for RKPM it keeps epsilon = A^-1 1
// (row sums of A^-1) and spreads ds epsilon_l F_l. Markers of different
// bodies are not coupled (one matrix per body). Dense Cholesky in FP64.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "btdf_internal.h"

namespace btdf {
namespace host {

double phi_host(int kind, double r);

namespace {

// A of eq 22 for the markers l0 .. l0+n-1 of one body (row-major n x n).
// Nodes are integer; the offset between two stencil bases is reduced to
// the nearest periodic image, so markers given on either side of a
// periodic seam pair up correctly.
void body_matrix(const btdf_t *h, int l0, int n, double ds, std::vector<double> &A) {
  const int S = stencil_size(h->kind);
  std::vector<int> bx(n), by(n);
  std::vector<double> wx(4 * (size_t)n, 0.0), wy(4 * (size_t)n, 0.0);
  for (int l = 0; l < n; ++l) {
    const double X = h->X[l0 + l], Y = h->Y[l0 + l];
    bx[l] = stencil_base(h->kind, X);
    by[l] = stencil_base(h->kind, Y);
    for (int a = 0; a < S; ++a) {
      wx[4 * (size_t)l + a] = phi_host(h->kind, (double)(bx[l] + a) - X);
      wy[4 * (size_t)l + a] = phi_host(h->kind, (double)(by[l] + a) - Y);
    }
  }
  A.assign((size_t)n * n, 0.0);
  for (int l = 0; l < n; ++l) {
    for (int m = 0; m < n; ++m) {
      int ox = bx[m] - bx[l], oy = by[m] - by[l];
      if (h->xper()) ox -= h->nx * (int)std::floor((double)ox / h->nx + 0.5);
      if (h->yper()) oy -= h->ny * (int)std::floor((double)oy / h->ny + 0.5);
      if (ox <= -S || ox >= S || oy <= -S || oy >= S) continue;
      double s = 0.0;
      for (int c = 0; c < S; ++c) {
        const int cm = c - oy;
        if (cm < 0 || cm >= S) continue;
        for (int a = 0; a < S; ++a) {
          const int am = a - ox;
          if (am < 0 || am >= S) continue;
          s += wx[4 * (size_t)l + a] * wy[4 * (size_t)l + c] * wx[4 * (size_t)m + am] * wy[4 * (size_t)m + cm];
        }
      }
      A[(size_t)l * n + m] = ds * s;
    }
  }
}

// In-place Cholesky A = L L^T (lower triangle); false if A is not
// numerically positive definite.
bool cholesky(std::vector<double> &A, int n) {
  double dmax = 0.0;
  for (int k = 0; k < n; ++k) dmax = std::max(dmax, A[(size_t)k * n + k]);
  for (int k = 0; k < n; ++k) {
    double d = A[(size_t)k * n + k];
    for (int t = 0; t < k; ++t) d -= A[(size_t)k * n + t] * A[(size_t)k * n + t];
    if (!(d > 1e-12 * dmax)) return false;
    const double lk = std::sqrt(d);
    A[(size_t)k * n + k] = lk;
    for (int r = k + 1; r < n; ++r) {
      double v = A[(size_t)r * n + k];
      for (int t = 0; t < k; ++t) v -= A[(size_t)r * n + t] * A[(size_t)k * n + t];
      A[(size_t)r * n + k] = v / lk;
    }
  }
  return true;
}

// Solve L L^T x = b in place (L from cholesky).
void chol_solve(const std::vector<double> &L, int n, double *x) {
  for (int r = 0; r < n; ++r) {
    double v = x[r];
    for (int t = 0; t < r; ++t) v -= L[(size_t)r * n + t] * x[t];
    x[r] = v / L[(size_t)r * n + r];
  }
  for (int r = n - 1; r >= 0; --r) {
    double v = x[r];
    for (int t = r + 1; t < n; ++t) v -= L[(size_t)t * n + r] * x[t];
    x[r] = v / L[(size_t)r * n + r];
  }
}

}  // namespace

std::string forcing_setup(btdf_t *h) {
  h->minv.clear();
  h->minv_off.assign(1, 0);
  h->s_rkpm.clear();
  h->max_body = 0;
  if (h->method == BTDF_FORCING_DIRECT) return "";
  const int nb = h->nb();
  for (int b = 0; b < nb; ++b) h->max_body = std::max(h->max_body, h->off[b + 1] - h->off[b]);
  if (h->max_body > kMaxImplicitBody) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "implicit and RKPM forcing take bodies of at most %d markers (got %d)",
                  kMaxImplicitBody, h->max_body);
    return msg;
  }
  if (h->method == BTDF_FORCING_RKPM) h->s_rkpm.assign(h->X.size(), 0.0);
  std::vector<double> A;
  for (int b = 0; b < nb; ++b) {
    const int l0 = h->off[b], n = h->off[b + 1] - l0;
    const double ds = h->bds[b];
    body_matrix(h, l0, n, ds, A);
    if (!cholesky(A, n)) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "matrix A of body %d is singular to working precision (markers too dense)", b);
      return msg;
    }
    if (h->method == BTDF_FORCING_RKPM) {
      // epsilon = A^-1 1 (eq B54); the spreading factor of marker l is ds epsilon_l
      std::vector<double> e(n, 1.0);
      chol_solve(A, n, e.data());
      for (int l = 0; l < n; ++l) h->s_rkpm[l0 + l] = ds * e[l];
    } else {
      // (D_I D_E)^-1 = (drs A)^-1, kept column-major: entry (i, j) at j n + i
      const size_t base = h->minv.size();
      h->minv.resize(base + (size_t)n * n);
      std::vector<double> col(n);
      for (int j = 0; j < n; ++j) {
        std::fill(col.begin(), col.end(), 0.0);
        col[j] = 1.0 / h->drs;
        chol_solve(A, n, col.data());
        std::memcpy(&h->minv[base + (size_t)j * n], col.data(), (size_t)n * sizeof(double));
      }
    }
    h->minv_off.push_back((long long)h->minv.size());
  }
  return "";
}

}  // namespace host
}  // namespace btdf
