// Control logic of Algorithm 1 (Section 6) shared by the host driver (one large
// matrix) and the batched kernel (one workgroup per small matrix): the finish test
// of the scaling loop, the Denman-Beavers stopping rule and the degree selection.
// Norms and estimates are supplied by the caller; an estimator callable
// est(q, r, &e) returns e = est ||B2^q B^r||_1 and false on failure.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace logm {

// Largest scheme with coefficients (k = 1 .. kKMax).
constexpr int kKMax = 9;
// Theta of eq. theta_Eb recomputed for our own fits of eq. five_mult_degopt (the
// paper prints no coefficients for k = 6..9), summed over every order of the
// polynomial with its coefficients rounded to double, rounded down.
constexpr double kTheta6Fit = 0.4258;
constexpr double kTheta7Fit = 0.5284;
constexpr double kTheta8Fit = 0.5739;
constexpr double kTheta9Fit = 0.6371;

// Table 2 (k -> m_k, Theta_{m_k}) as Algorithm 1 uses it: the printed Theta where
// the shipped polynomial's own Theta is at least that (k <= 6), the fits' own below
// it (k = 7, 8, 9: the printed values belong to the paper's polynomials).  theta_source
// 1 replaces Theta_5 by 0.2448, the value Table 1 yields when recomputed, and
// Theta_6 by the value recomputed for our six-product fit.
struct ThetaTable {
  int m[10];
  double th[10];
};

__host__ __device__ inline ThetaTable theta_table(int source) {
  const int m[10] = {0, 2, 4, 8, 14, 14, 20, 24, 27, 28};
  const double th[10] = {0.0, 1.83e-8, 1.53e-4, 1.33e-2, 9.31e-2, 2.46e-1,
                         3.72e-1, 5.86e-1, 6.69e-1, 7.28e-1};
  ThetaTable t;
  for (int k = 0; k < 10; ++k) {
    t.m[k] = m[k];
    t.th[k] = th[k];
  }
  t.th[7] = kTheta7Fit;
  t.th[8] = kTheta8Fit;
  t.th[9] = kTheta9Fit;
  if (source == 1) {
    t.th[5] = 0.2448;
    t.th[6] = kTheta6Fit;
  }
  return t;
}

// Coefficients of the schemes k = 1..kKMax of eq. five_mult_degopt packed in one
// array, as the batched kernel takes them: scheme k holds h (rows j = 2..k, row j
// with the j weights of P_2..P_{j+1}), then g in the same layout, then y_1..y_{k+2}.
__host__ __device__ constexpr int scheme_coef_count(int k) { return k * k + 2 * k; }
__host__ __device__ constexpr int scheme_coef_base(int k) {
  int b = 0;
  for (int q = 1; q < k; ++q) b += scheme_coef_count(q);
  return b;
}
constexpr int kSchemeCoefTotal = scheme_coef_base(kKMax + 1);

struct PackedScheme {
  const double* c;   // scheme_coef_count(k) values from scheme_coef_base(k)
  int k;
  __host__ __device__ int rows() const { return k * (k + 1) / 2 - 1; }   // values in h
  __host__ __device__ static int row(int j) { return j * (j - 1) / 2 - 1; }
  __host__ __device__ double h(int j, int i) const { return c[row(j) + i - 2]; }
  __host__ __device__ double g(int j, int i) const { return c[rows() + row(j) + i - 2]; }
  __host__ __device__ double y(int q) const { return c[2 * rows() + q - 1]; }
};

// Schemes available up to k_max, increasing (shipped: 1 to kKMax).
struct SchemeSet {
  int k[kKMax];
  int n;
};

__host__ __device__ inline SchemeSet scheme_set(int k_max) {
  SchemeSet s;
  s.n = 0;
  for (int k = 1; k <= kKMax; ++k)
    if (k <= k_max) s.k[s.n++] = k;
  return s;
}

// tabmin_im of the degree-selection procedure (index r - 1 for the first j with
// ||B^2||^{1/2} <= Theta_j).
__host__ __device__ inline int tabmin(int r) {
  const int t[9] = {1, 2, 3, 4, 4, 5, 5, 6, 6};
  return t[r < 1 ? 0 : (r > 9 ? 8 : r - 1)];
}

// Denman-Beavers stopping rule (the paper gives none): stop at rel <= tol
// (sqrt(n) u) or, once scaling is off, on stagnation below 1e-6; scaling is
// switched off once rel < 1e-2.
__host__ __device__ inline bool db_stop(double rel, double rel_prev, bool& scaled, double tol) {
  if (rel < 1e-2) scaled = false;
  return rel <= tol || (!scaled && rel < 1e-6 && rel > rel_prev / 2.0);
}

// Finish test of the scaling loop for the largest scheme (m = mtop, Theta = thtop):
// term 1 by ||B^2||^{1/2} (eq. alpha2term1) or the estimate of ||B^2^{mtop/2}||;
// term 2 by (base ||B||)^{1/(mtop+1)} (eq. normAm9plus1) or the estimate of
// ||B^2^{mtop/2} B||.  Records which estimates were made for the degree selection.
template <class Est>
__host__ __device__ bool finish_test(Est& est, double n1, double n2, int mtop, double thtop,
                                     bool& have_top, double& e_top, bool& have_top1,
                                     double& e_top1, int* n_est, bool* ok) {
  const int htop = mtop / 2;
  have_top = have_top1 = false;
  bool t1, t2 = false;
  double base;
  if (sqrt(n2) <= thtop) {
    t1 = true;
    base = pow(n2, (double)htop);
  } else {
    if (!est(htop, 0, &e_top)) {
      *ok = false;
      return false;
    }
    ++*n_est;
    have_top = true;
    t1 = pow(e_top, 1.0 / mtop) <= thtop;
    base = e_top;
  }
  if (t1) {
    if (pow(base * n1, 1.0 / (mtop + 1)) <= thtop) {
      t2 = true;
    } else {
      if (!est(htop, 1, &e_top1)) {
        *ok = false;
        return false;
      }
      ++*n_est;
      have_top1 = true;
      t2 = pow(e_top1, 1.0 / (mtop + 1)) <= thtop;
    }
  }
  return t1 && t2;
}

// Degree selection after Algorithm 1: min_in from the last pass's estimates (eqs.
// min_in, min_inp) or from ||B^2||^{1/2} with tabmin (eq. roughmin_in); max_in from
// (||B^2||^{m/2} ||B||)^{1/(m+1)} (eqs. alpharoughbound_even, roughmax_even); then
// candidates from min_in upward with estimates skipped whenever a bound decides,
// and the "j+1" shortcut.
template <class Est>
__host__ __device__ int select_degree(Est& est, const ThetaTable& T, const SchemeSet& K, double n1,
                                      double n2, bool have_top, double e_top, bool have_top1,
                                      double e_top1, int* n_est, bool* ok) {
  const int ktop = K.k[K.n - 1];
  const int mtop = T.m[ktop];
  const double sq2 = sqrt(n2);
  auto first_pass = [&](double v) {
    for (int i = 0; i < K.n; ++i)
      if (v <= T.th[K.k[i]]) return K.k[i];
    return ktop;
  };
  int min_in;
  if (have_top) {
    min_in = first_pass(pow(e_top, 1.0 / mtop));
    if (have_top1) {
      const int m2 = first_pass(pow(e_top1, 1.0 / (mtop + 1)));
      min_in = min_in > m2 ? min_in : m2;
    }
  } else {
    const int t = tabmin(first_pass(sq2));
    min_in = K.k[0];
    for (int i = 0; i < K.n; ++i)
      if (K.k[i] <= t) min_in = K.k[i];
    if (sq2 > T.th[1]) {
      bool has2 = false;
      for (int i = 0; i < K.n; ++i) has2 |= (K.k[i] == 2);
      if (has2 && min_in < 2) min_in = 2;
    } else {
      min_in = K.k[0];
    }
  }
  int max_in = ktop;
  for (int i = 0; i < K.n; ++i) {
    const int j = K.k[i];
    const int m = T.m[j];
    if (pow(pow(n2, m / 2.0) * n1, 1.0 / (m + 1)) <= T.th[j]) {
      max_in = j;
      break;
    }
  }
  if (min_in >= max_in) return max_in;
  int idx = 0;
  while (K.k[idx] != min_in) ++idx;
  while (K.k[idx] < max_in) {
    const int j = K.k[idx];
    const int nxt = K.k[idx + 1];
    const double thj = T.th[j], thn = T.th[nxt];
    const int m = T.m[j];
    const int h = m / 2;
    double e1, t1;
    if (h == 1) {
      e1 = n2;
      t1 = sq2;
    } else if (sq2 <= thj) {
      e1 = pow(n2, (double)h);
      t1 = sq2;
    } else {
      if (!est(h, 0, &e1)) {
        *ok = false;
        return max_in;
      }
      ++*n_est;
      t1 = pow(e1, 1.0 / m);
    }
    double alpha;
    if (t1 > thn) {
      alpha = t1;
    } else {
      const double tau = (t1 <= thj) ? thj : thn;
      const double bound = pow(e1 * n1, 1.0 / (m + 1));
      double t2;
      if (bound <= tau) {
        t2 = bound;
      } else {
        double e2;
        if (!est(h, 1, &e2)) {
          *ok = false;
          return max_in;
        }
        ++*n_est;
        t2 = pow(e2, 1.0 / (m + 1));
      }
      alpha = t1 > t2 ? t1 : t2;
    }
    if (alpha <= thj) return j;
    if (alpha <= thn) return nxt;
    ++idx;
  }
  return max_in;
}

}  // namespace logm
