/* FP64 direct-sum correlation over many patterns (plain C, OpenMP over patterns, then zones).
 *
 * TEST INFRASTRUCTURE ONLY: part of the oracle; never linked into the product.
 *
 * Paper: Methods > Correlation Pattern Matching.  For every pattern this builds
 * the sparse polar image (Eq. image_polar) cell by cell, then evaluates the
 * correlogram and its mirror as the plain circular cross-correlation that the
 * paper's FFT route equals:
 *     C[z,n]  = sum_{cells (b,s) with X != 0} X[b,s] P[z, (b - n) mod N, s]
 *     Cm[z,n] = sum_{cells (b,s) with X != 0} X[b,s] P[z, (-b - n) mod N, s]
 * and reports, per zone, the best value over (n, branch) with the tie rule
 * smallest n then non-mirror first, plus the two cyclic neighbours of that bin
 * in its branch (for the parabolic refinement done in Python).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double wrap_pi(double x) {
  const double tp = 2.0 * M_PI;
  double y = x + M_PI;
  y = y - tp * floor(y / tp);
  return y - M_PI;
}

static double kern(double d, double delta, int kind, double sigma) {
  if (kind == 0) return d < delta ? 1.0 - d / delta : 0.0;
  return d < 3.0 * sigma ? exp(-d * d / (2.0 * sigma * sigma)) : 0.0;
}

/* Polar image of one pattern into X[N][R] (zeroed here). */
static void polar_image(int N, int R, const double* q_s, int m0, int m1, const float* qx,
                        const float* qy, const float* I, double delta, double gamma, double omega,
                        int kind, double sigma, double* X) {
  const double rad = kind == 0 ? delta : 3.0 * sigma;
  memset(X, 0, sizeof(double) * (size_t)N * R);
  for (int m = m0; m < m1; ++m) {
    double x = qx[m], y = qy[m], in = I[m];
    double q = sqrt(x * x + y * y), g = atan2(y, x);
    double w = pow(q, gamma) * pow(in, 0.5 * omega);
    for (int s = 0; s < R; ++s) {
      double dq = q - q_s[s];
      if (fabs(dq) >= rad) continue;
      for (int a = 0; a < N; ++a) {
        double dp = wrap_pi(2.0 * M_PI * a / N - g) * q_s[s];
        double k = kern(sqrt(dq * dq + dp * dp), delta, kind, sigma);
        if (k > 0.0) X[(size_t)a * R + s] += w * k;
      }
    }
  }
}

int acom_oracle_directsum(int Z, int N, int R, const double* P, const double* q_s, int n_pat,
                          const long long* offsets, const float* qx, const float* qy,
                          const float* I, double delta, double gamma, double omega, int kind,
                          double sigma, double* zscore, int* zn, int* zmir, double* zcm1,
                          double* zcp1, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int fail = 0;
  /* 1. every pattern's image and the list of its nonzero cells (b, s, X) */
  int* nnz = (int*)calloc((size_t)(n_pat > 0 ? n_pat : 1), sizeof(int));
  int** cb = (int**)calloc((size_t)(n_pat > 0 ? n_pat : 1), sizeof(int*));
  int** cs = (int**)calloc((size_t)(n_pat > 0 ? n_pat : 1), sizeof(int*));
  double** cx = (double**)calloc((size_t)(n_pat > 0 ? n_pat : 1), sizeof(double*));
  if (!nnz || !cb || !cs || !cx) fail = 1;
  if (!fail) {
#pragma omp parallel
    {
      double* X = (double*)malloc(sizeof(double) * (size_t)N * R);
      if (!X) {
#pragma omp atomic write
        fail = 1;
      } else {
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < n_pat; ++p) {
          polar_image(N, R, q_s, (int)offsets[p], (int)offsets[p + 1], qx, qy, I, delta, gamma,
                      omega, kind, sigma, X);
          int J = 0;
          for (size_t i = 0; i < (size_t)N * R; ++i) J += X[i] != 0.0;
          cb[p] = (int*)malloc(sizeof(int) * (size_t)(J > 0 ? J : 1));
          cs[p] = (int*)malloc(sizeof(int) * (size_t)(J > 0 ? J : 1));
          cx[p] = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
          if (!cb[p] || !cs[p] || !cx[p]) {
#pragma omp atomic write
            fail = 1;
            continue;
          }
          J = 0;
          for (int a = 0; a < N; ++a)
            for (int s = 0; s < R; ++s)
              if (X[(size_t)a * R + s] != 0.0) {
                cb[p][J] = a;
                cs[p][J] = s;
                cx[p][J] = X[(size_t)a * R + s];
                ++J;
              }
          nnz[p] = J;
        }
      }
      free(X);
    }
  }
  /* 2. every (zone, pattern): the two correlograms as direct sums over the
   * pattern's nonzero cells in raster order, then the best (n, branch).  The
   * zone's plan is read through a copy stored [s][a], so that the sum over
   * shifts n walks one contiguous row; the products and their order are those
   * of the definition above. */
  if (!fail) {
#pragma omp parallel
    {
      double* PT = (double*)malloc(sizeof(double) * (size_t)N * R);
      double* C0 = (double*)malloc(sizeof(double) * (size_t)N);
      double* C1 = (double*)malloc(sizeof(double) * (size_t)N);
      if (!PT || !C0 || !C1) {
#pragma omp atomic write
        fail = 1;
      } else {
#pragma omp for schedule(dynamic, 1)
        for (int z = 0; z < Z; ++z) {
          const double* Pz = P + (size_t)z * N * R;
          for (int a = 0; a < N; ++a)
            for (int s = 0; s < R; ++s) PT[(size_t)s * N + a] = Pz[(size_t)a * R + s];
          for (int p = 0; p < n_pat; ++p) {
            for (int n = 0; n < N; ++n) C0[n] = C1[n] = 0.0;
            for (int j = 0; j < nnz[p]; ++j) {
              const int b = cb[p][j];
              const double x = cx[p][j];
              const double* row = PT + (size_t)cs[p][j] * N;
              int i0 = b;                 /* (b - n) mod N at n = 0 */
              int i1 = (N - b) % N;       /* (-b - n) mod N at n = 0 */
              for (int n = 0; n < N; ++n) {
                C0[n] += x * row[i0];
                C1[n] += x * row[i1];
                i0 = i0 == 0 ? N - 1 : i0 - 1;
                i1 = i1 == 0 ? N - 1 : i1 - 1;
              }
            }
            /* best over (n, branch): the first maximum in the order n, then branch */
            int bn = 0, bm = 0;
            double bv = C0[0];
            for (int n = 0; n < N; ++n) {
              if (C0[n] > bv) { bv = C0[n]; bn = n; bm = 0; }
              if (C1[n] > bv) { bv = C1[n]; bn = n; bm = 1; }
            }
            const double* Cb = bm ? C1 : C0;
            const size_t o = (size_t)p * Z + z;
            zscore[o] = bv;
            zn[o] = bn;
            zmir[o] = bm;
            zcm1[o] = Cb[(bn - 1 + N) % N];
            zcp1[o] = Cb[(bn + 1) % N];
          }
        }
      }
      free(PT);
      free(C0);
      free(C1);
    }
  }
  if (cb)
    for (int p = 0; p < n_pat; ++p) free(cb[p]);
  if (cs)
    for (int p = 0; p < n_pat; ++p) free(cs[p]);
  if (cx)
    for (int p = 0; p < n_pat; ++p) free(cx[p]);
  free(cb);
  free(cs);
  free(cx);
  free(nnz);
  return fail ? -1 : 0;
}

int acom_oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
