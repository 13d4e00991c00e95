/* FP64 direct-sum correlation over many patterns (plain C, OpenMP over patterns).
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
#pragma omp parallel
  {
    double* X = (double*)malloc(sizeof(double) * (size_t)N * R);
    int* cb = (int*)malloc(sizeof(int) * (size_t)N * R);
    int* cs = (int*)malloc(sizeof(int) * (size_t)N * R);
    double* cx = (double*)malloc(sizeof(double) * (size_t)N * R);
    double* C = (double*)malloc(sizeof(double) * 2 * (size_t)N);
    if (!X || !cb || !cs || !cx || !C) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int p = 0; p < n_pat; ++p) {
        polar_image(N, R, q_s, (int)offsets[p], (int)offsets[p + 1], qx, qy, I, delta, gamma,
                    omega, kind, sigma, X);
        int J = 0;
        for (int a = 0; a < N; ++a)
          for (int s = 0; s < R; ++s)
            if (X[(size_t)a * R + s] != 0.0) {
              cb[J] = a;
              cs[J] = s;
              cx[J] = X[(size_t)a * R + s];
              ++J;
            }
        for (int z = 0; z < Z; ++z) {
          const double* Pz = P + (size_t)z * N * R;
          for (int n = 0; n < 2 * N; ++n) C[n] = 0.0;
          for (int j = 0; j < J; ++j) {
            const int b = cb[j], s = cs[j];
            const double x = cx[j];
            for (int n = 0; n < N; ++n) {
              int i0 = ((b - n) % N + N) % N;
              int i1 = ((-b - n) % N + 2 * N) % N;
              C[2 * n] += x * Pz[(size_t)i0 * R + s];
              C[2 * n + 1] += x * Pz[(size_t)i1 * R + s];
            }
          }
          int best = 0;
          for (int i = 1; i < 2 * N; ++i)
            if (C[i] > C[best]) best = i;
          const int n = best / 2, mi = best % 2;
          const size_t o = (size_t)p * Z + z;
          zscore[o] = C[best];
          zn[o] = n;
          zmir[o] = mi;
          zcm1[o] = C[2 * ((n - 1 + N) % N) + mi];
          zcp1[o] = C[2 * ((n + 1) % N) + mi];
        }
      }
    }
    free(X);
    free(cb);
    free(cs);
    free(cx);
    free(C);
  }
  return fail ? -1 : 0;
}

int acom_oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
