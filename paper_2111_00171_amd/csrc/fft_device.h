// Block-cooperative mixed-radix FFTs in LDS (radices 8, 9, 4, 2, 3, 5).
//
// The angular axis phi3 is transformed many sequences at a time: element a of
// sequence q lives at buf[a * nseq + q], so consecutive threads touch
// consecutive LDS words.  Twiddles come from a table tw[m] = (cos, sin)(2 pi m / N).
//
// block_fft_inplace: in-place decimation in time.  With N = R_1 R_2 ... R_m, the
// transform of length L at level i splits into R_i transforms of length
// S = L / R_i over the inputs r + R_i n'' (r < R_i), stored contiguously, and
// combines them: X[k'' + S r'] = sum_r w_R^(r r') w_L^(r k'') Y_r[k''].  Levels
// run from the innermost (shortest) outwards, every butterfly reading and
// writing the same R positions, so one buffer suffices.  The input must be
// stored in digit-reversed order, x[n] at rev[n] with
// rev[n] = sum_i (N / (R_1 .. R_i)) * digit_i(n), digit_i the mixed-radix digits
// of n (least significant first); the output is in natural order.
//
// block_fft_inplace_ct<N, NSEQ> is the same transform with the length and the
// (power-of-two) sequence count known at compile time, so every index
// computation folds to shifts and constant divisions.
#pragma once

#include <hip/hip_runtime.h>

namespace acom {

constexpr int kMaxRadicesDev = 12;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i*sg  (sg = +1: forward transform sign e^{-i...})
__device__ __forceinline__ float2 rot_mi(float2 a, float sg) { return make_float2(sg * a.y, -sg * a.x); }

__device__ __forceinline__ void dft3(float2& a, float2& b, float2& d, float sg) {
  const float c = -0.5f, s = 0.866025403784438647f;
  const float2 t = cadd(b, d);
  const float2 m = make_float2(a.x + c * t.x, a.y + c * t.y);
  const float2 u = rot_mi(csub(b, d), sg);  // -i sg (b - d)
  a = cadd(a, t);
  b = make_float2(m.x + s * u.x, m.y + s * u.y);
  d = make_float2(m.x - s * u.x, m.y - s * u.y);
}

__device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d, float sg) {
  const float2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d);
  const float2 d1 = rot_mi(csub(b, d), sg);
  a = cadd(s0, s1);
  c = csub(s0, s1);
  b = cadd(d0, d1);
  d = csub(d0, d1);
}

// z * w with w = (cos t, -sg sin t): the forward transform's e^{-i t}
__device__ __forceinline__ float2 twid(float2 z, float c, float s, float sg) {
  const float sy = -sg * s;
  return make_float2(z.x * c - z.y * sy, z.x * sy + z.y * c);
}

// In-register R-point DFT, sign sg = +1 for exp(-2 pi i r k / R), -1 for exp(+...).
__device__ __forceinline__ void dft_small(float2* v, int R, float sg) {
  if (R == 8) {
    // two 4-point DFTs over the even and odd inputs, joined by w8^k
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3, sg);
    dft4(o0, o1, o2, o3, sg);
    const float h = 0.707106781186547524f;
    const float2 w1 = cadd(o1, rot_mi(o1, sg));                  // (1 - i sg) o1, times 1/sqrt2 below
    const float2 t1 = make_float2(h * w1.x, h * w1.y);
    const float2 t2 = rot_mi(o2, sg);                            // -i sg o2
    const float2 w3 = rot_mi(cadd(o3, rot_mi(o3, sg)), sg);      // -i sg (1 - i sg) o3
    const float2 t3 = make_float2(h * w3.x, h * w3.y);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1);
    v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2);
    v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3);
    v[7] = csub(e3, t3);
  } else if (R == 9) {
    // n = 3 n1 + n2, k = k1 + 3 k2: 3-point DFTs over n1, twiddles w9^(n2 k1),
    // 3-point DFTs over n2
    float2 y00 = v[0], y01 = v[3], y02 = v[6];
    float2 y10 = v[1], y11 = v[4], y12 = v[7];
    float2 y20 = v[2], y21 = v[5], y22 = v[8];
    dft3(y00, y01, y02, sg);
    dft3(y10, y11, y12, sg);
    dft3(y20, y21, y22, sg);
    const float c1 = 0.766044443118978035f, s1 = 0.642787609686539326f;   // 2 pi / 9
    const float c2 = 0.173648177666930349f, s2 = 0.984807753012208059f;   // 4 pi / 9
    const float c4 = -0.939692620785908384f, s4 = 0.342020143325668734f;  // 8 pi / 9
    y11 = twid(y11, c1, s1, sg);
    y12 = twid(y12, c2, s2, sg);
    y21 = twid(y21, c2, s2, sg);
    y22 = twid(y22, c4, s4, sg);
    dft3(y00, y10, y20, sg);
    dft3(y01, y11, y21, sg);
    dft3(y02, y12, y22, sg);
    v[0] = y00; v[3] = y10; v[6] = y20;
    v[1] = y01; v[4] = y11; v[7] = y21;
    v[2] = y02; v[5] = y12; v[8] = y22;
  } else if (R == 2) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (R == 3) {
    const float c = -0.5f, s = 0.866025403784438647f;
    float2 a = v[0], b = v[1], d = v[2];
    float2 t = cadd(b, d);
    float2 m = make_float2(a.x + c * t.x, a.y + c * t.y);
    float2 u = rot_mi(csub(b, d), sg);  // -i sg (b - d)
    v[0] = cadd(a, t);
    v[1] = make_float2(m.x + s * u.x, m.y + s * u.y);
    v[2] = make_float2(m.x - s * u.x, m.y - s * u.y);
  } else if (R == 4) {
    float2 a = v[0], b = v[1], c = v[2], d = v[3];
    float2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d);
    float2 d1 = rot_mi(csub(b, d), sg);
    v[0] = cadd(s0, s1);
    v[2] = csub(s0, s1);
    v[1] = cadd(d0, d1);
    v[3] = csub(d0, d1);
  } else {  // R == 5
    const float c1 = 0.309016994374947424f, c2 = -0.809016994374947424f;
    const float s1 = 0.951056516295153572f, s2 = 0.587785252292473129f;
    float2 a0 = v[0];
    float2 p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
    float2 p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
    float2 r1 = make_float2(a0.x + c1 * p1.x + c2 * p2.x, a0.y + c1 * p1.y + c2 * p2.y);
    float2 r2 = make_float2(a0.x + c2 * p1.x + c1 * p2.x, a0.y + c2 * p1.y + c1 * p2.y);
    float2 i1 = rot_mi(make_float2(s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y), sg);
    float2 i2 = rot_mi(make_float2(s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y), sg);
    v[0] = make_float2(a0.x + p1.x + p2.x, a0.y + p1.y + p2.y);
    v[1] = cadd(r1, i1);
    v[4] = csub(r1, i1);
    v[2] = cadd(r2, i2);
    v[3] = csub(r2, i2);
  }
}

// q = n / d and r = n % d for 0 <= n < 2^20, 0 < d < 2^12, using a float
// reciprocal inv_d = 1/d and one correction step (exact in that range).
__device__ __forceinline__ int fdivmod(int n, int d, float inv_d, int* r) {
  int q = (int)((float)n * inv_d);
  int rem = n - q * d;
  if (rem < 0) {
    --q;
    rem += d;
  } else if (rem >= d) {
    ++q;
    rem -= d;
  }
  *r = rem;
  return q;
}

// In-place transform of `nseq` interleaved sequences of length N (input in
// digit-reversed order, output natural).  sg = +1 forward, -1 inverse
// (unnormalised).  All threads of the block must call it.
__device__ inline void block_fft_inplace(float2* buf, const float2* tw, int N, int nseq, const int* radix,
                                         int nrad, float sg) {
  int Ls[kMaxRadicesDev];
  int L = N;
  for (int i = 0; i < nrad; ++i) {
    Ls[i] = L;
    L /= radix[i];
  }
  const float inv_nseq = 1.0f / (float)nseq;
  for (int i = nrad - 1; i >= 0; --i) {
    const int R = radix[i];
    const int Li = Ls[i];
    const int S = Li / R;
    const int step = N / Li;
    const int items = (N / R) * nseq;
    const float inv_s = 1.0f / (float)S;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
      int q;
      const int t = fdivmod(it, nseq, inv_nseq, &q);
      int kk;
      const int b = fdivmod(t, S, inv_s, &kk);
      const int base = b * Li + kk;
      float2 v[9];
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        if (r < R) {
          float2 x = buf[(base + S * r) * nseq + q];
          if (r > 0 && kk > 0) {
            float2 w = tw[step * r * kk];  // step * r * kk < N
            w.y *= -sg;                    // forward uses conj(w)
            x = cmul(x, w);
          }
          v[r] = x;
        }
      }
      dft_small(v, R, sg);
#pragma unroll
      for (int r = 0; r < 9; ++r)
        if (r < R) buf[(base + S * r) * nseq + q] = v[r];
    }
    __syncthreads();
  }
}

struct RadixPlan {
  int n;
  int rest;  // 1 when N factors completely into 2, 3, 5
  int r[kMaxRadicesDev];
  int L[kMaxRadicesDev];
};

// Radices 8, 9, 4, 2, 3, 5 taken greedily in that order (the same
// factorisation the host uses for the digit-reversal table) and the level
// lengths L_0 = N, L_{i+1} = L_i / R_i.
__host__ __device__ constexpr RadixPlan make_radix_plan(int N) {
  RadixPlan p{};
  int m = N;
  const int fs[6] = {8, 9, 4, 2, 3, 5};
  for (int f = 0; f < 6; ++f)
    while (m % fs[f] == 0 && p.n < kMaxRadicesDev) {
      p.r[p.n++] = fs[f];
      m /= fs[f];
    }
  p.rest = m;
  int L = N;
  for (int i = 0; i < p.n; ++i) {
    p.L[i] = L;
    L /= p.r[i];
  }
  return p;
}

template <int N, int NSEQ, int LEVEL>
__device__ __forceinline__ void fft_level_ct(float2* buf, const float2* tw, float sg) {
  constexpr RadixPlan P = make_radix_plan(N);
  constexpr int R = P.r[LEVEL];
  constexpr int Li = P.L[LEVEL];
  constexpr int S = Li / R;
  constexpr int step = N / Li;
  constexpr int items = (N / R) * NSEQ;
  static_assert((NSEQ & (NSEQ - 1)) == 0, "power-of-two sequence count");
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int q = it % NSEQ;
    const int t = it / NSEQ;
    const int b = t / S, kk = t % S;
    const int base = b * Li + kk;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float2 x = buf[(base + S * r) * NSEQ + q];
      if (r > 0 && kk > 0) {
        float2 w = tw[step * r * kk];
        w.y *= -sg;
        x = cmul(x, w);
      }
      v[r] = x;
    }
    dft_small(v, R, sg);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[(base + S * r) * NSEQ + q] = v[r];
  }
  __syncthreads();
  if constexpr (LEVEL > 0) fft_level_ct<N, NSEQ, LEVEL - 1>(buf, tw, sg);
}

// Forward 360-point DFT (exp(-2 pi i n k / 360)) of NSEQ interleaved
// sequences in natural order, buf[n * NSEQ + q], in two LDS passes instead of
// three: 360 = 24 x 15 by Cooley-Tukey over n = n1 + 24 n2, k = k2 + 15 k1,
//   X[k2 + 15 k1] = sum_n1 W24^(n1 k1) W360^(n1 k2) sum_n2 W15^(n2 k2) x[n1 + 24 n2],
// each factor in registers by Good's prime-factor maps (15 = 3 x 5 with input
// (5 i + 3 j) mod 15 and output (10 i + 6 j) mod 15; 24 = 3 x 8 with input
// (8 i + 3 j) mod 24 and output (16 i + 9 j) mod 24: no inner twiddles).
// Pass 1 writes the twiddled 15-point spectra over n2 in place; pass 2 the
// 24-point spectra over n1, so frequency k ends at position
// (k / 15) + 24 (k % 15). tw[i] = exp(+2 pi i i / 360). Every thread calls;
// ends with a barrier.
template <int NSEQ>
__device__ __forceinline__ void block_fft360_fwd(float2* buf, const float2* tw) {
  for (int it = threadIdx.x; it < 24 * NSEQ; it += blockDim.x) {
    const int q = it % NSEQ, n1 = it / NSEQ;
    float2 a[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 5; ++j) a[i][j] = buf[(n1 + 24 * ((5 * i + 3 * j) % 15)) * NSEQ + q];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      float2 t[3] = {a[0][j], a[1][j], a[2][j]};
      dft_small(t, 3, 1.0f);
      a[0][j] = t[0];
      a[1][j] = t[1];
      a[2][j] = t[2];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) dft_small(a[i], 5, 1.0f);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const int k2 = (10 * i + 6 * j) % 15;
        float2 y = a[i][j];
        if (k2 > 0 && n1 > 0) {
          const float2 w = tw[n1 * k2];  // n1 k2 <= 23 * 14 < 360
          y = cmul(y, make_float2(w.x, -w.y));
        }
        buf[(n1 + 24 * k2) * NSEQ + q] = y;
      }
  }
  __syncthreads();
  for (int it = threadIdx.x; it < 15 * NSEQ; it += blockDim.x) {
    const int q = it % NSEQ, k2 = it / NSEQ;
    float2 a[3][8];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) a[i][j] = buf[((8 * i + 3 * j) % 24 + 24 * k2) * NSEQ + q];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float2 t[3] = {a[0][j], a[1][j], a[2][j]};
      dft_small(t, 3, 1.0f);
      a[0][j] = t[0];
      a[1][j] = t[1];
      a[2][j] = t[2];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) dft_small(a[i], 8, 1.0f);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) buf[((16 * i + 9 * j) % 24 + 24 * k2) * NSEQ + q] = a[i][j];
  }
  __syncthreads();
}
// Position of frequency k in the output of block_fft360_fwd.
__device__ __forceinline__ int fft360_pos(int k) { return k / 15 + 24 * (k % 15); }

template <int N, int NSEQ>
__device__ __forceinline__ void block_fft_inplace_ct(float2* buf, const float2* tw, float sg) {
  constexpr RadixPlan P = make_radix_plan(N);
  static_assert(P.n > 0 && P.rest == 1, "length must factor into 2, 3, 5");
  fft_level_ct<N, NSEQ, P.n - 1>(buf, tw, sg);
}

}  // namespace acom
