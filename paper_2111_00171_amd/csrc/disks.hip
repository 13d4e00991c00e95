// Bragg disk detection on raw diffraction frames (Methods > Correlation
// Pattern Matching and Software Implementation: each pattern's peak list comes
// from correlating the frame with the image of the probe over vacuum, the
// correlation maxima being the disk positions and the correlation value the
// peak intensity).
//
// One workgroup per N x N frame (N = 64 or 128), the whole correlation in LDS:
//   frame -> packed complex rows z_j = f[2j] + i f[2j+1] -> FFT along x
//   -> split into the half spectra of the rows (columns kx = 0 and N/2, both
//      real, packed into one complex column) -> FFT along y
//   -> times the conjugate probe spectrum (1/N^2 folded in) -> inverse FFT
//      along y -> re-pack two rows per complex sequence -> inverse FFT along x
//   -> C[2j][x] = Re, C[2j+1][x] = Im.
// Every FFT pass maps lanes to sequences (N/2 of them) and butterflies to
// positions along the transform, so each LDS access of a pass is a run of
// consecutive complex words; the two transposes are the split and re-pack
// steps.  Then, on C: strict 3x3 maxima in the interior, a threshold relative
// to the largest one, ranking by (C descending, raster index ascending),
// greedy minimum spacing in one wave, and the per-axis parabolic vertex.
#include <cmath>

#include "acom_internal.h"

namespace acom {
hipError_t launch_scan_counts(const int32_t* counts, int n, int64_t* offsets, hipStream_t s);

namespace {

constexpr int kDiskMaxCand = 1024;
constexpr int kDiskMaxPeaks = 256;

template <int N>
struct DiskShape;
template <>
struct DiskShape<64> {
  static constexpr int R1 = 8, R2 = 8, NT = 256;
};
template <>
struct DiskShape<128> {
  static constexpr int R1 = 16, R2 = 8, NT = 512;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot_i(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = rot_i<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// cos and sin of 2 pi k / 16, k < 8.
constexpr float kCos16[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                             0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
constexpr float kSin16[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                             1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};

// In-register DFT of length R (4, 8 or 16) by radix-2 decimation in time:
// X_k = E_k + W^k O_k, X_{k+R/2} = E_k - W^k O_k, W = exp(-+2 pi i / R).
template <int R, bool INV>
struct SmallDft {
  static_assert(R == 8 || R == 16, "radix 4, 8 or 16");
  __device__ __forceinline__ static void run(float2* v) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    SmallDft<R / 2, INV>::run(e);
    SmallDft<R / 2, INV>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      float2 t;
      if (k == 0) {
        t = o[k];
      } else if (4 * k == R) {
        t = rot_i<INV>(o[k]);
      } else {
        const float c = kCos16[k * (16 / R)], sn = kSin16[k * (16 / R)];
        t = cmul(make_float2(c, INV ? sn : -sn), o[k]);
      }
      v[k] = cadd(e[k], t);
      v[k + R / 2] = csub(e[k], t);
    }
  }
};
template <bool INV>
struct SmallDft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }
};

// One Stockham pass of radix R over all N/2 sequences stored as buf[pos * P + seq]
// (Ns = product of the earlier radices).  Reads everything into registers,
// waits, writes the permuted outputs, waits.
template <int N, int NT, int R, int Ns, bool INV>
__device__ __forceinline__ void fft_pass(float2* buf, const float2* tw) {
  constexpr int H = N / 2, P = H + 1, NB = N / R, PER = H * NB / NT;
  static_assert(H * NB % NT == 0, "butterflies per pass must split evenly over the threads");
  const int tid = threadIdx.x;
  float2 v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * NT, s = idx % H, b = idx / H;
#pragma unroll
    for (int r = 0; r < R; ++r) v[q][r] = buf[(b + r * NB) * P + s];
    if (Ns > 1) {
      const int step = (b % Ns) * (N / (Ns * R));
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * step];
        if (INV) w.y = -w.y;
        v[q][r] = cmul(v[q][r], w);
      }
    }
    SmallDft<R, INV>::run(v[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * NT, s = idx % H, b = idx / H;
    const int base = (b / Ns) * Ns * R + (b % Ns);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[(base + r * Ns) * P + s] = v[q][r];
  }
  __syncthreads();
}

template <int N, bool INV>
__device__ __forceinline__ void fft_all(float2* buf, const float2* tw) {
  using S = DiskShape<N>;
  fft_pass<N, S::NT, S::R1, 1, INV>(buf, tw);
  fft_pass<N, S::NT, S::R2, S::R1, INV>(buf, tw);
  static_assert(S::R1 * S::R2 == N, "two passes cover the transform");
}

// The column stage without a round trip between the transforms: forward
// pass B of the column FFT (radix R2 over positions b + r N/R2, b < R1) leaves
// each thread the frequencies f = b + R1 r of its sequence; it multiplies them
// by the conjugate probe spectrum and, since the inverse transform splits as
// x[m + R2 j] = sum_b W_N^{-bm} W_R1^{-bj} Y_b[m] with
// Y_b[m] = sum_r X[b + R1 r] W_R2^{-rm}, takes the R2-point inverse DFT over r
// in registers and writes Y_b[m] at position m R1 + b.  Column 0 holds
// F0 + i F_H (the DC and Nyquist columns), whose product needs X[f] and
// X[N - f]: its threads exchange them through `xch`.
template <int N>
__device__ __forceinline__ void col_forward_product_inverse1(float2* buf, const float2* tw, const float2* spec,
                                                             float2* xch) {
  using S = DiskShape<N>;
  constexpr int H = N / 2, P = H + 1, R1 = S::R1, R2 = S::R2, NB = N / R2, PER = H * R1 / S::NT;
  static_assert(H * R1 % S::NT == 0 && R1 * R2 == N, "one forward pass B per thread and butterfly");
  const int tid = threadIdx.x;
  float2 v[PER][R2];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * S::NT, sq = idx % H, b = idx / H;
#pragma unroll
    for (int r = 0; r < R2; ++r) v[q][r] = buf[(b + r * NB) * P + sq];
#pragma unroll
    for (int r = 1; r < R2; ++r) v[q][r] = cmul(v[q][r], tw[r * b]);
    SmallDft<R2, false>::run(v[q]);  // v[q][r] = X[b + R1 r]
    if (sq == 0) {
#pragma unroll
      for (int r = 0; r < R2; ++r) xch[b + R1 * r] = v[q][r];
    }
  }
  __syncthreads();  // every load above is done, and column 0's spectrum is in xch
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * S::NT, sq = idx % H, b = idx / H;
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int f = b + R1 * r;
      if (sq == 0) {
        // split F0 + i F_H at f and N - f, multiply each, re-pack G0 + i G_H
        const float2 z = v[q][r], zm = xch[(N - f) & (N - 1)];
        const float2 f0 = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
        const float2 fh = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
        const float2 g0 = cmul(f0, spec[f * (H + 1)]), gh = cmul(fh, spec[f * (H + 1) + H]);
        v[q][r] = make_float2(g0.x - gh.y, g0.y + gh.x);
      } else {
        v[q][r] = cmul(v[q][r], spec[f * (H + 1) + sq]);
      }
    }
    SmallDft<R2, true>::run(v[q]);  // v[q][m] = Y_b[m]
#pragma unroll
    for (int m = 0; m < R2; ++m) buf[(m * R1 + b) * P + sq] = v[q][m];
  }
  __syncthreads();
}

// Second inverse stage of the column transform: for each m, the twiddles
// W_N^{-bm} and an R1-point inverse DFT over b give x[m + R2 j], j < R1.
template <int N>
__device__ __forceinline__ void col_inverse2(float2* buf, const float2* tw) {
  using S = DiskShape<N>;
  constexpr int H = N / 2, P = H + 1, R1 = S::R1, R2 = S::R2, PER = H * R2 / S::NT;
  static_assert(H * R2 % S::NT == 0, "inverse butterflies must split evenly over the threads");
  const int tid = threadIdx.x;
  float2 v[PER][R1];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * S::NT, sq = idx % H, m = idx / H;
#pragma unroll
    for (int b = 0; b < R1; ++b) v[q][b] = buf[(m * R1 + b) * P + sq];
#pragma unroll
    for (int b = 1; b < R1; ++b) {
      float2 w = tw[b * m];
      w.y = -w.y;
      v[q][b] = cmul(v[q][b], w);
    }
    SmallDft<R1, true>::run(v[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * S::NT, sq = idx % H, m = idx / H;
#pragma unroll
    for (int j = 0; j < R1; ++j) buf[(m + R2 * j) * P + sq] = v[q][j];
  }
  __syncthreads();
}

// Forward twiddles exp(-2 pi i t / N), t < N.
template <int N>
__device__ __forceinline__ void make_twiddles(float2* tw) {
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    float s, c;
    sincospif(2.0f * (float)t / (float)N, &s, &c);
    tw[t] = make_float2(c, -s);
  }
}

// Row spectra (Z-view, pos = kx, seq = row pair j) -> column layout (S-view,
// pos = y, seq = kx), kx = 0 and N/2 packed as one complex column.  Lanes run
// over kx: the reads step by one LDS row, the writes are consecutive.
template <int N>
__device__ __forceinline__ void split_rows(float2* buf) {
  using S = DiskShape<N>;
  constexpr int H = N / 2, P = H + 1, PER = H * H / S::NT;
  const int tid = threadIdx.x;
  float2 lo[PER], hi[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * S::NT, k = idx % H, j = idx / H;
    const float2 a = buf[k * P + j];
    const float2 b = buf[(k == 0 ? H : N - k) * P + j];
    if (k == 0) {
      lo[q] = make_float2(a.x, b.x);  // row 2j: DC, Nyquist
      hi[q] = make_float2(a.y, b.y);  // row 2j+1
    } else {
      // A = (Z_k + conj Z_{N-k}) / 2, B = (Z_k - conj Z_{N-k}) / (2i)
      lo[q] = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
      hi[q] = make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x));
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * S::NT, k = idx % H, j = idx / H;
    buf[(2 * j) * P + k] = lo[q];
    buf[(2 * j + 1) * P + k] = hi[q];
  }
  __syncthreads();
}

// Inverse of split_rows: half spectra of rows 2j, 2j+1 -> Z_k = A_k + i B_k
// over the full kx range (A_{N-k} = conj A_k); lanes over kx.
template <int N>
__device__ __forceinline__ void join_rows(float2* buf) {
  using S = DiskShape<N>;
  constexpr int H = N / 2, P = H + 1, PER = H * H / S::NT;
  const int tid = threadIdx.x;
  float2 u[PER], w[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * S::NT, k = idx % H, j = idx / H;
    const float2 A = buf[(2 * j) * P + k];
    const float2 B = buf[(2 * j + 1) * P + k];
    if (k == 0) {
      u[q] = make_float2(A.x, B.x);  // Z_0
      w[q] = make_float2(A.y, B.y);  // Z_{N/2}
    } else {
      u[q] = make_float2(A.x - B.y, A.y + B.x);   // A + iB
      w[q] = make_float2(A.x + B.y, -A.y + B.x);  // conj A + i conj B
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * S::NT, k = idx % H, j = idx / H;
    buf[k * P + j] = u[q];
    buf[(k == 0 ? H : N - k) * P + j] = w[q];
  }
  __syncthreads();
}

// Forward 2-D spectrum of the N x N real image img(y, x) (a device functor)
// into buf in the S-view.
template <int N, class Img>
__device__ __forceinline__ void forward_2d(float2* buf, const float2* tw, Img img) {
  using S = DiskShape<N>;
  constexpr int H = N / 2, P = H + 1;
  for (int idx = threadIdx.x; idx < H * N; idx += S::NT) {
    const int x = idx % N, j = idx / N;
    buf[x * P + j] = make_float2(img(2 * j, x), img(2 * j + 1, x));
  }
  __syncthreads();
  fft_all<N, false>(buf, tw);
  split_rows<N>(buf);
  fft_all<N, false>(buf, tw);
}

struct DiskArgs {
  const float* frames;
  int64_t n;
  const float2* spec;  // N x (N/2 + 1)
  float min_rel, min_abs, cy, cx, r2_excl, pixel_size;
  int edge, spacing2, max_peaks;
  int32_t* counts;
  float *qx, *qy, *I;
  int32_t* pix;
  int32_t* flags;
};

template <int N>
struct DiskLds {
  float2 buf[N * (N / 2 + 1)];
  float2 tw[N];
  float2 xch[N];  // column 0's spectrum during the product
  float cand_v[kDiskMaxCand];
  int32_t cand_i[kDiskMaxCand];
  int16_t order[kDiskMaxCand];
  float red[DiskShape<N>::NT / 64];
  int32_t wsum[DiskShape<N>::NT / 64];
};

template <int N>
__global__ void __launch_bounds__(DiskShape<N>::NT) disk_template_kernel(const float* probe, int cy0, int cx0,
                                                                         float2* spec) {
  constexpr int H = N / 2, P = H + 1;
  __shared__ float2 buf[N * P];
  __shared__ float2 tw[N];
  make_twiddles<N>(tw);
  __syncthreads();
  auto img = [&](int y, int x) { return probe[((y + cy0) & (N - 1)) * N + ((x + cx0) & (N - 1))]; };
  forward_2d<N>(buf, tw, img);
  const float inv = 1.0f / (float)(N * N);
  for (int idx = threadIdx.x; idx < N * (H + 1); idx += blockDim.x) {
    const int y = idx / (H + 1), k = idx % (H + 1);
    float2 v;
    if (k == 0 || k == H) {
      // column 0 holds F0 + i F_H (both spectra of real columns)
      const float2 a = buf[y * P], b = buf[((N - y) & (N - 1)) * P];
      v = k == 0 ? make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y))
                 : make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x));
    } else {
      v = buf[y * P + k];
    }
    spec[idx] = make_float2(v.x * inv, -v.y * inv);  // conjugate, 1/N^2
  }
}

template <int N>
__global__ void __launch_bounds__(DiskShape<N>::NT) disk_detect_kernel(DiskArgs a) {
  using S = DiskShape<N>;
  constexpr int NT = S::NT, H = N / 2, P = H + 1, PIX = N * N / NT, NW = NT / 64;
  static_assert(PIX <= 32 && N % PIX == 0, "one run of at most 32 pixels of one row per thread");
  __shared__ DiskLds<N> L;
  const int p = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  make_twiddles<N>(L.tw);
  const float* f = a.frames + (size_t)p * (N * N);
  // ---- load: packed rows, Z-view (pos = x, seq = j); lanes over x, so each
  // wave reads 256 contiguous bytes of a row and writes one LDS column
#pragma unroll 4
  for (int idx = tid; idx < H * N; idx += NT) {
    const int x = idx % N, j = idx / N;
    L.buf[x * P + j] = make_float2(f[(2 * j) * N + x], f[(2 * j + 1) * N + x]);
  }
  __syncthreads();
  fft_all<N, false>(L.buf, L.tw);
  split_rows<N>(L.buf);
  // ---- column transform, product with conj(probe spectrum) / N^2, inverse
  fft_pass<N, NT, S::R1, 1, false>(L.buf, L.tw);
  col_forward_product_inverse1<N>(L.buf, L.tw, a.spec, L.xch);
  col_inverse2<N>(L.buf, L.tw);
  join_rows<N>(L.buf);
  fft_all<N, true>(L.buf, L.tw);
  // C(y, x) = component (y & 1) of buf[x * P + y / 2]
  const float* cf = reinterpret_cast<const float*>(L.buf);
  auto C = [&](int y, int x) { return cf[2 * (x * P + (y >> 1)) + (y & 1)]; };

  // ---- strict 3x3 maxima in the interior.  Thread: PIX consecutive pixels of
  // row y starting at x0; lanes run over y so that each read is 64 consecutive
  // words.  Its raster slot (y * N / PIX + run) orders the compaction.
  constexpr int RUNS = N / PIX;
  const int y = tid % N, run = tid / N, x0 = run * PIX;
  const int slot = y * RUNS + run;
  // interior pixels of the run as a bit mask (rows and columns at least `edge`
  // from the border); edge >= 1, so the rows above and below exist
  unsigned inmask = 0u;
  if (y >= a.edge && y < N - a.edge) {
    const int lo = max(x0, a.edge) - x0, hi = min(x0 + PIX, N - a.edge) - x0;
    if (hi > lo) inmask = (hi >= 32 ? 0xFFFFFFFFu : (1u << hi) - 1u) & ~((1u << lo) - 1u);
  }
  unsigned mask = 0u;
  float vmax = -INFINITY;
  if (inmask) {
    // fully unrolled over the run: column maxima of the rows above and below
    // slide along x; the two reads outside the frame (x0 - 1 < 0, x0 + PIX = N)
    // are clamped and only feed pixels outside the interior mask
    const int xl = max(x0 - 1, 0), xr = min(x0 + PIX, N - 1);
    float v0 = fmaxf(C(y - 1, xl), C(y + 1, xl)), m0 = C(y, xl);
    float v1 = fmaxf(C(y - 1, x0), C(y + 1, x0)), m1 = C(y, x0);
    const float dy2 = ((float)y - a.cy) * ((float)y - a.cy);
#pragma unroll
    for (int i = 0; i < PIX; ++i) {
      const int xn = i + 1 < PIX ? x0 + i + 1 : xr;
      const float v2 = fmaxf(C(y - 1, xn), C(y + 1, xn)), m2 = C(y, xn);
      const float nb = fmaxf(fmaxf(v0, v1), fmaxf(fmaxf(v2, m0), m2));
      const float dx = (float)(x0 + i) - a.cx;
      if (m1 > nb && fmaf(dx, dx, dy2) >= a.r2_excl) {
        mask |= 1u << i;
        vmax = fmaxf(vmax, m1);
      }
      v0 = v1; m0 = m1;
      v1 = v2; m1 = m2;
    }
    // pixels outside the interior never count, nor does their maximum
    if (mask & ~inmask) {
      mask &= inmask;
      vmax = -INFINITY;
      for (unsigned m = mask; m; m &= m - 1u) vmax = fmaxf(vmax, C(y, x0 + __builtin_ctz(m)));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
  if (lane == 0) L.red[wave] = vmax;
  __syncthreads();
  float cmax = L.red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) cmax = fmaxf(cmax, L.red[w]);
  const float thr = fmaxf(a.min_abs, a.min_rel * cmax);
  // ---- candidates above the threshold, compacted in raster order: counts by
  // raster slot, an exclusive scan over the slots, then each run writes its own
  int cnt = 0;
  for (unsigned m = mask; m; m &= m - 1u) cnt += C(y, x0 + __builtin_ctz(m)) > thr;
  L.order[slot] = (int16_t)cnt;
  __syncthreads();
  const int mine = L.order[tid];
  int incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) L.wsum[wave] = incl;
  __syncthreads();
  int before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    before += w < wave ? L.wsum[w] : 0;
    total += L.wsum[w];
  }
  L.order[tid] = (int16_t)min(before + incl - mine, kDiskMaxCand);
  __syncthreads();
  int pos = L.order[slot];
  for (unsigned m = mask; m; m &= m - 1u) {
    const int x = x0 + __builtin_ctz(m);
    const float v = C(y, x);
    if (v > thr) {
      if (pos < kDiskMaxCand) {
        L.cand_v[pos] = v;
        L.cand_i[pos] = y * N + x;
      }
      ++pos;
    }
  }
  __syncthreads();
  const int K = min(total, kDiskMaxCand);
  // ---- rank by (C descending, raster index ascending)
  for (int i = tid; i < K; i += NT) {
    const float vi = L.cand_v[i];
    const int ii = L.cand_i[i];
    int rank = 0;
    for (int j = 0; j < K; ++j) {
      const float vj = L.cand_v[j];
      rank += (vj > vi) || (vj == vi && L.cand_i[j] < ii);
    }
    L.order[rank] = (int16_t)i;
  }
  __syncthreads();
  if (wave != 0) return;
  // ---- greedy minimum spacing, one wave; lane l keeps peaks l, l + 64, ...
  constexpr int KS = kDiskMaxPeaks / 64;
  int ky[KS], kx[KS];
#pragma unroll
  for (int c = 0; c < KS; ++c) ky[c] = kx[c] = 0;
  int m = 0;
  for (int r = 0; r < K && m < a.max_peaks; ++r) {
    const int ci = L.cand_i[L.order[r]];
    const int cy = ci / N, cx = ci % N;
    bool clash = false;
#pragma unroll
    for (int c = 0; c < KS; ++c) {
      const int t = c * 64 + lane;
      const int ddy = cy - ky[c], ddx = cx - kx[c];
      clash |= t < m && ddy * ddy + ddx * ddx < a.spacing2;
    }
    if (__ballot(clash) == 0ull) {
#pragma unroll
      for (int c = 0; c < KS; ++c)
        if (m == c * 64 + lane) {
          ky[c] = cy;
          kx[c] = cx;
        }
      ++m;
    }
  }
  // ---- parabolic vertex per axis, outputs in keep order
  const int64_t o = (int64_t)p * a.max_peaks;
#pragma unroll
  for (int c = 0; c < KS; ++c) {
    const int t = c * 64 + lane;
    if (t < m) {
      const int py = ky[c], px = kx[c];
      const float c0 = C(py, px);
      const float xm = C(py, px - 1), xp = C(py, px + 1), ym = C(py - 1, px), yp = C(py + 1, px);
      const float ddx = (xm - xp) / (2.0f * (xm - 2.0f * c0 + xp));
      const float ddy = (ym - yp) / (2.0f * (ym - 2.0f * c0 + yp));
      a.qx[o + t] = ((float)px + ddx - a.cx) * a.pixel_size;
      a.qy[o + t] = ((float)py + ddy - a.cy) * a.pixel_size;
      a.I[o + t] = c0;
      if (a.pix) a.pix[o + t] = py * N + px;
    }
  }
  if (lane == 0) {
    a.counts[p] = m;
    if (a.flags) a.flags[p] = total > kDiskMaxCand ? 1 : 0;
  }
}

__global__ void gather_peaks_kernel(int64_t n, int max_peaks, const int32_t* counts, const int64_t* offsets,
                                    const float* sqx, const float* sqy, const float* sI, float* qx, float* qy,
                                    float* I, int64_t capacity) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * max_peaks) return;
  const int64_t p = g / max_peaks;
  const int t = (int)(g % max_peaks);
  if (t >= counts[p]) return;
  const int64_t o = offsets[p] + t;
  if (o < 0 || o >= capacity) return;  // inconsistent offsets: never written outside the arrays
  qx[o] = sqx[g];
  qy[o] = sqy[g];
  I[o] = sI[g];
}

bool disk_size_ok(int32_t size) { return size == 64 || size == 128; }

}  // namespace
}  // namespace acom

using namespace acom;

extern "C" acom_status_t acom_disk_template(const float* probe, int32_t size, int32_t cy0, int32_t cx0,
                                            float* spectrum, void* stream) {
  if (!disk_size_ok(size)) return fail(ACOM_E_INVALID, "frame size must be 64 or 128");
  if (!probe || !spectrum) return fail(ACOM_E_INVALID, "probe and spectrum are required");
  if (cy0 < 0 || cy0 >= size || cx0 < 0 || cx0 >= size) return fail(ACOM_E_INVALID, "probe centre outside the frame");
  hipStream_t s = (hipStream_t)stream;
  if (size == 64)
    disk_template_kernel<64><<<1, DiskShape<64>::NT, 0, s>>>(probe, cy0, cx0, (float2*)spectrum);
  else
    disk_template_kernel<128><<<1, DiskShape<128>::NT, 0, s>>>(probe, cy0, cx0, (float2*)spectrum);
  ACOM_HIP(hipGetLastError());
  return ACOM_OK;
}

extern "C" acom_status_t acom_detect_disks(const float* frames, int64_t n, const float* spectrum,
                                           const acom_disk_params_t* prm, int32_t* counts, int64_t* offsets,
                                           float* slot_qx, float* slot_qy, float* slot_I, int32_t* slot_pixel,
                                           int32_t* flags, void* stream) {
  if (!prm) return fail(ACOM_E_INVALID, "params are required");
  const int N = prm->size;
  if (!disk_size_ok(N)) return fail(ACOM_E_INVALID, "frame size must be 64 or 128");
  if (n < 0 || n > (1 << 26)) return fail(ACOM_E_INVALID, "n must be in [0, 2^26]");
  if (prm->edge < 1 || prm->edge >= N / 2) return fail(ACOM_E_INVALID, "edge must be in [1, size/2)");
  if (prm->max_peaks < 1 || prm->max_peaks > kDiskMaxPeaks) return fail(ACOM_E_INVALID, "max_peaks must be in [1, 256]");
  if (prm->min_spacing < 0 || prm->min_spacing > 2 * N) return fail(ACOM_E_INVALID, "min_spacing must be in [0, 2 size]");
  if (!(prm->min_rel >= 0.0f) || !std::isfinite(prm->min_rel) || !std::isfinite(prm->min_abs))
    return fail(ACOM_E_INVALID, "min_rel must be finite and >= 0, min_abs finite");
  if (!(prm->pixel_size > 0.0f) || !std::isfinite(prm->pixel_size)) return fail(ACOM_E_INVALID, "pixel_size must be > 0");
  if (!std::isfinite(prm->center_y) || !std::isfinite(prm->center_x) || !(prm->exclusion_radius >= 0.0f) ||
      !std::isfinite(prm->exclusion_radius))
    return fail(ACOM_E_INVALID, "centre and exclusion radius must be finite (radius >= 0)");
  if (!offsets || (n > 0 && !counts)) return fail(ACOM_E_INVALID, "counts and offsets are required");
  if (((uintptr_t)frames & 15u) != 0) return fail(ACOM_E_INVALID, "frames must be 16-byte aligned");
  if (n > 0 && (!frames || !spectrum || !slot_qx || !slot_qy || !slot_I))
    return fail(ACOM_E_INVALID, "frames, spectrum and slot outputs are required");
  DiskArgs a;
  a.frames = frames;
  a.n = n;
  a.spec = (const float2*)spectrum;
  a.min_rel = prm->min_rel;
  a.min_abs = prm->min_abs;
  a.cy = prm->center_y;
  a.cx = prm->center_x;
  a.r2_excl = prm->exclusion_radius * prm->exclusion_radius;
  a.pixel_size = prm->pixel_size;
  a.edge = prm->edge;
  a.spacing2 = prm->min_spacing * prm->min_spacing;
  a.max_peaks = prm->max_peaks;
  a.counts = counts;
  a.qx = slot_qx;
  a.qy = slot_qy;
  a.I = slot_I;
  a.pix = slot_pixel;
  a.flags = flags;
  hipStream_t s = (hipStream_t)stream;
  if (n > 0) {
    if (N == 64)
      disk_detect_kernel<64><<<dim3((unsigned)n), DiskShape<64>::NT, 0, s>>>(a);
    else
      disk_detect_kernel<128><<<dim3((unsigned)n), DiskShape<128>::NT, 0, s>>>(a);
    ACOM_HIP(hipGetLastError());
  }
  ACOM_HIP(launch_scan_counts(counts, (int)n, offsets, s));
  return ACOM_OK;
}

extern "C" acom_status_t acom_gather_peaks(int64_t n, int32_t max_peaks, const int32_t* counts,
                                           const int64_t* offsets, const float* slot_qx, const float* slot_qy,
                                           const float* slot_I, float* qx, float* qy, float* intensity,
                                           int64_t capacity, void* stream) {
  if (n < 0 || n > (1 << 26)) return fail(ACOM_E_INVALID, "n must be in [0, 2^26]");
  if (max_peaks < 1 || max_peaks > kDiskMaxPeaks) return fail(ACOM_E_INVALID, "max_peaks must be in [1, 256]");
  if (capacity < 0) return fail(ACOM_E_INVALID, "negative capacity");
  if (n == 0) return ACOM_OK;
  if (!counts || !offsets || !slot_qx || !slot_qy || !slot_I || !qx || !qy || !intensity)
    return fail(ACOM_E_INVALID, "null argument");
  const int64_t total = n * max_peaks;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  gather_peaks_kernel<<<blocks, 256, 0, (hipStream_t)stream>>>(n, max_peaks, counts, offsets, slot_qx, slot_qy,
                                                             slot_I, qx, qy, intensity, capacity);
  ACOM_HIP(hipGetLastError());
  return ACOM_OK;
}
