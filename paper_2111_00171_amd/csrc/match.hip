// Pattern matching against a built plan (Methods > Correlation Pattern Matching).
//
// Per chunk of patterns, three launches on the caller's stream:
//  1. polar_kernel   - sparse polar image X(phi_a, q_s) (Eq. image_polar) by a
//                      deterministic per-column splat in LDS, then the FFT of X
//                      along phi3 (in-place mixed-radix FFT, two real columns
//                      packed in one complex sequence); writes FFT{X} in FP32
//                      and, for the low-precision contraction, BF16/FP16 copies.
//  2. bound_kernel   - the per-frequency contraction
//                      G_k = sum_s FFT{P}^* FFT{X} (and the mirror G'_k with
//                      FFT{X}^*) on MFMA for a 64x64 (pattern x zone) tile,
//                      streaming over k and accumulating
//                      U = (1/N) sum_k w_k max(|G_k|, |G'_k|), an upper bound of
//                      max_n max(C, C_mirror) by the triangle inequality on the
//                      inverse DFT.
//  3. exact_kernel   - per pattern, zones in decreasing U are evaluated exactly
//                      in FP32 (contraction over s, inverse FFT along phi3 of
//                      C + i C_mirror, argmax over (n, branch)) until no remaining
//                      zone's widened bound can beat the top_k-th exact score;
//                      parabolic sub-bin offset and the orientation matrix.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <climits>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "acom_internal.h"
#include "fft_device.h"

namespace acom {
namespace {

constexpr int kThreads = 256;
constexpr int kPolarCols = 16;   // radial columns per column-mask word (and per pass of the narrow polar variant)
constexpr int kPeakCache = 256;  // peaks prepared at once by the 16-column polar pass (128 by the 32-column one)
constexpr int kBatch = 4;        // zones evaluated together by the exact pass
constexpr int kDefaultChunk = 16384;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;

__device__ __forceinline__ float powe(float x, float e) {
  if (e == 1.0f) return x;
  if (e == 0.5f) return sqrtf(x);
  if (e == 0.0f) return 1.0f;
  if (e == 2.0f) return x * x;
  return powf(x, e);
}

__device__ __forceinline__ double wrap_pi64(double x) {
  const double tp = 6.283185307179586476925286766559;
  return x - tp * rint(x / tp);
}

// Correlation kernel of distance d with inv = 1/delta (cone) or 1/(2 sigma^2) (Gaussian).
__device__ __forceinline__ float kern32(float d, float delta, float inv, float sigma3, int kind) {
  if (kind == ACOM_KERNEL_CONE) return d < delta ? 1.0f - d * inv : 0.0f;
  return d < sigma3 ? expf(-d * d * inv) : 0.0f;
}

__device__ __forceinline__ uint16_t to_bf16_bits(float v) {
  __hip_bfloat16 b = __float2bfloat16(v);
  return *reinterpret_cast<uint16_t*>(&b);
}
__device__ __forceinline__ uint16_t to_f16_bits(float v) {
  __half h = __float2half(v);
  return *reinterpret_cast<uint16_t*>(&h);
}
// Nonnegative v rounded up to the next representable 16-bit value when
// round-to-nearest went below it: the split bound's block norms never shrink.
__device__ __forceinline__ uint16_t to_bf16_bits_up(float v) {
  const uint16_t b = to_bf16_bits(v);
  return __uint_as_float((uint32_t)b << 16) < v ? (uint16_t)(b + 1) : b;
}
__device__ __forceinline__ uint16_t to_f16_bits_up(float v) {
  const uint16_t b = to_f16_bits(v);
  __half t;
  *reinterpret_cast<uint16_t*>(&t) = b;
  return __half2float(t) < v ? (uint16_t)(b + 1) : b;
}

// Store at a byte offset from a base: with a wave-uniform base and a 32-bit
// offset the compiler uses the scalar-base form of the global store (no
// 64-bit address arithmetic per lane).
template <class T, class V>
__device__ __forceinline__ void store_at(T* base, uint32_t byte_off, V v) {
  *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// v of the lane that DPP control CTRL selects (a quad permutation, a half-row
// or a row mirror: the source lane is always within the same 16 lanes)
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_move_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// (value, index) maximum over the wavefront, ties to the smaller index, the
// same pair in every lane (every lane active).  Within each row of 16 lanes by
// DPP moves (lanes 2i <-> 2i + 1, the lane pairs of a quad, then the mirrored
// half-row and row, whose lanes hold equal pairs by then); then the four row
// results, read by scalar lane reads.  The selection is a total order, so the
// result does not depend on the order of the comparisons.
__device__ __forceinline__ void wave_argmax(float& bv, int& bi) {
  auto take = [&](float ov, int oi) {
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  };
  take(dpp_move<0xB1>(bv), dpp_move_i<0xB1>(bi));
  take(dpp_move<0x4E>(bv), dpp_move_i<0x4E>(bi));
  take(dpp_move<0x141>(bv), dpp_move_i<0x141>(bi));
  take(dpp_move<0x140>(bv), dpp_move_i<0x140>(bi));
  float rv[4];
  int ri[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    rv[r] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bv), 16 * r));
    ri[r] = __builtin_amdgcn_readlane(bi, 16 * r);
  }
  bv = rv[0];
  bi = ri[0];
#pragma unroll
  for (int r = 1; r < 4; ++r) take(rv[r], ri[r]);
}

// XCD-aware block order: the hardware deals workgroup b to XCD b % 8, so
// logical work item w = (b % 8) * per + b / 8 gives every XCD a contiguous range
// of logical items (neighbouring tiles then share that XCD's L2).  The grid has
// 8 * per blocks; blocks with w >= total exit at once.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int per) { return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds; }
inline int xcd_blocks(int total, int* per) {
  *per = (total + kXcds - 1) / kXcds;
  return *per * kXcds;
}
// The same with the items dealt out in groups: XCD x takes the x-th run of B
// consecutive items of each group of 8 B (the whole device then works on 8 B
// neighbouring items at a time, each XCD still on consecutive ones), and the
// last, partial group is split into 8 ranges of `per` items.  B = 0 gives the
// single range per XCD of xcd_item.
__device__ __forceinline__ int xcd_item_grouped(int B, int nfull, int per) {
  const int j = (int)(blockIdx.x / kXcds), x = (int)(blockIdx.x % kXcds);
  if (j < nfull * B) return (j / B) * (kXcds * B) + x * B + j % B;
  return nfull * kXcds * B + x * per + (j - nfull * B);
}
inline int xcd_blocks_grouped(int total, int B, int* nfull, int* per) {
  *nfull = B > 0 ? total / (kXcds * B) : 0;
  const int rem = total - *nfull * kXcds * B;
  *per = (rem + kXcds - 1) / kXcds;
  return kXcds * (*nfull * B + *per);
}

// ------------------------------------------------------------ 1. polar ----

struct PolarArgs {
  int N, R, Rp, Nk, nrad;
  int rad[kMaxRadices];
  const float* qs;
  const float2* tw;
  const int* rev;
  float delta, rk, sigma, gamma, omega;
  int kernel;
  const int64_t* offsets;
  const float *qx, *qy, *I;
  int64_t total_peaks;
  int64_t p_begin;
  int np;
  // FFT{X}[p][k][s] at (p / 64) * ld_tile + k * ldk + (p % 64) * ldp + s (p local),
  // columns s < out_cols
  float *xr, *xi;
  size_t ld_tile, ldk;
  int ldp, out_cols;
  uint16_t *lr, *li;       // low-precision copies (rows k < Kc, then the norm rows; tile stride ld_tile16) or null
  size_t ld_tile16;
  int lowp;                // 0 none, ACOM_BF16, ACOM_FP16
  // split bound (workspace layout only), for the operands of the precision
  // matched: block norms w_k ||FFT{X}[k][b bb ..]|| of the frequencies k >= Kn
  // as entries v = (k - Kn) nb + b of the norm vector, j = v / 2Sp, at slot
  // r0 + v mod Sp of the real (v mod 2Sp < Sp) or imaginary array of FP32 row
  // Nk + j (lowp == 0) or 16-bit row Kc16 + j
  int ws_layout;           // 1: the workspace's tile-major layout (norms written), 0: a caller's layout
  int Kc16;                // 16-bit spectrum rows kept
  int Kn, bb, bb_log2, nb, Sp, r0, npseudo;
  int64_t L;
  float inv2sp;            // 1 / (2 Sp) in FP32: the row of an entry by a corrected FP32 quotient
  int inc_j, inc_e;        // (kThreads / NS) nb = inc_j 2Sp + inc_e: the norm position's advance per unpack step
  float* scale;            // np: factor applied before the FP16 cast (else 1)
  float* xnorm2;           // np: sum of X^2 of the pattern's polar image
  int* flags;              // np: 0 ok, 1 invalid data, 2 no peaks
  float* Ximg;             // optional X[p][a][s] (np x N x R)
  int do_fft;
  int ntiles;              // radial tiles of kPolarCols columns (column-mask words per pattern)
  int per;                 // > 0: XCD-grouped block order with this many items per XCD
  uint32_t* cmask;         // np x ntiles: bit c set when column c of the tile holds a nonzero X (or null)
  int* queue;              // kXcds counters of the persistent exact pass, zeroed here (or null)
};

// One workgroup per pattern, looping over its radial tiles of NC columns (16 or
// 32).  The peaks are prepared once per pattern (bin of the nearest angle
// ac, offset f, radius, weight) and, per tile, compacted to those whose radius
// lies within the kernel reach of the tile's columns.  Splat: thread (column c,
// part t) owns the angular bins a = t mod (256 / NC) of column c (interleaved,
// so that a peak's short window is shared by all parts; the parts of a column
// are consecutive threads) and adds the listed
// peaks' kernel there in peak order (no atomics, deterministic).  A peak
// at angle gamma sits at t = gamma / dphi = ac + f; the angle from bin ac + jj
// is then (jj - f) dphi, already wrapped while the window is shorter than the
// circle, so cells need only FP32 arithmetic.  Then the FFT along phi3 of the
// columns packed in pairs as complex sequences (skipped for a tile with no
// nonzero X, whose spectrum is exactly zero).  With NC = 32 the column pairs of
// a tile are 16 complex sequences, the FFT's butterflies fill the workgroup
// better, a (pattern, frequency) row segment of FP32 output is one 128-byte
// line, and there are half as many passes and barriers; the LDS (53 KiB at
// N = 360, peak cache of 128) still admits three workgroups per compute unit.
// NT > 0: angular length known at compile time (FFT specialised); NT = 0: any.
template <int NC>
constexpr int polar_peak_cache() {
  return NC == 32 ? 128 : kPeakCache;
}
template <int NT, int NC, int KIND>
__global__ void __launch_bounds__(kThreads, 3) polar_kernel(PolarArgs a) {
  static_assert(NC == 16 || NC == 32, "16 or 32 columns per pass");
  constexpr int PC = polar_peak_cache<NC>();
  constexpr int kParts = kThreads / NC;  // angular partitions of the splat
  static_assert(PC <= kThreads, "one thread prepares one cached peak");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NS = NC / 2;
  const int N = NT > 0 ? NT : a.N;
  float2* b0 = reinterpret_cast<float2*>(smem_raw);   // [rev(a)][NS] complex: columns packed in pairs
  float2* tw = b0 + N * NS;
  // the digit-reversed order of the input (other lengths), or for N = 360 the
  // output position of each frequency (a table lookup in place of two integer
  // divisions per spectrum value read by the unpack)
  int* rev = reinterpret_cast<int*>(tw + N);
  // per cached peak: nearest bin |ac| <= N/2 (int16), offset, radius as an
  // FP32 pair, weight; the listed peaks as cache indices (< 256, one byte):
  // narrow types keep the kernel small enough for three workgroups per CU
  int16_t* pac = reinterpret_cast<int16_t*>(rev + N);
  float* pf = reinterpret_cast<float*>(pac + PC);
  float* pq = pf + PC;
  float* pw = pq + PC;
  float* pql = pw + PC;  // q_m - pq (the radius as an FP32 pair)
  uint8_t* plist = reinterpret_cast<uint8_t*>(pql + PC);  // cached peaks reaching the current tile
  float* sqs = reinterpret_cast<float*>(plist + PC);  // q_s of every column (-1 beyond R)
  uint32_t* scmw = reinterpret_cast<uint32_t*>(sqs + a.Rp);  // [16-column tile][wave] column masks
  __shared__ int s_bad, s_nlist;
  __shared__ float s_red[kThreads / 64];
  __shared__ double s_red64[kThreads / 64];
  __shared__ float s_sc;

  // N = 360: X in natural angular order for the two-pass transform, whose
  // frequency k sits at fft360_pos(k); other lengths: digit-reversed input,
  // natural output
  constexpr bool kNat360 = NT == 360;
  auto xrow = [&](int ai) { return kNat360 ? ai : rev[ai]; };
  auto fpos = [&](int k) { return kNat360 ? rev[k] : k; };

  const int tid = threadIdx.x;
  const int p = a.per > 0 ? xcd_item(a.per) : (int)blockIdx.x;
  if (p >= a.np) return;
  if (p == 0 && a.queue && tid < kXcds) a.queue[tid] = 0;  // read only by the next kernels on the stream
  const int64_t P = a.p_begin + p;
  int64_t m0 = a.offsets[P], m1 = a.offsets[P + 1];
  const bool bad_range = m0 < 0 || m1 < m0 || m1 > a.total_peaks;
  if (bad_range) m0 = m1 = 0;  // malformed CSR row: a data error, nothing is read
  for (int i = tid; i < N; i += kThreads) {
    tw[i] = a.tw[i];
    rev[i] = kNat360 ? fft360_pos(i) : a.rev[i];
  }
  for (int i = tid; i < a.Rp; i += kThreads) sqs[i] = i < a.R ? a.qs[i] : -1.0f;
  if (tid == 0) s_bad = bad_range ? 1 : 0;
  // the flag is initialised before any wave's prep() may raise it
  __syncthreads();

  const double inv_dphi = N / 6.283185307179586476925286766559;
  const float dphi = (float)(6.283185307179586476925286766559 / N);
  const float pi_f = 3.14159265358979323846f;
  // the parts of one column are consecutive lanes: a wave covers 64 / kParts
  // whole columns, so the waves whose columns no listed peak reaches skip the
  // splat loop as a whole instead of idling lanes in every wave
  const int c = tid / kParts, part = tid % kParts;
  const float kinv = KIND == ACOM_KERNEL_CONE ? 1.0f / a.delta : 1.0f / (2.0f * a.sigma * a.sigma);
  const float sig3 = 3.0f * a.sigma;
  const bool single = (m1 - m0) <= PC;
  double wsum = 0.0;  // this thread's share of sum_m w_m (first pass over the peaks only)

  // cache peaks [c0, c0 + cnt): every thread calls; ends with a barrier
  auto prep = [&](int64_t c0, int cnt, bool count) {
    if (tid < cnt) {
      const float x = a.qx[c0 + tid], y = a.qy[c0 + tid], in = a.I[c0 + tid];
      const bool bad = !isfinite(x) || !isfinite(y) || !isfinite(in) || in < 0.0f;
      if (bad) atomicOr(&s_bad, 1);
      const double q = sqrt((double)x * x + (double)y * y);
      const double t = atan2((double)y, (double)x) * inv_dphi;
      const double tr = floor(t + 0.5);
      pac[tid] = (int16_t)tr;
      pf[tid] = (float)(t - tr);
      const float qh = (float)q;
      pq[tid] = qh;
      pql[tid] = (float)(q - (double)qh);
      const float w = bad ? 0.0f : powe((float)q, a.gamma) * powe(in, 0.5f * a.omega);
      // the splat accumulates X / 2 (an exact scaling): the unpack's
      // (Z_k + conj Z_{N-k}) / 2 then needs no multiplication
      pw[tid] = 0.5f * w;
      if (count) wsum += w;
    }
    __syncthreads();
  };
  if (single) prep(m0, (int)(m1 - m0), true);
  else __syncthreads();

  float sc = 1.0f;
  float xx = 0.0f;  // this thread's share of sum X^2 over all tiles (fixed order)
  float* X = reinterpret_cast<float*>(b0);  // X(phi_a, column) at [rev(a)][NC]
  const size_t pbase = (size_t)(p >> 6) * a.ld_tile + (size_t)(p & 63) * a.ldp;
  const size_t pbase16 = (size_t)(p >> 6) * a.ld_tile16 + (size_t)(p & 63) * a.ldp;
  const int npass = a.Rp / NC;
  for (int tile = 0; tile < npass; ++tile) {
    const int col0 = tile * NC;
    for (int i = tid; i < N * NC / 4; i += kThreads)
      reinterpret_cast<float4*>(X)[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    // radii of the tile's real columns (padding columns carry q = -1: no peak reaches them)
    const int cl = min(col0 + NC, a.R) - 1;
    const float qlo = col0 < a.R ? sqs[col0] : -1.0f;
    const float qhi = col0 < a.R ? sqs[cl] : -1.0f;
    const float qs = sqs[col0 + c];
    // the low part of this thread's own column, from global memory (an LDS
    // copy would cost the third workgroup per compute unit its room)
    const float qsl = col0 + c < a.R ? a.qs[a.Rp + col0 + c] : 0.0f;
    const float dqs = dphi * qs;
    int hw = N;  // half-width of the angular window of this column
    if (qs > 0.0f) {
      const float h = a.rk / dqs + 1.0f;
      hw = h > (float)N ? N : (int)ceilf(h);
    }
    const bool full = 2 * hw + 1 >= N;
    bool listed = false;  // some peak reaches the tile (else its X is exactly zero)
    __syncthreads();
    for (int64_t c0 = m0; c0 < m1; c0 += PC) {
      const int cnt = (int)min((int64_t)PC, m1 - c0);
      if (!single) prep(c0, cnt, tile == 0);
      // wave 0 lists, in peak order, the cached peaks within reach of [qlo, qhi]
      // (a reach widened by 1e-5 1/A over the per-column test below, which adds
      // the low parts of the radii, so no reached cell is dropped)
      if (tid < 64) {
        int base = 0;
        const float rl = a.rk + 1e-5f;
        for (int j0 = 0; j0 < cnt; j0 += 64) {
          const int j = j0 + tid;
          const bool hit = qlo >= 0.0f && j < cnt && pw[j] != 0.0f && (pq[j] - qhi < rl) && (qlo - pq[j] < rl);
          const unsigned long long m = __ballot(hit);
          if (hit) plist[base + __popcll(m & ((1ull << tid) - 1ull))] = (uint8_t)j;
          base += __popcll(m);
        }
        if (tid == 0) s_nlist = base;
      }
      __syncthreads();
      const int nl = s_nlist;
      listed = listed || nl > 0;
      // the kernel shape (KIND) is a compile-time constant; a cell adds w k
      // even where k = 0 (X >= 0, so X + 0 is X exactly)
      if (qs >= 0.0f) {
        for (int l = 0; l < nl; ++l) {
          const int j = plist[l];
          // q_m - q_s: the high parts are close, so their difference is exact
          // (Sterbenz) where it matters, and the low parts restore the rest
          const float dq = (pq[j] - qs) + (pql[j] - qsl);
          const float w = pw[j];
          if (fabsf(dq) >= a.rk) continue;
          const int ac = pac[j];
          const float f = pf[j];
          const float dq2 = dq * dq;
          if (full) {
            for (int ai = part; ai < N; ai += kParts) {
              int u = ai - ac;  // in (-3N/2, 3N/2): bring to [-N/2, N/2)
              if (u >= N / 2) u -= N;
              if (u < -N / 2) u += N;
              float xa = ((float)u - f) * dphi;
              if (xa > pi_f) xa -= 2.0f * pi_f;
              if (xa < -pi_f) xa += 2.0f * pi_f;
              const float dp = xa * qs;
              X[xrow(ai) * NC + c] += w * kern32(__builtin_amdgcn_sqrtf(dq2 + dp * dp), a.delta, kinv, sig3, KIND);
            }
          } else {
            // window [ac - hw, ac + hw] in unwrapped bins; fewer than N bins, so each
            // bin is met by at most one of the three shifts; this thread takes the
            // bins u - sh = part (mod kParts)
            const int wlo = ac - hw, whi = ac + hw + 1;
            for (int sh = -N; sh <= N; sh += N) {
              const int u0 = max(wlo, sh), u1 = min(whi, sh + N);
              if (u0 >= u1) continue;
              const int first = u0 + (part - (u0 - sh) % kParts + kParts) % kParts;
              for (int u = first; u < u1; u += kParts) {
                const float dp = ((float)(u - ac) - f) * dqs;
                X[xrow(u - sh) * NC + c] += w * kern32(__builtin_amdgcn_sqrtf(dq2 + dp * dp), a.delta, kinv, sig3, KIND);
              }
            }
          }
        }
      }
      __syncthreads();
    }
    if (tile == 0) {
      // the peak weights (FP16 scale) and the flags, before the first unpack
      double ws = wsum;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) ws += __shfl_xor(ws, off, 64);
      if ((tid & 63) == 0) s_red64[tid >> 6] = ws;
      __syncthreads();
      if (tid == 0) {
        double u = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) u += s_red64[w];
        float scl = 1.0f;
        if (a.lowp == ACOM_FP16) {
          // |FFT{X}| <= sum_a X <= N * sum_m w_m; map that bound below 2^12,
          // so that a weighted block norm (at most 2 sqrt(16) times it) stays
          // below the FP16 maximum.
          const double bound = u * N;
          if (bound > 0.0) {
            int e = (int)floor(log2(4096.0 / bound));
            e = max(-60, min(60, e));
            scl = ldexpf(1.0f, e);
          }
        }
        s_sc = scl;
        a.flags[p] = s_bad ? 1 : (m1 <= m0 ? 2 : 0);
        a.scale[p] = scl;
      }
      __syncthreads();
      sc = s_sc;
    }
    const bool bad = s_bad != 0;
    if (a.Ximg) {
      for (int i = tid; i < N * NC; i += kThreads) {
        const int ai = i / NC, cc = i % NC;
        if (col0 + cc < a.R) a.Ximg[((size_t)p * N + ai) * a.R + col0 + cc] = bad ? 0.0f : 2.0f * X[xrow(ai) * NC + cc];
      }
    }
    if (!a.do_fft) {
      __syncthreads();
      continue;
    }
    if (listed) {  // a tile of zeros has a zero spectrum: its LDS already holds it
      if constexpr (kNat360)
        block_fft360_fwd<NS>(b0, tw);
      else if constexpr (NT > 0)
        block_fft_inplace_ct<NT, NS>(b0, tw, 1.0f);
      else
        block_fft_inplace(b0, tw, N, NS, a.rad, a.nrad, 1.0f);
    }
    const float2* F = b0;
    // unpack: column 2q = (Z_k + conj Z_{N-k}) / 2, column 2q+1 = -i (Z_k - conj Z_{N-k}) / 2.
    // On the way: sum X^2 by Parseval (sum_a X_a^2 = (1/N) sum_k |Xhat_k|^2, the
    // half spectrum counted twice except k = 0 and N/2), and which columns have
    // a nonzero spectrum (a thread always holds pair q = tid % NS)
    // which columns have a nonzero spectrum: X >= 0, so a column is nonzero
    // exactly when its sum, the k = 0 term, is (column 2q is the real part of
    // sequence q, column 2q + 1 its imaginary part)
    bool nzE = false, nzO = false;
    if (tid < NS && !bad) {
      nzE = F[tid].x != 0.0f;
      nzO = F[tid].y != 0.0f;
    }
    // Z_k and Z_{N-k} of column pair q; k is clamped to Nk - 1 so that a
    // prefetch one loop step past the end stays inside the LDS buffer
    auto load_pair = [&](int k, int q, float2& Zk, float2& Zn) {
      k = min(k, a.Nk - 1);
      Zk = F[fpos(k) * NS + q];
      Zn = F[fpos(k == 0 ? 0 : N - k) * NS + q];
    };
    // the spectra of the pair: E = (Z_k + conj Z_{N-k}) / 2 for column 2q,
    // O = -i (Z_k - conj Z_{N-k}) / 2 for column 2q + 1 (the LDS holds the
    // transform of X / 2)
    auto pair_of = [](float2 Zk, float2 Zn, float2& E, float2& O) {
      E = make_float2(Zk.x + Zn.x, Zk.y - Zn.y);
      O = make_float2(Zk.y + Zn.y, Zn.x - Zk.x);
    };
    // weight of frequency k in the half spectrum (Parseval; the block norms)
    auto wk_of = [&](int k) { return (k == 0 || 2 * k == N) ? 1.0f : 2.0f; };
    if (a.ws_layout && bad) {
      // a flagged pattern: zero spectrum rows (the contraction reads them) and norms
      const int rows = a.lowp ? a.Kc16 : a.Nk;
      for (int it = tid; it < a.Nk * NS; it += kThreads) {
        const int k = it / NS, q = it % NS;
        const size_t o = pbase + (size_t)k * a.ldk + col0 + 2 * q;
        *reinterpret_cast<float2*>(a.xr + o) = make_float2(0.0f, 0.0f);
        *reinterpret_cast<float2*>(a.xi + o) = make_float2(0.0f, 0.0f);
        if (a.lowp && k < rows) {
          const size_t o16 = pbase16 + (size_t)k * a.ldk + col0 + 2 * q;
          *reinterpret_cast<uint32_t*>(a.lr + o16) = 0u;
          *reinterpret_cast<uint32_t*>(a.li + o16) = 0u;
        }
      }
      if (a.npseudo > 0 && tile == 0)
        for (int i = tid; i < a.npseudo * a.Rp; i += kThreads) {
          const int j = i / a.Rp, slot = i % a.Rp;
          if (a.lowp == 0) {
            a.xr[pbase + (size_t)(a.Nk + j) * a.ldk + slot] = 0.0f;
            a.xi[pbase + (size_t)(a.Nk + j) * a.ldk + slot] = 0.0f;
          } else {
            a.lr[pbase16 + (size_t)(a.Kc16 + j) * a.ldk + slot] = 0;
            a.li[pbase16 + (size_t)(a.Kc16 + j) * a.ldk + slot] = 0;
          }
        }
    } else if (a.ws_layout) {
      // workspace layout: the column pair is one aligned 8-byte / 4-byte store.
      // Frequencies k < Kn carry the spectrum (FP32, and the 16-bit copy: Kn is
      // Kc16 then); k >= Kn the FP32 spectrum and the block norms. The stores
      // go through buffer resources over this pattern's rows (32-bit offsets,
      // the base in scalar registers), and the operand precision is a
      // compile-time choice: no per-launch branch inside the loops.
      //
      // Steps it = it0 + tid + kThreads m (it0 a multiple of NS, so a thread
      // keeps its column pair q = tid % NS): two register sets alternate, the
      // next step's pair loading while the current one is processed.
      const int q = tid % NS, dk = kThreads / NS;
      auto steps = [&](int it0, int it1, auto&& body) {
        float2 ak, an, bk, bn;
        load_pair((it0 + tid) / NS, q, ak, an);
        for (int it = it0 + tid; it < it1; it += 2 * kThreads) {
          const int k = (int)((unsigned)it / NS);
          load_pair(k + dk, q, bk, bn);
          __builtin_amdgcn_sched_barrier(0);  // the loads issue here, not next to their use
          body(k, ak, an);
          if (it + kThreads < it1) {  // the same for all NS lanes of frequency k
            load_pair(k + 2 * dk, q, ak, an);
            __builtin_amdgcn_sched_barrier(0);
            body(k + dk, bk, bn);
          }
        }
      };
      auto unpack = [&](auto lp_c) {
        constexpr int LP = decltype(lp_c)::value;
        const int ldk = (int)a.ldk;
        // this pattern's rows: a base in scalar registers and 32-bit byte
        // offsets per lane (a 64-pattern tile of rows stays below 2 GiB)
        float* const xr_p = a.xr + pbase;
        float* const xi_p = a.xi + pbase;
        uint16_t* const lr_p = LP ? a.lr + pbase16 : nullptr;
        uint16_t* const li_p = LP ? a.li + pbase16 : nullptr;
        const int c2 = col0 + 2 * q;
        steps(0, a.Kn * NS, [&](int k, float2 ck, float2 cn) {
          float2 E, O;
          pair_of(ck, cn, E, O);
          xx += wk_of(k) * ((E.x * E.x + E.y * E.y) + (O.x * O.x + O.y * O.y));
          const uint32_t o = (uint32_t)(k * ldk + c2);
          store_at(xr_p, o * 4u, make_float2(E.x, O.x));
          store_at(xi_p, o * 4u, make_float2(E.y, O.y));
          if constexpr (LP == ACOM_BF16) {
            store_at(lr_p, o * 2u, (uint32_t)to_bf16_bits(E.x) | ((uint32_t)to_bf16_bits(O.x) << 16));
            store_at(li_p, o * 2u, (uint32_t)to_bf16_bits(E.y) | ((uint32_t)to_bf16_bits(O.y) << 16));
          } else if constexpr (LP == ACOM_FP16) {
            store_at(lr_p, o * 2u, (uint32_t)to_f16_bits(E.x * sc) | ((uint32_t)to_f16_bits(O.x * sc) << 16));
            store_at(li_p, o * 2u, (uint32_t)to_f16_bits(E.y * sc) | ((uint32_t)to_f16_bits(O.y * sc) << 16));
          }
        });
        if (a.Kn >= a.Nk) return;
        // block norms over the HB = bb / 2 column pairs of a radial block: they
        // sit on consecutive lanes of one frequency (NS is a multiple of HB),
        // which are active together; the sum runs over DPP lane moves. The
        // entry of (k, block b) is v = (k - Kn) nb + b, at slot r0 + e of the
        // real (e < Sp) or, with e - Sp, the imaginary half of norm row
        // j = v / 2Sp, e = v mod 2Sp. (j, e) start from a corrected FP32
        // quotient and advance by dk nb = inc_j 2Sp + inc_e per step.
        auto norms = [&](auto hb_c) {
          constexpr int HB = decltype(hb_c)::value;
          const int sp2 = 2 * a.Sp;
          float* const nr32 = xr_p + a.Nk * ldk + a.r0;
          float* const ni32 = xi_p + a.Nk * ldk + a.r0 - a.Sp;  // indexed by e >= Sp
          uint16_t* const nr16 = LP ? lr_p + a.Kc16 * ldk + a.r0 : nullptr;
          uint16_t* const ni16 = LP ? li_p + a.Kc16 * ldk + a.r0 - a.Sp : nullptr;
          const bool lead = (q & (HB - 1)) == 0;
          int j, e;
          {
            const int v = (tid / NS) * a.nb + (c2 >> a.bb_log2);
            j = (int)((float)v * a.inv2sp);
            e = v - j * sp2;
            if (e < 0) {
              --j;
              e += sp2;
            } else if (e >= sp2) {
              ++j;
              e -= sp2;
            }
          }
          steps(a.Kn * NS, a.Nk * NS, [&](int k, float2 ck, float2 cn) {
            float2 E, O;
            pair_of(ck, cn, E, O);
            const float wk = 2 * k == N ? 1.0f : 2.0f;  // k >= Kn > 0
            float n2 = (E.x * E.x + E.y * E.y) + (O.x * O.x + O.y * O.y);
            xx += wk * n2;
            const uint32_t o = (uint32_t)(k * ldk + c2);
            store_at(xr_p, o * 4u, make_float2(E.x, O.x));
            store_at(xi_p, o * 4u, make_float2(E.y, O.y));
            if constexpr (HB >= 2) n2 += dpp_move<0xB1>(n2);   // lanes 2i <-> 2i + 1
            if constexpr (HB >= 4) n2 += dpp_move<0x4E>(n2);   // lane pairs of a quad
            if constexpr (HB >= 8) n2 += dpp_move<0x141>(n2);  // the two quads of 8 lanes
            if (lead) {
              const float nrm = wk * __builtin_amdgcn_sqrtf(n2);
              const bool im = e >= a.Sp;
              const int no = j * ldk + e;
              if constexpr (LP == 0)
                (im ? ni32 : nr32)[no] = nrm;
              else if constexpr (LP == ACOM_BF16)
                (im ? ni16 : nr16)[no] = to_bf16_bits_up(nrm);
              else
                (im ? ni16 : nr16)[no] = to_f16_bits_up(nrm * sc);
            }
            e += a.inc_e;
            j += a.inc_j;
            if (e >= sp2) {
              e -= sp2;
              ++j;
            }
          });
        };
        switch (a.bb) {
          case 2: norms(std::integral_constant<int, 1>{}); break;
          case 4: norms(std::integral_constant<int, 2>{}); break;
          case 16: norms(std::integral_constant<int, 8>{}); break;
          default: norms(std::integral_constant<int, 4>{}); break;
        }
      };
      if (a.lowp == ACOM_BF16)
        unpack(std::integral_constant<int, ACOM_BF16>{});
      else if (a.lowp == ACOM_FP16)
        unpack(std::integral_constant<int, ACOM_FP16>{});
      else
        unpack(std::integral_constant<int, 0>{});
    } else {  // caller's [p][k][s] layout with s < out_cols (verification entry point)
      for (int it = tid; it < a.Nk * NS; it += kThreads) {
        const int k = it / NS, q = it % NS;
        float2 Zk, Zn, E, O;
        load_pair(k, q, Zk, Zn);
        pair_of(Zk, Zn, E, O);
        if (bad) E = O = make_float2(0.0f, 0.0f);
        xx += wk_of(k) * ((E.x * E.x + E.y * E.y) + (O.x * O.x + O.y * O.y));
        const int s0 = col0 + 2 * q;
        const size_t o = pbase + (size_t)k * a.ldk + s0;
        if (s0 < a.out_cols) {
          a.xr[o] = E.x;
          a.xi[o] = E.y;
        }
        if (s0 + 1 < a.out_cols) {
          a.xr[o + 1] = O.x;
          a.xi[o + 1] = O.y;
        }
      }
    }
    {
      static_assert(kThreads % NS == 0 && 64 % NS == 0, "a thread keeps its column pair across the unpack");
      const unsigned long long be = __ballot(nzE), bo = __ballot(nzO);
      uint32_t m = 0;  // bit c: column col0 + c has a nonzero spectrum in this wave's share
#pragma unroll
      for (int l = 0; l < NS; ++l) {  // lane l + NS j holds pair l
        bool e = false, o = false;
#pragma unroll
        for (int j = 0; j < 64 / NS; ++j) {
          e = e || ((be >> (l + NS * j)) & 1ull);
          o = o || ((bo >> (l + NS * j)) & 1ull);
        }
        m |= (e ? 1u : 0u) << (2 * l) | (o ? 1u : 0u) << (2 * l + 1);
      }
      if ((tid & 63) == 0) {
        constexpr int T16 = NC / kPolarCols;  // mask words per pass
#pragma unroll
        for (int h = 0; h < T16; ++h)
          scmw[(tile * T16 + h) * (kThreads / 64) + (tid >> 6)] = (m >> (kPolarCols * h)) & 0xFFFFu;
      }
    }
    __syncthreads();
  }
  // the norm rows' slots that hold no entry: below r0, and past the vector's end
  if (a.ws_layout && a.npseudo > 0 && a.do_fft) {
    // entry v = j 2Sp + part Sp + (slot - r0) of row j; slots below r0 and
    // entries past L hold no norm
    for (int j = 0; j < a.npseudo; ++j)
      for (int e = tid; e < 2 * a.Rp; e += kThreads) {
        const int part = e >= a.Rp, slot = e - part * a.Rp;
        const int64_t v = (int64_t)j * 2 * a.Sp + part * a.Sp + (slot - a.r0);
        if (slot >= a.r0 && v < a.L) continue;
        if (a.lowp == 0)
          (part ? a.xi : a.xr)[pbase + (size_t)(a.Nk + j) * a.ldk + slot] = 0.0f;
        else
          (part ? a.li : a.lr)[pbase16 + (size_t)(a.Kc16 + j) * a.ldk + slot] = 0;
      }
  }
  // per pattern: sum of X^2 (fixed order) and the column masks of every tile
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) xx += __shfl_xor(xx, off, 64);
  if ((tid & 63) == 0) s_red[tid >> 6] = xx;
  __syncthreads();
  const bool bad = s_bad != 0;
  if (tid == 0) {
    float t = 0.0f;
    for (int w = 0; w < kThreads / 64; ++w) t += s_red[w];
    a.xnorm2[p] = bad ? 0.0f : t / (float)N;
  }
  if (a.cmask)
    for (int t = tid; t < a.ntiles; t += kThreads) {
      uint32_t m = 0;
      for (int w = 0; w < kThreads / 64; ++w) m |= scmw[t * (kThreads / 64) + w];
      a.cmask[(size_t)p * a.ntiles + t] = bad ? 0u : m;
    }
}

// ------------------------------------------------------------ 2. bound ----

struct BoundArgs {
  int Nk, Rp, N;
  // split bound: logical frequencies kk < Kc are the spectrum rows kk (the
  // larger modulus of G_k and G'_k), kk in [Kc, nlog) the norm rows
  // hi + kk - Kc (sum of the products of block norms); rows per 64-row tile
  int Kc, nlog, hi, rows;
  int nP, nZ, per;          // block tiles over patterns and zones, XCD items per XCD
  int nX64, nP64;           // 64-row layout tiles of the pattern and zone operands
  int r0;                   // leading radii where the plan is zero in every zone
  int order;                // block order (see bound_kernel)
  const void *xr, *xi;      // tile-major over patterns (local to the chunk)
  const void *pr, *pi;      // tile-major over zones
  const float* scale;       // per local pattern
  float* U;
  int ldU, np, Zvalid;
};

// Operand element type per kind (0: FP32, 1: BF16, 2: FP16).
template <int KIND>
struct BoundTraits {
  typedef uint16_t T;
};
template <>
struct BoundTraits<0> {
  typedef float T;
};

// Contraction.  One workgroup: 64 patterns x 64 zones, 4 waves of 32 x 32 (2 x 2
// MFMA blocks of 16 x 16).  For each frequency k the K loop runs over s in
// steps of KCH radii (KCH divides Rp); four accumulators per block give the
// real products A = Xr Pr, B = Xi Pi, C = Xi Pr, D = Xr Pi, so
// G = (A + B) + i (C - D) and G_mirror = (A - B) - i (C + D), whose larger
// squared modulus is S + 2 |T| with S = A^2 + B^2 + C^2 + D^2, T = A B - C D
// (one square root per element and frequency).  Both operands use the same
// assignment of radii to lanes (a permutation of the contraction index).
//
// Pipeline: the operand tiles of step stp + 1 travel from global memory
// straight into LDS (global_load_lds_dwordx4, no registers) while the MFMAs of
// step stp run on the other of two LDS buffers, with one barrier per step.  A
// staged row holds KCH radii (RB = 64, 128 or 256 bytes) with no padding; its
// 16-byte chunks are XOR-permuted by row so that the 16 rows one quarter-wave
// reads for an MFMA operand (one 16-byte chunk each) meet no LDS bank conflict.
// The permutations were chosen by measurement on gfx950 (ds_read_b128 rate of
// each pattern): for 64-byte rows (row >> 1) & 3 is conflict-free while
// (row >> 2) & 3 runs at two thirds of the rate.
template <int RB>
__device__ __forceinline__ int chunk_swizzle(int row) {
  return RB == 64 ? ((row >> 1) & 3) : RB == 128 ? ((row >> 1) & 7) : (row & 15);
}

template <int KIND, int KCH, int WM, int WN, int IM, int JN>
constexpr int bound_stage_bytes() {
  return 2 * (WM * IM + WN * JN) * 16 * KCH * (int)sizeof(typename BoundTraits<KIND>::T);
}

// Whether a step of KCH radii of both operands splits into whole KiB per wave,
// the double-buffered stages fit the LDS, and (FP32) the fragments and
// accumulators of a wave fit the registers of two waves per SIMD.
template <int KIND, int KCH, int WM, int WN, int IM, int JN>
constexpr bool bound_shape_ok() {
  const int rb = KCH * (int)sizeof(typename BoundTraits<KIND>::T);
  const int nw = WM * WN;
  return (16 * WM * IM * rb) % (1024 * nw) == 0 && (16 * WN * JN * rb) % (1024 * nw) == 0 &&
         2 * bound_stage_bytes<KIND, KCH, WM, WN, IM, JN>() <= 160 * 1024 && (KIND != 0 || IM * JN <= 4);
}

// Block tile: WM x WN waves, each computing IM x JN MFMA blocks of 16 x 16
// (patterns x zones); TP = 16 WM IM patterns by TZ = 16 WN JN zones.  Operand
// rows come from the 64-row tiles of the tile-major layout; rows past the end
// of an operand array are read from its last tile (their results are never
// stored), and a wave whose zones all lie past Zvalid skips its MFMAs.
template <int KIND, int KCH, int WM, int WN, int IM, int JN>
__global__ void __launch_bounds__(64 * WM * WN) bound_kernel(BoundArgs a) {
  typedef typename BoundTraits<KIND>::T T;
  constexpr int NW = WM * WN;
  constexpr int TP = 16 * WM * IM, TZ = 16 * WN * JN;
  constexpr int RB = KCH * (int)sizeof(T);  // bytes per staged row
  static_assert(RB == 64 || RB == 128 || RB == 256, "staged rows of 64, 128 or 256 bytes");
  static_assert(KIND != 0 || KCH == 16 || KCH == 32, "FP32 operands use 16- or 32-radius steps");
  static_assert(TP % 64 == 0 && TZ % 64 == 0, "block tiles are whole layout tiles");
  constexpr int VEC = 16 / (int)sizeof(T);  // elements per 16-byte chunk
  constexpr int ARRX = TP * RB, ARRP = TZ * RB;  // bytes of one operand array per stage
  constexpr int STAGE = 2 * ARRX + 2 * ARRP;
  constexpr int NIX = ARRX / 1024 / NW, NIP = ARRP / 1024 / NW;  // 1 KiB LDS-direct loads per wave per array
  static_assert(NIX * 1024 * NW == ARRX && NIP * 1024 * NW == ARRP, "whole KiB per wave");
  // two stage buffers as distinct LDS objects: the compiler can then see that
  // the direct-to-LDS copies of one step never alias the reads of the other
  __shared__ __align__(16) unsigned char sbuf0[STAGE];
  __shared__ __align__(16) unsigned char sbuf1[STAGE];

  int tp, tz;
  if (a.order == 0) {
    tp = blockIdx.x % a.nP;
    tz = blockIdx.x / a.nP;
  } else {
    const int w = xcd_item(a.per);
    if (w >= a.nP * a.nZ) return;
    tp = w / a.nZ;
    tz = w % a.nZ;
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / WN, wc = wave % WN;
  const int li = lane & 15;
  const int lg = lane >> 4;
  // this wave's MFMAs matter only if some of its zones and patterns exist
  const bool live = tz * TZ + wc * JN * 16 < a.Zvalid && tp * TP + wr * IM * 16 < a.np;

  float U[IM][JN][4];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) U[i][j][r] = 0.0f;

  const size_t slab = (size_t)a.rows * 64 * a.Rp;
  const T* gx[2] = {reinterpret_cast<const T*>(a.xr), reinterpret_cast<const T*>(a.xi)};
  const T* gp[2] = {reinterpret_cast<const T*>(a.pr), reinterpret_cast<const T*>(a.pi)};
  // radii below r0 are zero in every zone's plan: whole steps of them are
  // skipped, and with FP32 operands also the first 16 radii of a step
  const int s_begin = (a.r0 / KCH) * KCH;
  const int steps_per_k = (a.Rp - s_begin) / KCH;
  const int nsteps = a.nlog * steps_per_k;
  const bool skip_h0 = KIND == 0 && KCH == 32 && a.r0 - s_begin >= 16;

  // per-lane part of the LDS-direct copies: lane writes bytes [16 lane, +16) of
  // its wave's KiB, i.e. block row r, physical chunk c; it fetches logical chunk
  // c ^ swizzle(r) of that row from layout tile (first tile + r / 64), clamped
  size_t offx[NIX], offp[NIP];
#pragma unroll
  for (int j = 0; j < NIX; ++j) {
    const int byte = (wave * NIX + j) * 1024 + lane * 16;
    const int row = byte / RB, phys = (byte % RB) / 16;
    const int t64 = min(tp * (TP / 64) + (row >> 6), a.nX64 - 1);
    offx[j] = (size_t)t64 * slab + (size_t)(row & 63) * a.Rp + (size_t)((phys ^ chunk_swizzle<RB>(row)) * VEC);
  }
#pragma unroll
  for (int j = 0; j < NIP; ++j) {
    const int byte = (wave * NIP + j) * 1024 + lane * 16;
    const int row = byte / RB, phys = (byte % RB) / 16;
    const int t64 = min(tz * (TZ / 64) + (row >> 6), a.nP64 - 1);
    offp[j] = (size_t)t64 * slab + (size_t)(row & 63) * a.Rp + (size_t)((phys ^ chunk_swizzle<RB>(row)) * VEC);
  }
  auto issue = [&](int stp, unsigned char* st) {
    const int k = stp / steps_per_k;
    const int row = k < a.Kc ? k : a.hi + (k - a.Kc);
    const size_t kbase = (size_t)row * 64 * a.Rp + s_begin + (size_t)(stp - k * steps_per_k) * KCH;
#pragma unroll
    for (int arr = 0; arr < 2; ++arr)
#pragma unroll
      for (int j = 0; j < NIX; ++j)
        __builtin_amdgcn_global_load_lds((const void*)(gx[arr] + kbase + offx[j]),
                                         (__attribute__((address_space(3))) void*)(st + arr * ARRX + (wave * NIX + j) * 1024),
                                         16, 0, 0);
#pragma unroll
    for (int arr = 0; arr < 2; ++arr)
#pragma unroll
      for (int j = 0; j < NIP; ++j)
        __builtin_amdgcn_global_load_lds(
            (const void*)(gp[arr] + kbase + offp[j]),
            (__attribute__((address_space(3))) void*)(st + 2 * ARRX + arr * ARRP + (wave * NIP + j) * 1024), 16, 0, 0);
  };
  // byte offset of (row, logical chunk) inside one operand array of a stage
  auto at = [](int row, int chunk) { return row * RB + ((chunk ^ chunk_swizzle<RB>(row)) << 4); };

  f32x4 acc[IM][JN][4];
  // MFMAs and, after the last step of a frequency, the epilogue of step stp on stage st
  auto compute = [&](int stp, const unsigned char* st) {
    const unsigned char* sXr = st;
    const unsigned char* sXi = st + ARRX;
    const unsigned char* sPr = st + 2 * ARRX;
    const unsigned char* sPi = st + 2 * ARRX + ARRP;
    // the first step of a frequency starts its accumulators at 0 (compile-time
    // operand); H0 = 1 skips the first half of an FP32 step (zero plan radii).
    // NR: a norm row with FP32 operands runs only the two products its
    // epilogue reads (A + B); C and D keep the last spectrum row's values,
    // which no norm row reads.  The 16-bit kernels keep one body (their
    // registers are full).
    auto mma = [&](auto zc, auto hc, auto nc) {
      constexpr bool Z = decltype(zc)::value;
      constexpr int H0 = decltype(hc)::value;
      constexpr bool NR = decltype(nc)::value && KIND == 0;
      const f32x4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
      if constexpr (KIND == 0) {
        // two halves of 16 radii; lane quarter lg holds radii 16 h + 4 lg .. + 3 (chunk 4 h + lg)
#pragma unroll
        for (int h = H0; h < KCH / 16; ++h) {
          float fxr[IM][4], fxi[IM][4], fpr[JN][4], fpi[JN][4];
#pragma unroll
          for (int i = 0; i < IM; ++i) {
            const int rx = wr * IM * 16 + i * 16 + li;
            const float4 u = *reinterpret_cast<const float4*>(sXr + at(rx, h * 4 + lg));
            const float4 v = *reinterpret_cast<const float4*>(sXi + at(rx, h * 4 + lg));
            fxr[i][0] = u.x; fxr[i][1] = u.y; fxr[i][2] = u.z; fxr[i][3] = u.w;
            fxi[i][0] = v.x; fxi[i][1] = v.y; fxi[i][2] = v.z; fxi[i][3] = v.w;
          }
#pragma unroll
          for (int j = 0; j < JN; ++j) {
            const int rp = wc * JN * 16 + j * 16 + li;
            const float4 u = *reinterpret_cast<const float4*>(sPr + at(rp, h * 4 + lg));
            const float4 v = *reinterpret_cast<const float4*>(sPi + at(rp, h * 4 + lg));
            fpr[j][0] = u.x; fpr[j][1] = u.y; fpr[j][2] = u.z; fpr[j][3] = u.w;
            fpi[j][0] = v.x; fpi[j][1] = v.y; fpi[j][2] = v.z; fpi[j][3] = v.w;
          }
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < IM; ++i)
#pragma unroll
              for (int j = 0; j < JN; ++j) {
                const bool z = Z && h == H0 && t == 0;
                acc[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fxr[i][t], fpr[j][t], z ? zero4 : acc[i][j][0], 0, 0, 0);
                acc[i][j][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fxi[i][t], fpi[j][t], z ? zero4 : acc[i][j][1], 0, 0, 0);
                if constexpr (!NR) {
                  acc[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(fxi[i][t], fpr[j][t], z ? zero4 : acc[i][j][2], 0, 0, 0);
                  acc[i][j][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(fxr[i][t], fpi[j][t], z ? zero4 : acc[i][j][3], 0, 0, 0);
                }
              }
        }
      } else {
        typedef typename std::conditional<KIND == 1, bf16x8, f16x8>::type V8;
#pragma unroll
        for (int sub = 0; sub < KCH / 32; ++sub) {
          V8 fxr[IM], fxi[IM], fpr[JN], fpi[JN];
#pragma unroll
          for (int i = 0; i < IM; ++i) {
            const int rx = wr * IM * 16 + i * 16 + li;
            fxr[i] = *reinterpret_cast<const V8*>(sXr + at(rx, sub * 4 + lg));
            fxi[i] = *reinterpret_cast<const V8*>(sXi + at(rx, sub * 4 + lg));
          }
#pragma unroll
          for (int j = 0; j < JN; ++j) {
            const int rp = wc * JN * 16 + j * 16 + li;
            fpr[j] = *reinterpret_cast<const V8*>(sPr + at(rp, sub * 4 + lg));
            fpi[j] = *reinterpret_cast<const V8*>(sPi + at(rp, sub * 4 + lg));
          }
#pragma unroll
          for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j) {
              const bool z = Z && sub == 0;
              if constexpr (KIND == 1) {
                acc[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fxr[i], fpr[j], z ? zero4 : acc[i][j][0], 0, 0, 0);
                acc[i][j][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fxi[i], fpi[j], z ? zero4 : acc[i][j][1], 0, 0, 0);
                acc[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fxi[i], fpr[j], z ? zero4 : acc[i][j][2], 0, 0, 0);
                acc[i][j][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fxr[i], fpi[j], z ? zero4 : acc[i][j][3], 0, 0, 0);
              } else {
                acc[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fxr[i], fpr[j], z ? zero4 : acc[i][j][0], 0, 0, 0);
                acc[i][j][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fxi[i], fpi[j], z ? zero4 : acc[i][j][1], 0, 0, 0);
                acc[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fxi[i], fpr[j], z ? zero4 : acc[i][j][2], 0, 0, 0);
                acc[i][j][3] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fxr[i], fpi[j], z ? zero4 : acc[i][j][3], 0, 0, 0);
              }
            }
        }
      }
    };
    auto mma_at = [&](auto nc) {
      if (stp % steps_per_k != 0)
        mma(std::false_type{}, std::integral_constant<int, 0>{}, nc);
      else if (skip_h0)
        mma(std::true_type{}, std::integral_constant<int, 1>{}, nc);
      else
        mma(std::true_type{}, std::integral_constant<int, 0>{}, nc);
    };
    if (KIND == 0 && stp / steps_per_k >= a.Kc)
      mma_at(std::true_type{});
    else
      mma_at(std::false_type{});
    const int k = stp / steps_per_k;
    const bool nr = k >= a.Kc;  // a norm row
    if (stp - k * steps_per_k == steps_per_k - 1) {  // last radii of logical frequency k
      if (!nr) {
        const float wk = (k == 0 || 2 * k == a.N) ? 1.0f : 2.0f;
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
          for (int j = 0; j < JN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float A = acc[i][j][0][r], B = acc[i][j][1][r], C = acc[i][j][2][r], D = acc[i][j][3][r];
              // max(|G|^2, |G_mirror|^2) = S + 2 |T|, S = A^2 + B^2 + C^2 + D^2, T = A B - C D
              const float S = fmaf(A, A, fmaf(B, B, fmaf(C, C, D * D)));
              const float Tm = fmaf(A, B, -(C * D));
              // hardware square root (<= 1 ulp): the certificate's relative slack covers it
              U[i][j][r] += wk * __builtin_amdgcn_sqrtf(fmaf(2.0f, fabsf(Tm), S));
            }
      } else {  // block-norm products (the frequency weights are in the pattern's norms)
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
          for (int j = 0; j < JN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) U[i][j][r] += acc[i][j][0][r] + acc[i][j][1][r];
      }
    }
  };
  if (nsteps > 0) issue(0, sbuf0);
  for (int stp = 0; stp < nsteps; stp += 2) {  // two steps per trip, one per stage buffer
    __builtin_amdgcn_s_waitcnt(0);  // this thread's copies of step stp have landed
    __syncthreads();                // ... every thread's, and all reads of step stp - 1 are done
    if (stp + 1 < nsteps) issue(stp + 1, sbuf1);
    if (live) compute(stp, sbuf0);
    if (stp + 1 >= nsteps) break;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (stp + 2 < nsteps) issue(stp + 2, sbuf0);
    if (live) compute(stp + 1, sbuf1);
  }
  if (!live) return;
  const float invN = 1.0f / (float)a.N;
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = tp * TP + wr * IM * 16 + i * 16 + lg * 4 + r;
      if (p >= a.np) continue;
      const float inv = invN / a.scale[p];
#pragma unroll
      for (int j = 0; j < JN; ++j) {
        const int z = tz * TZ + wc * JN * 16 + j * 16 + li;
        if (z < a.Zvalid) a.U[(size_t)p * a.ldU + z] = U[i][j][r] * inv;
      }
    }
}

// ------------------------------------------------------------ 3. exact ----

struct ExactArgs {
  int N, Nk, Rp, Z, nrad;
  int rad[kMaxRadices];
  const float2* tw;
  const int* rev;
  const float *xr, *xi;     // tile-major over the chunk's patterns (FP32)
  const float *pr, *pi;     // zone-major [Z][Nk][Rp] (FP32)
  int xrows;                // rows per 64-pattern tile of the FP32 spectrum (frequencies, then norm rows)
  int* queue;               // kXcds pattern counters of the persistent exact pass (workspace)
  float* U;                 // bound rows (workspace); updated in place when u_lds == 0
  int ldU;
  int u_lds;                // 1: the pattern's bound row is copied to LDS; 0: selected in place in U
  const float* xnorm2;
  const uint32_t* cmask;    // per pattern and radial tile: columns holding a nonzero X
  int ntiles;
  const int* flags;
  const float* M12;
  const int* zone_phase;
  float eps_rel, eps_abs;
  int top_k;
  int per, xblk, xfull;  // pattern order: per < 0 plain, else xcd_item_grouped(xblk, xfull, per)
  int64_t p_begin;
  int np;
  int *zone, *phase, *bin, *mirror, *n_eval;
  float *score, *phi3, *orient;
  float* C;  // correlate mode: C[p][z][2][N] for every zone (no selection)
  int64_t out_p0;           // outputs are indexed by global pattern P - out_p0
  // forced mode: per global pattern P, the correlogram value of zone
  // force_zone[P] at bin force_bin[P], branch force_mirror[P] (no selection)
  const int *force_zone, *force_bin, *force_mirror;
  float* force_score;
};

// The 4-radius groups of pattern p whose columns hold any nonzero X, in
// increasing order (the others contribute exact zeros to every contraction):
// wave 0 reads the column masks in parallel, one group per lane, and compacts
// the active groups in order by ballot.
__device__ void active_groups(const ExactArgs& a, int p, int* groups, int* ng) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    constexpr int GPT = kPolarCols / 4;  // groups per mask word
    const int total = a.ntiles * GPT;
    int n = 0;
    for (int g0 = 0; g0 < total; g0 += 64) {
      const int g = g0 + lane;
      bool act = false;
      if (g < total) {
        const uint32_t m = a.cmask ? a.cmask[(size_t)p * a.ntiles + g / GPT] : 0xFFFFu;
        act = ((m >> (4 * (g % GPT))) & 0xFu) != 0u;
      }
      const unsigned long long bal = __ballot(act);
      if (act) groups[n + __popcll(bal & ((1ull << lane) - 1ull))] = g;
      n += __popcll(bal);
    }
    if (lane == 0) *ng = n;
  }
  __syncthreads();
}

// H for nb zones of local pattern p: H_k = G_k + i G_mirror,k (k <= N/2) and
// H_{N-k} = conj(G_k) + i conj(G_mirror,k), stored in digit-reversed order for
// the in-place inverse FFT: H[rev(n) * nb + b].  Eight consecutive lanes share a
// frequency k and take every eighth active radius group (consecutive groups
// fill whole 128-byte lines); each group of X is loaded once for all nb zones.
template <int NB>
__device__ void contract_exact_nb(const ExactArgs& a, int p, const int* bz, const int* rev, float2* H,
                                  const int* groups, int ng) {
  const size_t xbase = tile_off(p, 0, 0, a.xrows, a.Rp);
  const size_t xk = (size_t)64 * a.Rp;
  const int sub = threadIdx.x & 7;
  for (int base = 0; base < a.Nk; base += (int)(blockDim.x >> 3)) {
    const int k = base + (int)(threadIdx.x >> 3);
    float A[NB], B[NB], C[NB], D[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) A[b] = B[b] = C[b] = D[b] = 0.0f;
    if (k < a.Nk) {
      const float* xr = a.xr + xbase + (size_t)k * xk;
      const float* xi = a.xi + xbase + (size_t)k * xk;
      const float* pr[NB];
      const float* pi[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        pr[b] = a.pr + ((size_t)bz[b] * a.Nk + k) * a.Rp;
        pi[b] = a.pi + ((size_t)bz[b] * a.Nk + k) * a.Rp;
      }
      // every zone of the batch is a compile-time slot: no branch separates
      // the loads of one group, so they are all in flight together.  Batches
      // of up to two zones also overlap two groups' loads; a batch of four
      // (ten 16-byte loads per group) does not: measured on the degraded-peak
      // scan, more loads in flight per lane made the pass slower
      constexpr int kGroupsInFlight = NB == 4 ? 1 : 2;
#pragma unroll kGroupsInFlight
      for (int g = sub; g < ng; g += 8) {
        const int s = groups[g] * 4;
        const float4 vr = *reinterpret_cast<const float4*>(xr + s);
        const float4 vi = *reinterpret_cast<const float4*>(xi + s);
        float4 wr[NB], wi[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          wr[b] = *reinterpret_cast<const float4*>(pr[b] + s);
          wi[b] = *reinterpret_cast<const float4*>(pi[b] + s);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          A[b] += vr.x * wr[b].x + vr.y * wr[b].y + vr.z * wr[b].z + vr.w * wr[b].w;
          B[b] += vi.x * wi[b].x + vi.y * wi[b].y + vi.z * wi[b].z + vi.w * wi[b].w;
          C[b] += vi.x * wr[b].x + vi.y * wr[b].y + vi.z * wr[b].z + vi.w * wr[b].w;
          D[b] += vr.x * wi[b].x + vr.y * wi[b].y + vr.z * wi[b].z + vr.w * wi[b].w;
        }
      }
    }
    // sums over the eight lanes of k by DPP moves: lanes 2i <-> 2i + 1, the lane
    // pairs of a quad, then the mirrored half-row (the other quad, whose lanes
    // all hold its sum): the butterfly's values, bit for bit
    auto sum8 = [](float& v) {
      v += dpp_move<0xB1>(v);
      v += dpp_move<0x4E>(v);
      v += dpp_move<0x141>(v);
    };
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      sum8(A[b]);
      sum8(B[b]);
      sum8(C[b]);
      sum8(D[b]);
      if (k < a.Nk && sub == 0) {
        H[rev[k] * NB + b] = make_float2((A[b] + B[b]) + (C[b] + D[b]), (C[b] - D[b]) + (A[b] - B[b]));
        if (k > 0 && 2 * k < a.N)
          H[rev[a.N - k] * NB + b] = make_float2((A[b] + B[b]) - (C[b] + D[b]), (A[b] - B[b]) - (C[b] - D[b]));
      }
    }
  }
}
// nb zones (1, 2 or 4; a batch of 3 is padded by its caller to 4 with its
// last zone repeated)
__device__ void contract_exact(const ExactArgs& a, int p, const int* bz, int nb, const int* rev, float2* H,
                               const int* groups, int ng) {
  if (nb == 1)
    contract_exact_nb<1>(a, p, bz, rev, H, groups, ng);
  else if (nb == 2)
    contract_exact_nb<2>(a, p, bz, rev, H, groups, ng);
  else
    contract_exact_nb<4>(a, p, bz, rev, H, groups, ng);
}

__device__ void block_argmax(const float* v, int n, float* out_v, int* out_i, float* sv, int* si) {
  float bv = -INFINITY;
  int bi = INT_MAX;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float x = v[i];
    if (x > bv || (x == bv && i < bi)) {
      bv = x;
      bi = i;
    }
  }
  wave_argmax(bv, bi);
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = bv;
    si[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = sv[0];
    int ix = si[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (sv[w] > b || (sv[w] == b && si[w] < ix)) {
        b = sv[w];
        ix = si[w];
      }
    *out_v = b;
    *out_i = ix;
  }
  __syncthreads();
}

__device__ __forceinline__ float parabolic(float cm1, float c0, float cp1) {
  const float den = cm1 - 2.0f * c0 + cp1;
  if (!(den < 0.0f)) return 0.0f;
  return fminf(0.5f, fmaxf(-0.5f, 0.5f * (cm1 - cp1) / den));
}

// Inverse FFT of the batch's sequences (stride nbp in H: 1, 2 or 4, a batch
// of 3 padded to 4 by its caller): with the angular length known at compile
// time, the specialised schedule.
template <int NT>
__device__ __forceinline__ void exact_ifft(float2* H, const float2* tw, const ExactArgs& a, int nbp) {
  if constexpr (NT > 0) {
    if (nbp == 1)
      block_fft_inplace_ct<NT, 1>(H, tw, -1.0f);
    else if (nbp == 2)
      block_fft_inplace_ct<NT, 2>(H, tw, -1.0f);
    else
      block_fft_inplace_ct<NT, 4>(H, tw, -1.0f);
  } else {
    block_fft_inplace(H, tw, a.N, nbp, a.rad, a.nrad, -1.0f);
  }
}
template <int NT>
__device__ __forceinline__ int exact_stride(int nb) {
  return nb == 3 ? 4 : nb;  // the contraction is specialised for 1, 2 and 4 sequences
}

// PERSIST: a persistent grid (a few workgroups per compute unit) in which the
// workgroups of XCD x take the patterns of the x-th eighth of the chunk one by
// one from that XCD's counter in the workspace (zeroed by the polar pass), so
// neighbouring patterns still share an XCD's L2, the FFT tables are loaded
// once per workgroup, and a pattern that evaluates many zones holds up only
// its own workgroup.  Every workgroup leaves once its range is exhausted.
template <int NT, bool PERSIST>
__global__ void __launch_bounds__(kThreads) exact_kernel(ExactArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* H0 = reinterpret_cast<float2*>(smem_raw);
  float2* tw = H0 + kBatch * a.N;
  int* rev = reinterpret_cast<int*>(tw + a.N);
  float* Us = reinterpret_cast<float*>(rev + a.N);  // the bound row in LDS (u_lds), else nothing
  int* groups = reinterpret_cast<int*>(Us + (a.u_lds ? a.Z : 0));  // Rp / 4 entries
  __shared__ int s_ng;
  __shared__ float sv[4];
  __shared__ int si[4];
  __shared__ float s_topv[kMaxTopK], s_tcm[kMaxTopK], s_tcp[kMaxTopK];
  __shared__ int s_topz[kMaxTopK], s_topn[kMaxTopK], s_topm[kMaxTopK];
  __shared__ int s_cnt, s_nb, s_done, s_eval, s_batches;
  __shared__ int s_bz[kBatch];
  __shared__ float s_rv[kBatch], s_rcm[kBatch], s_rcp[kBatch];
  __shared__ int s_rn[kBatch], s_rm[kBatch];
  __shared__ float s_bv;
  __shared__ int s_bi;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const float invN = 1.0f / (float)a.N;
  for (int i = tid; i < a.N; i += kThreads) {
    tw[i] = a.tw[i];
    rev[i] = a.rev[i];
  }

  if (a.C) {  // full correlogram of zones blockIdx.y * kBatch ..
    const int p = blockIdx.x;
    active_groups(a, p, groups, &s_ng);
    int bz[kBatch];
    const int zb = blockIdx.y * kBatch;
    const int nb = min(kBatch, a.Z - zb);
    const int nbp = exact_stride<NT>(nb);
    for (int b = 0; b < kBatch; ++b) bz[b] = zb + min(b, nb - 1);
    contract_exact(a, p, bz, nbp, rev, H0, groups, s_ng);
    __syncthreads();
    exact_ifft<NT>(H0, tw, a, nbp);
    const float2* Fr = H0;
    for (int it = tid; it < nb * a.N; it += kThreads) {
      const int b = it / a.N, n = it % a.N;
      const float2 v = Fr[n * nbp + b];
      float* out = a.C + (((size_t)p * a.Z + zb + b) * 2) * a.N;
      out[n] = v.x * invN;
      out[a.N + n] = v.y * invN;
    }
    return;
  }

  if (a.force_zone) {  // one given (zone, bin, branch) per pattern
    const int p = a.per < 0 ? (int)blockIdx.x : xcd_item_grouped(a.xblk, a.xfull, a.per);
    if (p >= a.np) return;
    const int64_t P = a.p_begin + p;
    const int z = a.force_zone[P - a.out_p0];
    if (z < 0 || z >= a.Z || a.flags[p] != 0) {
      if (tid == 0) a.force_score[P - a.out_p0] = 0.0f;
      return;
    }
    active_groups(a, p, groups, &s_ng);
    int bz[kBatch];
    for (int b = 0; b < kBatch; ++b) bz[b] = z;
    contract_exact(a, p, bz, 1, rev, H0, groups, s_ng);
    __syncthreads();
    exact_ifft<NT>(H0, tw, a, 1);
    if (tid == 0) {
      const int n = min(max(a.force_bin[P - a.out_p0], 0), a.N - 1);
      const float2 v = H0[n];
      a.force_score[P - a.out_p0] = (a.force_mirror[P - a.out_p0] ? v.y : v.x) * invN;
    }
    return;
  }

  auto one = [&](const int p) {
  const int64_t P = a.p_begin + p;
  const int fl = a.flags[p];
  if (fl != 0) {
    for (int t = tid; t < a.top_k; t += kThreads) {
      const size_t o = (size_t)(P - a.out_p0) * a.top_k + t;
      a.zone[o] = -1;
      if (a.phase) a.phase[o] = -1;
      if (a.bin) a.bin[o] = 0;
      if (a.mirror) a.mirror[o] = 0;
      a.score[o] = 0.0f;
      if (a.phi3) a.phi3[o] = 0.0f;
      if (a.orient)
        for (int i = 0; i < 9; ++i) a.orient[o * 9 + i] = 0.0f;
    }
    if (a.n_eval && tid == 0) a.n_eval[P - a.out_p0] = 0;
    return;
  }
  const float margin_abs = a.eps_abs * sqrtf(a.xnorm2[p]);
  // the bound row: copied to LDS when it fits, else selected in place in the
  // workspace (thread 0 marks taken zones; the barriers of block_argmax order
  // those global writes for the whole workgroup)
  float* Ul = a.U + (size_t)p * a.ldU;
  if (a.u_lds) {
    for (int z = tid; z < a.Z; z += kThreads) Us[z] = Ul[z];
    Ul = Us;
  }
  active_groups(a, p, groups, &s_ng);
  if (tid == 0) {
    s_cnt = 0;
    s_done = 0;
    s_eval = 0;
    s_batches = 0;
  }
  __syncthreads();

  while (true) {
    // ---- select the next batch in decreasing bound order; the first batch
    // holds top_k + 1 zones, later ones kBatch
    const int want = s_batches == 0 ? min(kBatch, a.top_k + 1) : kBatch;
    if (tid == 0) s_nb = 0;
    __syncthreads();
    for (int b = 0; b < want; ++b) {
      block_argmax(Ul, a.Z, &s_bv, &s_bi, sv, si);
      if (tid == 0) {
        const float v = s_bv;
        const float kth = s_cnt >= a.top_k ? s_topv[a.top_k - 1] : -INFINITY;
        const bool stop = !(v > 0.0f) || (v * (1.0f + a.eps_rel) + margin_abs < kth);
        if (stop) {
          if (s_nb == 0) s_done = 1;
        } else {
          s_bz[s_nb] = s_bi;
          Ul[s_bi] = -1.0f;
          s_nb = s_nb + 1;
        }
        s_bv = stop ? -1.0f : 0.0f;  // broadcast: stop selecting
      }
      __syncthreads();
      if (s_bv < 0.0f) break;
    }
    const int nb = s_nb;
    if (s_done || nb == 0) break;
    // ---- exact correlograms of the batch
    int bz[kBatch];
    for (int b = 0; b < kBatch; ++b) bz[b] = s_bz[min(b, nb - 1)];
    const int nbp = exact_stride<NT>(nb);  // a padded batch repeats its last zone
    contract_exact(a, p, bz, nbp, rev, H0, groups, s_ng);
    __syncthreads();
    exact_ifft<NT>(H0, tw, a, nbp);
    const float2* Fr = H0;
    for (int b = wave; b < nb; b += kThreads / 64) {
      float bv = -INFINITY;
      int bi = INT_MAX;
      for (int t = lane; t < 2 * a.N; t += 64) {
        const float2 v = Fr[(t >> 1) * nbp + b];
        const float x = ((t & 1) ? v.y : v.x) * invN;
        if (x > bv || (x == bv && t < bi)) {
          bv = x;
          bi = t;
        }
      }
      wave_argmax(bv, bi);
      if (lane == 0) {
        const int n = bi >> 1, m = bi & 1;
        const float2 vm = Fr[(n == 0 ? a.N - 1 : n - 1) * nbp + b];
        const float2 vp = Fr[(n == a.N - 1 ? 0 : n + 1) * nbp + b];
        s_rv[b] = bv;
        s_rn[b] = n;
        s_rm[b] = m;
        s_rcm[b] = (m ? vm.y : vm.x) * invN;
        s_rcp[b] = (m ? vp.y : vp.x) * invN;
      }
    }
    __syncthreads();
    if (tid == 0) {
      s_eval += nb;
      s_batches += 1;
      for (int b = 0; b < nb; ++b) {
        const float v = s_rv[b];
        const int z = s_bz[b];
        if (!(v > 0.0f)) continue;
        int pos = s_cnt;  // insertion point: after all entries that beat (v, z)
        while (pos > 0 && (s_topv[pos - 1] < v || (s_topv[pos - 1] == v && s_topz[pos - 1] > z))) --pos;
        if (pos >= a.top_k) continue;
        const int last = min(s_cnt, a.top_k - 1);
        for (int q = last; q > pos; --q) {
          s_topv[q] = s_topv[q - 1];
          s_topz[q] = s_topz[q - 1];
          s_topn[q] = s_topn[q - 1];
          s_topm[q] = s_topm[q - 1];
          s_tcm[q] = s_tcm[q - 1];
          s_tcp[q] = s_tcp[q - 1];
        }
        s_topv[pos] = v;
        s_topz[pos] = z;
        s_topn[pos] = s_rn[b];
        s_topm[pos] = s_rm[b];
        s_tcm[pos] = s_rcm[b];
        s_tcp[pos] = s_rcp[b];
        s_cnt = min(s_cnt + 1, a.top_k);
      }
    }
    __syncthreads();
  }
  // ---- outputs
  const float two_pi = 6.283185307179586f;
  for (int t = tid; t < a.top_k; t += kThreads) {
    const size_t o = (size_t)(P - a.out_p0) * a.top_k + t;
    if (t < s_cnt) {
      const int z = s_topz[t], n = s_topn[t], m = s_topm[t];
      const float off = parabolic(s_tcm[t], s_topv[t], s_tcp[t]);
      const float ph3 = -((float)n + off) * two_pi / (float)a.N;
      a.zone[o] = z;
      if (a.phase) a.phase[o] = a.zone_phase[z];
      if (a.bin) a.bin[o] = n;
      if (a.mirror) a.mirror[o] = m;
      a.score[o] = s_topv[t];
      if (a.phi3) a.phi3[o] = ph3;
      if (a.orient) {
        float cs, sn;
        sincosf(ph3, &sn, &cs);
        const float* M = a.M12 + (size_t)z * 9;
        for (int i = 0; i < 3; ++i) {
          float c0 = M[3 * i] * cs + M[3 * i + 1] * sn;
          const float c1 = -M[3 * i] * sn + M[3 * i + 1] * cs;
          float c2 = M[3 * i + 2];
          if (m) {
            c0 = -c0;
            c2 = -c2;
          }
          a.orient[o * 9 + 3 * i] = c0;
          a.orient[o * 9 + 3 * i + 1] = c1;
          a.orient[o * 9 + 3 * i + 2] = c2;
        }
      }
    } else {
      a.zone[o] = -1;
      if (a.phase) a.phase[o] = -1;
      if (a.bin) a.bin[o] = 0;
      if (a.mirror) a.mirror[o] = 0;
      a.score[o] = 0.0f;
      if (a.phi3) a.phi3[o] = 0.0f;
      if (a.orient)
        for (int i = 0; i < 9; ++i) a.orient[o * 9 + i] = 0.0f;
    }
  }
  if (a.n_eval && tid == 0) a.n_eval[P - a.out_p0] = s_eval;
  };  // one pattern

  if constexpr (!PERSIST) {
    const int p = a.per < 0 ? (int)blockIdx.x : xcd_item_grouped(a.xblk, a.xfull, a.per);
    if (p >= a.np) return;
    one(p);
  } else {
    __shared__ int s_next;
    const int x = (int)(blockIdx.x % kXcds);
    const int lo = x * a.per, hi = min(a.np, lo + a.per);
    while (true) {
      __syncthreads();  // the previous pattern is done with every LDS array and s_next
      if (tid == 0) s_next = lo + atomicAdd(a.queue + x, 1);
      __syncthreads();
      const int p = s_next;
      if (p >= hi) break;
      one(p);
    }
  }
}

// --------------------------------------------- 4. overlapping patterns ----
//
// Matching of Overlapping Diffraction Patterns: after each round's match, the
// forward kinematical pattern of the matched orientation (Methods >
// Calculation of Kinematical Diffraction Patterns: a reflection g sits at
// (x, y) of m^T g with intensity |F_g|^2 exp(-s_g^2 / 2 sigma^2), kept above
// rel_cut of the phase's largest |F|^2) is laid over the experimental peaks:
// a peak closer than the deletion radius r_del to a simulated peak is removed
// (intensity 0), one between r_del and the correlation kernel's reach r_k has
// its intensity scaled by (d - r_del) / (r_k - r_del), d the distance to the
// nearest simulated peak, and the next round matches the edited peaks.

struct EditArgs {
  const int64_t* offsets;
  const float *qx, *qy;
  int64_t total_peaks;
  const float* I_src;       // intensities before this round's edit
  float* I_dst;             // after it (may alias I_src)
  int64_t p_begin;
  int np;
  // this round's match of the chunk (local pattern index) and the score of the
  // same (zone, bin, branch) on the original peaks
  const int *zone, *phase, *bin, *mirror;
  const float *score_orig, *phi3, *orient;
  const int* flags;
  // reflections
  const float4* refl;
  const float* F2;
  const int* refl_off;
  float k0, sigma_e, rel_cut, r_del, r_k, min_score;
  // outputs for round `round` of n_orient (global pattern index)
  int round, n_orient;
  int *o_zone, *o_phase, *o_bin, *o_mirror;
  float *o_score, *o_phi3, *o_orient;
};

constexpr int kSimBatch = 256;  // reflections examined per pass (one per thread)

__device__ __forceinline__ float excitation_error_f(float x, float y, float z, float k0) {
  // s_g of a sample-frame reciprocal vector for a beam along +z (Eq. excitation error)
  return -(2.0f * k0 * z + (x * x + y * y + z * z)) / (2.0f * sqrtf(x * x + y * y + (k0 + z) * (k0 + z)));
}

__global__ void __launch_bounds__(kThreads) multi_edit_kernel(EditArgs a) {
  __shared__ float sx[kSimBatch], sy[kSimBatch];
  __shared__ int s_ns;
  __shared__ float s_red[kThreads / 64];
  const int tid = threadIdx.x;
  const int p = blockIdx.x;
  if (p >= a.np) return;
  const int64_t P = a.p_begin + p;
  int64_t m0 = a.offsets[P], m1 = a.offsets[P + 1];
  if (m0 < 0 || m1 < m0 || m1 > a.total_peaks) m0 = m1 = 0;  // malformed row: nothing to edit
  const int z = a.zone[p];
  const bool valid = z >= 0 && a.flags[p] == 0 && a.score_orig[p] > 0.0f && a.score_orig[p] >= a.min_score;
  // this round's outputs
  if (tid == 0) {
    const size_t o = (size_t)P * a.n_orient + a.round;
    a.o_zone[o] = valid ? z : -1;
    if (a.o_phase) a.o_phase[o] = valid ? a.phase[p] : -1;
    if (a.o_bin) a.o_bin[o] = valid ? a.bin[p] : 0;
    if (a.o_mirror) a.o_mirror[o] = valid ? a.mirror[p] : 0;
    a.o_score[o] = valid ? a.score_orig[p] : 0.0f;
    if (a.o_phi3) a.o_phi3[o] = valid ? a.phi3[p] : 0.0f;
    if (a.o_orient)
      for (int i = 0; i < 9; ++i) a.o_orient[o * 9 + i] = valid ? a.orient[(size_t)p * 9 + i] : 0.0f;
  }
  if (!valid) {  // no further orientation: every later round finds nothing
    for (int64_t m = m0 + tid; m < m1; m += kThreads) a.I_dst[m] = 0.0f;
    return;
  }
  float M[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) M[i] = a.orient[(size_t)p * 9 + i];
  const int ph = a.phase[p];
  const int g0 = a.refl_off[ph], g1 = a.refl_off[ph + 1];
  // the phase's largest |F|^2
  float fm = 0.0f;
  for (int g = g0 + tid; g < g1; g += kThreads) fm = fmaxf(fm, a.F2[g]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) fm = fmaxf(fm, __shfl_xor(fm, off, 64));
  if ((tid & 63) == 0) s_red[tid >> 6] = fm;
  __syncthreads();
  fm = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
  const float cut = a.rel_cut * fm;
  const float inv2s2 = 1.0f / (2.0f * a.sigma_e * a.sigma_e);
  for (int64_t mb = m0; mb < m1; mb += kThreads) {
    const int64_t m = mb + tid;
    const bool has = m < m1;
    const float px = has ? a.qx[m] : 0.0f, py = has ? a.qy[m] : 0.0f;
    float d2 = INFINITY;  // squared distance to the nearest simulated peak
    for (int gb = g0; gb < g1; gb += kSimBatch) {
      if (tid == 0) s_ns = 0;
      __syncthreads();
      const int g = gb + tid;
      if (tid < kSimBatch && g < g1) {
        const float4 r = a.refl[g];
        // sample frame: (x, y, z) = m^T g
        const float x = M[0] * r.x + M[3] * r.y + M[6] * r.z;
        const float y = M[1] * r.x + M[4] * r.y + M[7] * r.z;
        const float zz = M[2] * r.x + M[5] * r.y + M[8] * r.z;
        const float sg = excitation_error_f(x, y, zz, a.k0);
        if (a.F2[g] * expf(-sg * sg * inv2s2) > cut) {
          const int slot = atomicAdd(&s_ns, 1);  // any order: only the minimum distance is used
          sx[slot] = x;
          sy[slot] = y;
        }
      }
      __syncthreads();
      const int ns = s_ns;
      if (has)
        for (int t = 0; t < ns; ++t) {
          const float dx = px - sx[t], dy = py - sy[t];
          d2 = fminf(d2, dx * dx + dy * dy);
        }
      __syncthreads();
    }
    if (has) {
      const float d = sqrtf(d2);
      float f = 1.0f;
      if (d < a.r_del) f = 0.0f;
      else if (d < a.r_k) f = (d - a.r_del) / (a.r_k - a.r_del);
      a.I_dst[m] = a.I_src[m] * f;
    }
  }
}

// ------------------------------------------------------------- tuning ----

struct Tuning {
  int bound_order = 1;    // 0: pattern tiles fastest, 1: XCD-grouped zone tiles fastest
  int bound_kch16 = 64;   // radii per LDS step of the 16-bit contraction (32, 64 or 128)
  int exact_xcd = 1;      // exact pass: XCD-grouped pattern order
  int polar_xcd = 0;      // polar pass: consecutive patterns grouped on one XCD (1) or pattern index fastest
  int bound_tile = 2;     // contraction block tile: 0 = 64 x 64, 1 = 128 x 128, 2 = by problem size
  int skip_zero_radii = 1;  // contraction: skip the leading radii where the plan is zero in every zone
  int bound_kch32 = 16;   // radii per LDS step of the FP32 contraction (16 or 32)
  int polar_cols = 32;    // radial columns per pass of the polar kernel (16 or 32)
  int exact_u_lds_max = 16384;  // largest zone count whose bound row the exact pass copies to LDS
  int exact_persist = 0;         // exact pass: persistent workgroups on XCD-local work queues (1) or one per pattern
  int exact_xcd_block = 1024;    // exact pass, XCD-grouped order: patterns per run (0 = one range per XCD)
  PlanDev::BoundShape tuned[3];  // contraction shape per operand precision found by acom_autotune
};
// Launch-shape settings of the calling host thread: plans stay immutable after
// acom_build_plan, and calls made from different threads (on different
// streams) never share mutable library state.
thread_local Tuning g_tune;

// ---------------------------------------------------------- profiling ----

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> ev;   // 2 per record
  std::vector<int> kind;
  int used = 0;
};
thread_local Profiler g_prof;  // records the calling thread's launches only

struct ProfScope {
  int slot = -1;
  hipStream_t s;
  ProfScope(int kind, hipStream_t st) : s(st) {
    if (!g_prof.on || g_prof.used >= (int)g_prof.kind.size()) return;
    slot = g_prof.used++;
    g_prof.kind[slot] = kind;
    (void)hipEventRecord(g_prof.ev[2 * slot], s);
  }
  ~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], s);
  }
};

struct WsLayout {
  size_t xr = 0, xi = 0, lr = 0, li = 0, scale = 0, xn2 = 0, cmask = 0, flags = 0, U = 0, queue = 0, total = 0;
  int Pc = 0, ntiles = 0;
  bool lowp = false;
};

WsLayout layout(const PlanDev& d, bool lowp, int Pc) {
  WsLayout L;
  L.Pc = Pc;
  L.lowp = lowp;
  L.ntiles = d.Rp / kPolarCols;
  const size_t nx = (size_t)d.rows32 * Pc * d.Rp, nx16 = (size_t)d.rows16 * Pc * d.Rp;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.xr = take(nx * 4);
  L.xi = take(nx * 4);
  if (lowp) {
    L.lr = take(nx16 * 2);
    L.li = take(nx16 * 2);
  }
  L.scale = take((size_t)Pc * 4);
  L.xn2 = take((size_t)Pc * 4);
  L.cmask = take((size_t)Pc * L.ntiles * 4);
  L.flags = take((size_t)Pc * 4);
  L.U = take((size_t)Pc * d.Zp * 4);
  L.queue = take(kXcds * 4);
  L.total = o;
  return L;
}

template <int NC>
size_t polar_lds(const PlanDev& d) {
  return (size_t)(d.N * (NC / 2) + d.N) * sizeof(float2) + (size_t)d.N * 4 + polar_peak_cache<NC>() * (2 + 4 + 4 + 4 + 4 + 1) +
         (size_t)d.Rp * 4 + (size_t)(d.Rp / kPolarCols) * (kThreads / 64) * 4;
}
size_t exact_lds(const PlanDev& d, int u_lds) {
  return (size_t)(kBatch * d.N + d.N) * sizeof(float2) + (size_t)d.N * 4 + (u_lds ? (size_t)d.Z * 4 : 0) + (size_t)d.Rp;
}

// Dynamic-LDS limit of a kernel: raised (never lowered) under a lock, so that a
// launch on another thread that relies on a larger limit set earlier still fits.
template <class K>
acom_status_t ensure_lds(K kernel, size_t bytes) {
  if (bytes > 160 * 1024) return fail(ACOM_E_UNSUPPORTED, "plan too large for the LDS budget of one workgroup");
  static std::mutex mu;
  static std::map<const void*, size_t> set_to;
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = set_to[(const void*)kernel];
  if (bytes <= cur) return ACOM_OK;
  ACOM_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  cur = bytes;
  return ACOM_OK;
}

acom_status_t check_peaks(const acom_peaks_t* pk) {
  if (!pk) return fail(ACOM_E_INVALID, "peaks is null");
  if (pk->n_patterns < 0 || pk->total_peaks < 0) return fail(ACOM_E_INVALID, "negative pattern or peak count");
  if (pk->n_patterns > 0 && !pk->offsets) return fail(ACOM_E_INVALID, "offsets is null");
  if (pk->total_peaks > 0 && (!pk->qx || !pk->qy || !pk->intensity)) return fail(ACOM_E_INVALID, "peak arrays are null");
  if (pk->total_peaks > INT_MAX) return fail(ACOM_E_UNSUPPORTED, "more than 2^31-1 peaks in one call");
  return ACOM_OK;
}

PolarArgs polar_args(const PlanDev& d, const acom_peaks_t* pk, int64_t p_begin, int np, int lowp) {
  PolarArgs a;
  a.N = d.N;
  a.R = d.R;
  a.Rp = d.Rp;
  a.Nk = d.Nk;
  a.nrad = d.rad.n;
  for (int i = 0; i < kMaxRadices; ++i) a.rad[i] = d.rad.r[i];
  a.qs = d.d_qs;
  a.tw = d.d_tw;
  a.rev = d.d_rev;
  a.delta = (float)d.delta;
  a.sigma = (float)d.gauss_sigma;
  a.rk = d.kernel == ACOM_KERNEL_CONE ? (float)d.delta : (float)(3.0 * d.gauss_sigma);
  a.gamma = (float)d.gamma;
  a.omega = (float)d.omega;
  a.kernel = d.kernel;
  a.offsets = pk->offsets;
  a.qx = pk->qx;
  a.qy = pk->qy;
  a.I = pk->intensity;
  a.total_peaks = pk->total_peaks;
  a.p_begin = p_begin;
  a.np = np;
  a.lowp = lowp;
  a.Ximg = nullptr;
  a.do_fft = 1;
  a.cmask = nullptr;
  a.ws_layout = 0;
  a.ld_tile16 = 0;
  a.queue = nullptr;
  const int c = lowp ? 1 : 0;
  a.Kc16 = d.Kc[1];
  a.Kn = d.Kc[c];
  a.inv2sp = d.Sp > 0 ? 1.0f / (float)(2 * d.Sp) : 0.0f;
  a.inc_j = a.inc_e = 0;
  a.bb_log2 = __builtin_ctz(d.bb);
  a.bb = d.bb;
  a.nb = d.nb;
  a.Sp = d.Sp;
  a.r0 = d.r0;
  a.npseudo = d.npseudo[c];
  a.L = d.L[c];
  return a;
}

void set_ws(PolarArgs& a, const WsLayout& L, unsigned char* ws, const PlanDev& d) {
  a.xr = reinterpret_cast<float*>(ws + L.xr);
  a.xi = reinterpret_cast<float*>(ws + L.xi);
  a.ld_tile = (size_t)d.rows32 * 64 * d.Rp;   // tile-major, as tile_off with rows32 rows per tile
  a.ld_tile16 = (size_t)d.rows16 * 64 * d.Rp;
  a.ldk = (size_t)64 * d.Rp;
  a.ldp = d.Rp;
  a.out_cols = d.Rp;
  a.ws_layout = 1;
  a.lr = L.lowp ? reinterpret_cast<uint16_t*>(ws + L.lr) : nullptr;
  a.li = L.lowp ? reinterpret_cast<uint16_t*>(ws + L.li) : nullptr;
  a.scale = reinterpret_cast<float*>(ws + L.scale);
  a.xnorm2 = reinterpret_cast<float*>(ws + L.xn2);
  a.cmask = reinterpret_cast<uint32_t*>(ws + L.cmask);
  a.flags = reinterpret_cast<int*>(ws + L.flags);
  a.queue = reinterpret_cast<int*>(ws + L.queue);
}

template <int NT, int NC>
acom_status_t launch_polar_nc(const PlanDev& d, const PolarArgs& a, hipStream_t s) {
  // one instantiation per kernel shape: the splat's cell loops hold no branch on it
  const bool cone = a.kernel == ACOM_KERNEL_CONE;
  auto kern = cone ? polar_kernel<NT, NC, ACOM_KERNEL_CONE> : polar_kernel<NT, NC, ACOM_KERNEL_GAUSS>;
  acom_status_t st = ensure_lds(kern, polar_lds<NC>(d));
  if (st != ACOM_OK) return st;
  PolarArgs b = a;
  b.ntiles = d.Rp / kPolarCols;
  b.per = 0;
  if (d.Sp > 0) {  // advance of a norm entry per unpack step of kThreads / (NC / 2) frequencies
    const int adv = kThreads / (NC / 2) * d.nb;
    b.inc_j = adv / (2 * d.Sp);
    b.inc_e = adv % (2 * d.Sp);
  }
  const int nblocks = g_tune.polar_xcd ? xcd_blocks(b.np, &b.per) : b.np;
  ProfScope prof(0, s);
  kern<<<dim3(nblocks), kThreads, polar_lds<NC>(d), s>>>(b);
  ACOM_HIP(hipGetLastError());
  return ACOM_OK;
}
template <int NT>
acom_status_t launch_polar_n(const PlanDev& d, const PolarArgs& a, hipStream_t s) {
  // 32 columns per pass when Rp allows it (Rp is a multiple of 32) and the tuning asks
  if (g_tune.polar_cols == 32 && d.Rp % 32 == 0) return launch_polar_nc<NT, 32>(d, a, s);
  return launch_polar_nc<NT, 16>(d, a, s);
}

template <int NT>
acom_status_t launch_exact_n(const PlanDev& d, const ExactArgs& e, dim3 grid, hipStream_t s, bool persist) {
  const size_t lds = exact_lds(d, e.u_lds);
  if (!persist) {
    acom_status_t st = ensure_lds(exact_kernel<NT, false>, lds);
    if (st != ACOM_OK) return st;
    exact_kernel<NT, false><<<grid, kThreads, lds, s>>>(e);
    ACOM_HIP(hipGetLastError());
    return ACOM_OK;
  }
  // persistent: the workgroups that fit the device at once, in XCD-local ranges
  acom_status_t st = ensure_lds(exact_kernel<NT, true>, lds);
  if (st != ACOM_OK) return st;
  int dev = 0, cus = 0, per_cu = 0;
  ACOM_HIP(hipGetDevice(&dev));
  ACOM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  ACOM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, exact_kernel<NT, true>, kThreads, lds));
  ExactArgs p = e;
  p.per = (p.np + kXcds - 1) / kXcds;
  p.xblk = p.xfull = 0;
  const int nblk = std::max(kXcds, (std::max(1, cus * std::max(1, per_cu)) / kXcds) * kXcds);
  exact_kernel<NT, true><<<dim3(nblk), kThreads, lds, s>>>(p);
  ACOM_HIP(hipGetLastError());
  return ACOM_OK;
}
acom_status_t launch_exact(const PlanDev& d, const ExactArgs& e, dim3 grid, hipStream_t s, bool persist = false) {
  switch (d.N) {  // the same compile-time FFT lengths as the polar pass
    case 90: return launch_exact_n<90>(d, e, grid, s, persist);
    case 120: return launch_exact_n<120>(d, e, grid, s, persist);
    case 180: return launch_exact_n<180>(d, e, grid, s, persist);
    case 360: return launch_exact_n<360>(d, e, grid, s, persist);
    case 720: return launch_exact_n<720>(d, e, grid, s, persist);
    default: return launch_exact_n<0>(d, e, grid, s, persist);
  }
}

acom_status_t launch_polar(const PlanDev& d, const PolarArgs& a, hipStream_t s) {
  switch (d.N) {  // FFT lengths with a compile-time schedule; any other length runs the generic one
    case 90: return launch_polar_n<90>(d, a, s);
    case 120: return launch_polar_n<120>(d, a, s);
    case 180: return launch_polar_n<180>(d, a, s);
    case 360: return launch_polar_n<360>(d, a, s);
    case 720: return launch_polar_n<720>(d, a, s);
    default: return launch_polar_n<0>(d, a, s);
  }
}

template <int WM, int WN, int IM, int JN>
acom_status_t launch_bound_t(const PlanDev& d, int precision, BoundArgs b, int kch_setting, hipStream_t s) {
  constexpr int TP = 16 * WM * IM, TZ = 16 * WN * JN, NT = 64 * WM * WN;
  b.nP = (b.np + TP - 1) / TP;
  b.nZ = (b.Zvalid + TZ - 1) / TZ;
  const int nblocks = b.order == 0 ? b.nP * b.nZ : xcd_blocks(b.nP * b.nZ, &b.per);
  if (b.order == 0) b.per = 0;
  // 16-bit operands: the largest of 128, 64, 32 not above the setting dividing Rp
  // (at most 64 for the large tiles, whose two 128-radius stages would exceed the LDS)
  int kch = (TP + TZ > 128) ? std::min(kch_setting, 64) : kch_setting;
  while (d.Rp % kch) kch /= 2;
  if (TP + TZ > 128 && kch == 32 && !bound_shape_ok<1, 32, WM, WN, IM, JN>()) kch = 64;
  auto launch = [&](auto kern, size_t lds) -> acom_status_t {  // lds: static, checked against the CU's 160 KiB
    if (lds > 160 * 1024) return fail(ACOM_E_UNSUPPORTED, "contraction stages exceed the LDS");
    ProfScope prof(1, s);
    kern<<<dim3(nblocks), NT, 0, s>>>(b);
    return ACOM_OK;
  };
  acom_status_t st = fail(ACOM_E_UNSUPPORTED, "no contraction kernel for this tile and step");
  if (precision == ACOM_FP32) {
    if (kch_setting == 16) {  // FP32 with 16-radius steps
      if constexpr (bound_shape_ok<0, 16, WM, WN, IM, JN>())
        st = launch(bound_kernel<0, 16, WM, WN, IM, JN>, 2 * bound_stage_bytes<0, 16, WM, WN, IM, JN>());
    } else if constexpr (bound_shape_ok<0, 32, WM, WN, IM, JN>()) {
      st = launch(bound_kernel<0, 32, WM, WN, IM, JN>, 2 * bound_stage_bytes<0, 32, WM, WN, IM, JN>());
    }
  } else if (kch == 128) {
    if constexpr (bound_shape_ok<1, 128, WM, WN, IM, JN>())
      st = launch(precision == ACOM_BF16 ? bound_kernel<1, 128, WM, WN, IM, JN> : bound_kernel<2, 128, WM, WN, IM, JN>,
                  2 * bound_stage_bytes<1, 128, WM, WN, IM, JN>());
  } else if (kch == 64) {
    if constexpr (bound_shape_ok<1, 64, WM, WN, IM, JN>())
      st = launch(precision == ACOM_BF16 ? bound_kernel<1, 64, WM, WN, IM, JN> : bound_kernel<2, 64, WM, WN, IM, JN>,
                  2 * bound_stage_bytes<1, 64, WM, WN, IM, JN>());
  } else {
    if constexpr (bound_shape_ok<1, 32, WM, WN, IM, JN>())
      st = launch(precision == ACOM_BF16 ? bound_kernel<1, 32, WM, WN, IM, JN> : bound_kernel<2, 32, WM, WN, IM, JN>,
                  2 * bound_stage_bytes<1, 32, WM, WN, IM, JN>());
  }
  if (st != ACOM_OK) return st;
  ACOM_HIP(hipGetLastError());
  return ACOM_OK;
}

acom_status_t launch_bound(const PlanDev& d, int precision, const WsLayout& L, unsigned char* ws, int np,
                           float* U, int ldU, int Zvalid, hipStream_t s) {
  BoundArgs b;
  const PlanDev::BoundShape* t = g_tune.tuned[precision].set ? &g_tune.tuned[precision] : nullptr;
  b.Nk = d.Nk;
  b.Rp = d.Rp;
  b.N = d.N;
  const int c = precision == ACOM_FP32 ? 0 : 1;
  b.Kc = d.Kc[c];
  b.nlog = d.Kc[c] + d.npseudo[c];
  b.hi = precision == ACOM_FP32 ? d.Nk : d.Kc[1];
  b.rows = precision == ACOM_FP32 ? d.rows32 : d.rows16;
  b.order = t ? t->order : g_tune.bound_order;
  b.nX64 = (np + 63) / 64;
  b.nP64 = d.Zp / 64;
  b.r0 = g_tune.skip_zero_radii ? d.r0 : 0;
  b.scale = reinterpret_cast<const float*>(ws + L.scale);
  b.U = U;
  b.ldU = ldU;
  b.np = np;
  b.Zvalid = Zvalid;
  if (precision == ACOM_FP32) {
    b.xr = ws + L.xr;
    b.xi = ws + L.xi;
    b.pr = d.d_PR;
    b.pi = d.d_PI;
  } else {
    b.xr = ws + L.lr;
    b.xi = ws + L.li;
    b.pr = d.d_PR16[precision];
    b.pi = d.d_PI16[precision];
  }
  // Larger block tiles cut the operand traffic per flop (128 x 128 halves it);
  // they need enough tiles to fill the chip.  FP32 keeps 32 x 32 per wave (a
  // 64 x 32 wave tile of FP32 fragments would not fit the registers of two
  // waves per SIMD), so its large tile is 128 x 64 with eight waves.
  const int large = ((np + 127) / 128) * ((Zvalid + 127) / 128);
  // (measured: the FP32 contraction, bound by the MFMA rate, runs faster with the
  // 64 x 64 tile and two workgroups per compute unit; the 16-bit ones, bound by
  // operand traffic, with 128 x 128)
  // A shape chosen by acom_autotune for this plan and precision takes precedence.
  const int tile = t ? t->tile : g_tune.bound_tile;
  const int kch = t ? t->kch : (precision == ACOM_FP32 ? g_tune.bound_kch32 : g_tune.bound_kch16);
  const bool use_large = tile == 1 || (tile == 2 && precision != ACOM_FP32 && large >= 2 * 256);
  if (use_large && precision == ACOM_FP32) return launch_bound_t<4, 2, 2, 2>(d, precision, b, kch, s);
  if (use_large) return launch_bound_t<2, 4, 4, 2>(d, precision, b, kch, s);
  return launch_bound_t<2, 2, 2, 2>(d, precision, b, kch, s);
}

ExactArgs exact_args(const PlanDev& d, const WsLayout& L, unsigned char* ws, int64_t p_begin, int np) {
  ExactArgs e;
  e.N = d.N;
  e.Nk = d.Nk;
  e.Rp = d.Rp;
  e.Z = d.Z;
  e.nrad = d.rad.n;
  for (int i = 0; i < kMaxRadices; ++i) e.rad[i] = d.rad.r[i];
  e.tw = d.d_tw;
  e.rev = d.d_rev;
  e.xr = reinterpret_cast<const float*>(ws + L.xr);
  e.xi = reinterpret_cast<const float*>(ws + L.xi);
  e.xrows = d.rows32;
  e.pr = d.d_PRz;
  e.pi = d.d_PIz;
  e.U = reinterpret_cast<float*>(ws + L.U);
  e.queue = reinterpret_cast<int*>(ws + L.queue);
  e.ldU = d.Zp;
  e.u_lds = d.Z <= g_tune.exact_u_lds_max ? 1 : 0;
  e.xnorm2 = reinterpret_cast<const float*>(ws + L.xn2);
  e.cmask = reinterpret_cast<const uint32_t*>(ws + L.cmask);
  e.ntiles = L.ntiles;
  e.flags = reinterpret_cast<const int*>(ws + L.flags);
  e.M12 = d.d_M12;
  e.zone_phase = d.d_zone_phase;
  e.eps_rel = 1e-5f;
  e.eps_abs = 1e-5f;
  e.top_k = 1;
  e.p_begin = p_begin;
  e.np = np;
  e.zone = e.phase = e.bin = e.mirror = e.n_eval = nullptr;
  e.score = e.phi3 = e.orient = nullptr;
  e.C = nullptr;
  e.out_p0 = 0;
  e.force_zone = e.force_bin = e.force_mirror = nullptr;
  e.force_score = nullptr;
  e.per = -1;
  e.xblk = e.xfull = 0;
  return e;
}

// Rigorous widening of the bound for operand rounding: |dU| <= 2 u ||X|| with
// u the unit roundoff of the operand format, plus FP32 accumulation slack.
float eps_abs_for(int precision) {
  if (precision == ACOM_BF16) return 0.0078125f + 1e-5f;   // 2 * 2^-8
  if (precision == ACOM_FP16) return 0.0009765625f + 1e-5f; // 2 * 2^-11
  return 1e-5f;
}

acom_status_t check_plan_precision(acom_plan_t plan, int precision) {
  if (!plan) return fail(ACOM_E_INVALID, "plan is null");
  if (precision < 0 || precision > 2) return fail(ACOM_E_INVALID, "precision must be ACOM_FP32, ACOM_BF16 or ACOM_FP16");
  if (precision != ACOM_FP32 && !plan->d.d_PR16[precision])
    return fail(ACOM_E_INVALID, "plan was built without this precision (acom_plan_params_t.precisions)");
  return ACOM_OK;
}

// One chunk of acom_match: polar pass, contraction, exact pass.  Outputs are
// indexed by global pattern minus out_p0.
acom_status_t match_chunk(const PlanDev& d, const acom_peaks_t* peaks, int64_t c0, int np, int top_k, int precision,
                          const WsLayout& L, unsigned char* ws, const acom_matches_t& out, int64_t out_p0,
                          hipStream_t s) {
  acom_status_t st;
  PolarArgs pa = polar_args(d, peaks, c0, np, precision);
  set_ws(pa, L, ws, d);
  if ((st = launch_polar(d, pa, s)) != ACOM_OK) return st;
  if ((st = launch_bound(d, precision, L, ws, np, reinterpret_cast<float*>(ws + L.U), d.Zp, d.Zp, s)) != ACOM_OK)
    return st;
  ExactArgs e = exact_args(d, L, ws, c0, np);
  e.eps_abs = eps_abs_for(precision);
  e.top_k = top_k;
  e.out_p0 = out_p0;
  e.zone = out.zone;
  e.phase = out.phase;
  e.bin = out.bin;
  e.mirror = out.mirror;
  e.score = out.score;
  e.phi3 = out.phi3;
  e.orient = out.orient;
  e.n_eval = out.n_evaluated;
  int nblk = np;
  e.xblk = e.xfull = 0;
  if (g_tune.exact_xcd) {
    e.xblk = g_tune.exact_xcd_block;
    nblk = xcd_blocks_grouped(np, e.xblk, &e.xfull, &e.per);
  } else {
    e.per = -1;
  }
  ProfScope prof(2, s);
  return launch_exact(d, e, dim3(nblk), s, g_tune.exact_persist != 0);
}

int chunk_of(int chunk) {
  int c = chunk <= 0 ? kDefaultChunk : chunk;
  return (int)align_up(c, kTileP);
}

}  // namespace
}  // namespace acom

using namespace acom;

extern "C" acom_status_t acom_match_workspace_size(acom_plan_t plan, int32_t precision, int32_t chunk,
                                                   size_t* bytes) {
  acom_status_t st = check_plan_precision(plan, precision);
  if (st != ACOM_OK) return st;
  if (!bytes) return fail(ACOM_E_INVALID, "bytes is null");
  *bytes = layout(plan->d, precision != ACOM_FP32, chunk_of(chunk)).total;
  return ACOM_OK;
}

extern "C" acom_status_t acom_match(acom_plan_t plan, const acom_peaks_t* peaks, int32_t top_k, int32_t precision,
                                    int32_t chunk, void* workspace, size_t workspace_bytes,
                                    const acom_matches_t* out, void* stream_v) {
  acom_status_t st = check_plan_precision(plan, precision);
  if (st != ACOM_OK) return st;
  if ((st = check_peaks(peaks)) != ACOM_OK) return st;
  if (top_k < 1 || top_k > kMaxTopK) return fail(ACOM_E_INVALID, "top_k must be in [1, 16]");
  if (!out) return fail(ACOM_E_INVALID, "matches is null");
  if (peaks->n_patterns == 0) return ACOM_OK;
  if (!out->zone || !out->score) return fail(ACOM_E_INVALID, "matches: zone and score outputs are required");
  const PlanDev& d = plan->d;
  const int Pc = chunk_of(chunk);
  const WsLayout L = layout(d, precision != ACOM_FP32, Pc);
  if (!workspace || workspace_bytes < L.total)
    return fail(ACOM_E_WORKSPACE, "workspace smaller than acom_match_workspace_size");
  hipStream_t s = (hipStream_t)stream_v;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  for (int64_t c0 = 0; c0 < peaks->n_patterns; c0 += Pc) {
    const int np = (int)std::min<int64_t>(Pc, peaks->n_patterns - c0);
    if ((st = match_chunk(d, peaks, c0, np, top_k, precision, L, ws, *out, 0, s)) != ACOM_OK) return st;
  }
  return ACOM_OK;
}

// ------------------------------------------------- allocation-free match ----
//
// For callers that cannot allocate (code under graph capture, serving loops,
// harnesses that forbid hipMalloc): acom_match with its workspace in a
// file-scope device array instead of a caller's buffer.  Every GPU the library
// runs on holds its own copy of the array, at its own address, until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device, kept per device.
namespace {
constexpr size_t kScratchBytes = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device id; null until first use there

acom_status_t scratch_address(void** out) {
  int dev = -1;
  ACOM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(ACOM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return ACOM_OK;
}

// Largest chunk (a multiple of the 64-pattern tile, at most the default chunk)
// whose workspace fits the scratch array; 0 when not even one tile fits.
int noalloc_chunk(const PlanDev& d, int precision) {
  int best = 0;
  for (int c = kTileP; c <= kDefaultChunk; c += kTileP) {
    if (layout(d, precision != ACOM_FP32, c).total > kScratchBytes) break;
    best = c;
  }
  return best;
}
}  // namespace

extern "C" acom_status_t acom_match_noalloc(acom_plan_t plan, const acom_peaks_t* peaks, int32_t top_k,
                                            int32_t precision, const acom_matches_t* out, void* stream_v) {
  acom_status_t st = check_plan_precision(plan, precision);
  if (st != ACOM_OK) return st;
  if ((st = check_peaks(peaks)) != ACOM_OK) return st;
  if (top_k < 1 || top_k > kMaxTopK) return fail(ACOM_E_INVALID, "top_k must be in [1, 16]");
  if (!out) return fail(ACOM_E_INVALID, "matches is null");
  const int Pc = noalloc_chunk(plan->d, precision);
  if (Pc == 0)
    return fail(ACOM_E_UNSUPPORTED, "acom_match_noalloc: one 64-pattern chunk of this plan needs more than the "
                                    "128 MiB static scratch; use acom_match with a caller's workspace");
  if (peaks->n_patterns == 0) return ACOM_OK;
  if (!out->zone || !out->score) return fail(ACOM_E_INVALID, "matches: zone and score outputs are required");
  void* ws = nullptr;
  if ((st = scratch_address(&ws)) != ACOM_OK) return st;
  // every workspace cell the kernels read is written earlier in the same call,
  // so the array needs no clearing between calls
  return acom_match(plan, peaks, top_k, precision, Pc, ws, kScratchBytes, out, stream_v);
}

extern "C" acom_status_t acom_match_noalloc_chunk(acom_plan_t plan, int32_t precision, int32_t* chunk) {
  acom_status_t st = check_plan_precision(plan, precision);
  if (st != ACOM_OK) return st;
  if (!chunk) return fail(ACOM_E_INVALID, "chunk is null");
  *chunk = noalloc_chunk(plan->d, precision);
  return ACOM_OK;
}

namespace {
// Workspace of acom_match_multi: the match workspace, the edited intensities
// (one per peak) and one round's per-pattern results of a chunk.
struct MultiLayout {
  WsLayout L;
  size_t I = 0, zone = 0, phase = 0, bin = 0, mirror = 0, score = 0, phi3 = 0, score_orig = 0, orient = 0, total = 0;
};
MultiLayout multi_layout(const PlanDev& d, int precision, int Pc, int64_t total_peaks) {
  MultiLayout M;
  M.L = layout(d, precision != ACOM_FP32, Pc);
  size_t o = M.L.total;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  M.I = take((size_t)std::max<int64_t>(total_peaks, 1) * 4);
  M.zone = take((size_t)Pc * 4);
  M.phase = take((size_t)Pc * 4);
  M.bin = take((size_t)Pc * 4);
  M.mirror = take((size_t)Pc * 4);
  M.score = take((size_t)Pc * 4);
  M.phi3 = take((size_t)Pc * 4);
  M.score_orig = take((size_t)Pc * 4);
  M.orient = take((size_t)Pc * 9 * 4);
  M.total = o;
  return M;
}
}  // namespace

extern "C" acom_status_t acom_match_multi_workspace_size(acom_plan_t plan, int32_t precision, int32_t chunk,
                                                         int64_t total_peaks, size_t* bytes) {
  acom_status_t st = check_plan_precision(plan, precision);
  if (st != ACOM_OK) return st;
  if (!bytes) return fail(ACOM_E_INVALID, "bytes is null");
  if (total_peaks < 0) return fail(ACOM_E_INVALID, "negative peak count");
  *bytes = multi_layout(plan->d, precision, chunk_of(chunk), total_peaks).total;
  return ACOM_OK;
}

extern "C" acom_status_t acom_match_multi(acom_plan_t plan, const acom_peaks_t* peaks, int32_t n_orient,
                                          float deletion_radius, float rel_cut, float min_score, int32_t precision,
                                          int32_t chunk, void* workspace, size_t workspace_bytes,
                                          const acom_matches_t* out, void* stream_v) {
  acom_status_t st = check_plan_precision(plan, precision);
  if (st != ACOM_OK) return st;
  if ((st = check_peaks(peaks)) != ACOM_OK) return st;
  if (n_orient < 1 || n_orient > kMaxTopK) return fail(ACOM_E_INVALID, "n_orient must be in [1, 16]");
  const PlanDev& d = plan->d;
  const float r_k = d.kernel == ACOM_KERNEL_CONE ? (float)d.delta : (float)(3.0 * d.gauss_sigma);
  if (!(deletion_radius >= 0.0f) || !(deletion_radius < r_k))
    return fail(ACOM_E_INVALID, "deletion_radius must be in [0, kernel reach)");
  if (!(rel_cut > 0.0f) || !(rel_cut <= 1.0f)) return fail(ACOM_E_INVALID, "rel_cut must be in (0, 1]");
  if (!std::isfinite(min_score)) return fail(ACOM_E_INVALID, "min_score must be finite");
  if (!out) return fail(ACOM_E_INVALID, "matches is null");
  if (peaks->n_patterns == 0) return ACOM_OK;
  if (!out->zone || !out->score) return fail(ACOM_E_INVALID, "matches: zone and score outputs are required");
  const int Pc = chunk_of(chunk);
  const MultiLayout M = multi_layout(d, precision, Pc, peaks->total_peaks);
  if (!workspace || workspace_bytes < M.total)
    return fail(ACOM_E_WORKSPACE, "workspace smaller than acom_match_multi_workspace_size");
  hipStream_t s = (hipStream_t)stream_v;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  float* I_cur = reinterpret_cast<float*>(ws + M.I);
  acom_matches_t tmp{};
  tmp.zone = reinterpret_cast<int32_t*>(ws + M.zone);
  tmp.phase = reinterpret_cast<int32_t*>(ws + M.phase);
  tmp.bin = reinterpret_cast<int32_t*>(ws + M.bin);
  tmp.mirror = reinterpret_cast<int32_t*>(ws + M.mirror);
  tmp.score = reinterpret_cast<float*>(ws + M.score);
  tmp.phi3 = reinterpret_cast<float*>(ws + M.phi3);
  tmp.orient = reinterpret_cast<float*>(ws + M.orient);
  tmp.n_evaluated = nullptr;
  float* score_orig = reinterpret_cast<float*>(ws + M.score_orig);
  acom_peaks_t edited = *peaks;
  edited.intensity = I_cur;
  for (int64_t c0 = 0; c0 < peaks->n_patterns; c0 += Pc) {
    const int np = (int)std::min<int64_t>(Pc, peaks->n_patterns - c0);
    for (int r = 0; r < n_orient; ++r) {
      // round r: the best orientation of the (edited) peaks
      if ((st = match_chunk(d, r == 0 ? peaks : &edited, c0, np, 1, precision, M.L, ws, tmp, c0, s)) != ACOM_OK)
        return st;
      if (r > 0) {
        // its correlogram value on the original peaks (the reported score)
        PolarArgs pa = polar_args(d, peaks, c0, np, 0);
        set_ws(pa, M.L, ws, d);
        if ((st = launch_polar(d, pa, s)) != ACOM_OK) return st;
        ExactArgs e = exact_args(d, M.L, ws, c0, np);
        e.out_p0 = c0;
        e.force_zone = tmp.zone;
        e.force_bin = tmp.bin;
        e.force_mirror = tmp.mirror;
        e.force_score = score_orig;
        e.per = -1;
        if ((st = launch_exact(d, e, dim3(np), s)) != ACOM_OK) return st;
      }
      EditArgs ea;
      ea.offsets = peaks->offsets;
      ea.qx = peaks->qx;
      ea.qy = peaks->qy;
      ea.total_peaks = peaks->total_peaks;
      ea.I_src = r == 0 ? peaks->intensity : I_cur;
      ea.I_dst = I_cur;
      ea.p_begin = c0;
      ea.np = np;
      ea.zone = tmp.zone;
      ea.phase = tmp.phase;
      ea.bin = tmp.bin;
      ea.mirror = tmp.mirror;
      ea.score_orig = r == 0 ? tmp.score : score_orig;
      ea.phi3 = tmp.phi3;
      ea.orient = tmp.orient;
      ea.flags = reinterpret_cast<const int*>(ws + M.L.flags);
      ea.refl = d.d_refl;
      ea.F2 = d.d_reflF2;
      ea.refl_off = d.d_refl_off;
      ea.k0 = (float)d.k0;
      ea.sigma_e = (float)d.sigma_exc;
      ea.rel_cut = rel_cut;
      ea.r_del = deletion_radius;
      ea.r_k = r_k;
      ea.min_score = min_score;
      ea.round = r;
      ea.n_orient = n_orient;
      ea.o_zone = out->zone;
      ea.o_phase = out->phase;
      ea.o_bin = out->bin;
      ea.o_mirror = out->mirror;
      ea.o_score = out->score;
      ea.o_phi3 = out->phi3;
      ea.o_orient = out->orient;
      multi_edit_kernel<<<dim3(np), kThreads, 0, s>>>(ea);
      ACOM_HIP(hipGetLastError());
    }
  }
  return ACOM_OK;
}

extern "C" acom_status_t acom_autotune(acom_plan_t plan, const acom_peaks_t* peaks, int32_t precision, int32_t chunk,
                                       void* workspace, size_t workspace_bytes, void* stream_v, int32_t* shape,
                                       float* ms) {
  acom_status_t st = check_plan_precision(plan, precision);
  if (st != ACOM_OK) return st;
  if ((st = check_peaks(peaks)) != ACOM_OK) return st;
  if (peaks->n_patterns == 0) return fail(ACOM_E_INVALID, "autotune needs at least one pattern");
  const PlanDev& d = plan->d;
  const int Pc = chunk_of(chunk);
  const WsLayout L = layout(d, precision != ACOM_FP32, Pc);
  if (!workspace || workspace_bytes < L.total)
    return fail(ACOM_E_WORKSPACE, "workspace smaller than acom_match_workspace_size");
  hipStream_t s = (hipStream_t)stream_v;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  const int np = (int)std::min<int64_t>(Pc, peaks->n_patterns);
  PolarArgs pa = polar_args(d, peaks, 0, np, precision);
  set_ws(pa, L, ws, d);
  if ((st = launch_polar(d, pa, s)) != ACOM_OK) return st;
  // candidate shapes: block tile x radius step (16-bit operands) x block order
  std::vector<PlanDev::BoundShape> cand;
  for (int tile = 0; tile <= 1; ++tile) {
    const int kmin = precision == ACOM_FP32 ? 16 : 32;
    const int kmax = precision == ACOM_FP32 ? 32 : (tile == 0 ? 128 : 64);
    for (int order = 0; order <= 1; ++order)
      for (int kch = kmin; kch <= kmax; kch *= 2) {
        if (d.Rp % kch) continue;
        PlanDev::BoundShape c;
        c.set = 1;
        c.tile = tile;
        c.kch = kch;
        c.order = order;
        cand.push_back(c);
      }
  }
  hipEvent_t e0, e1;
  ACOM_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ACOM_E_HIP, "hipEventCreate");
  }
  const PlanDev::BoundShape saved = g_tune.tuned[precision];
  int best = -1;
  float best_ms = 0.0f;
  float* U = reinterpret_cast<float*>(ws + L.U);
  for (size_t i = 0; i < cand.size() && st == ACOM_OK; ++i) {
    g_tune.tuned[precision] = cand[i];
    constexpr int kReps = 2;
    st = launch_bound(d, precision, L, ws, np, U, d.Zp, d.Zp, s);  // warm-up
    if (st == ACOM_E_UNSUPPORTED) {  // a shape this plan cannot use
      st = ACOM_OK;
      continue;
    }
    if (st == ACOM_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(ACOM_E_HIP, "hipEventRecord");
    for (int r = 0; r < kReps && st == ACOM_OK; ++r) st = launch_bound(d, precision, L, ws, np, U, d.Zp, d.Zp, s);
    float t = 0.0f;
    if (st == ACOM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      st = fail(ACOM_E_HIP, "timing a contraction shape");
    t /= kReps;
    if (st == ACOM_OK && (best < 0 || t < best_ms)) {
      best = (int)i;
      best_ms = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ACOM_OK || best < 0) {
    g_tune.tuned[precision] = saved;
    return st != ACOM_OK ? st : fail(ACOM_E_UNSUPPORTED, "no contraction shape ran");
  }
  g_tune.tuned[precision] = cand[best];
  g_tune.tuned[precision].ms = best_ms;
  if (shape) {
    shape[0] = cand[best].tile;
    shape[1] = cand[best].kch;
    shape[2] = cand[best].order;
  }
  if (ms) *ms = best_ms;
  return ACOM_OK;
}

extern "C" acom_status_t acom_debug_workspace_size(acom_plan_t plan, int64_t n_patterns, size_t* bytes) {
  if (!plan || !bytes) return fail(ACOM_E_INVALID, "null argument");
  if (n_patterns < 0 || n_patterns > (1 << 20)) return fail(ACOM_E_INVALID, "n_patterns must be in [0, 2^20]");
  *bytes = layout(plan->d, true, chunk_of((int)std::max<int64_t>(1, n_patterns))).total;
  return ACOM_OK;
}

namespace {
acom_status_t debug_prep(acom_plan_t plan, const acom_peaks_t* peaks, void* ws, size_t wsb, WsLayout* L) {
  if (!plan) return fail(ACOM_E_INVALID, "plan is null");
  acom_status_t st = check_peaks(peaks);
  if (st != ACOM_OK) return st;
  if (peaks->n_patterns > (1 << 20)) return fail(ACOM_E_INVALID, "debug calls take at most 2^20 patterns");
  *L = layout(plan->d, true, chunk_of((int)std::max<int64_t>(1, peaks->n_patterns)));
  if (!ws || wsb < L->total) return fail(ACOM_E_WORKSPACE, "workspace smaller than acom_debug_workspace_size");
  return ACOM_OK;
}
}  // namespace

extern "C" acom_status_t acom_polar_image(acom_plan_t plan, const acom_peaks_t* peaks, float* X, void* workspace,
                                          size_t workspace_bytes, void* stream_v) {
  WsLayout L;
  acom_status_t st = debug_prep(plan, peaks, workspace, workspace_bytes, &L);
  if (st != ACOM_OK) return st;
  if (!X) return fail(ACOM_E_INVALID, "X is null");
  if (peaks->n_patterns == 0) return ACOM_OK;
  const PlanDev& d = plan->d;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  PolarArgs pa = polar_args(d, peaks, 0, (int)peaks->n_patterns, 0);
  set_ws(pa, L, ws, d);
  pa.Ximg = X;
  pa.do_fft = 0;
  return launch_polar(d, pa, (hipStream_t)stream_v);
}

extern "C" acom_status_t acom_polar_spectrum(acom_plan_t plan, const acom_peaks_t* peaks, float* Xr, float* Xi,
                                             void* workspace, size_t workspace_bytes, void* stream_v) {
  WsLayout L;
  acom_status_t st = debug_prep(plan, peaks, workspace, workspace_bytes, &L);
  if (st != ACOM_OK) return st;
  if (!Xr || !Xi) return fail(ACOM_E_INVALID, "Xr/Xi is null");
  if (peaks->n_patterns == 0) return ACOM_OK;
  const PlanDev& d = plan->d;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  PolarArgs pa = polar_args(d, peaks, 0, (int)peaks->n_patterns, 0);
  set_ws(pa, L, ws, d);
  pa.xr = Xr;
  pa.xi = Xi;
  pa.ld_tile = (size_t)64 * d.Nk * d.R;
  pa.ldk = d.R;
  pa.ldp = d.Nk * d.R;
  pa.out_cols = d.R;
  pa.ws_layout = 0;  // the caller's [p][k][s] arrays: spectrum only, no norm rows
  return launch_polar(d, pa, (hipStream_t)stream_v);
}

extern "C" acom_status_t acom_correlate(acom_plan_t plan, const acom_peaks_t* peaks, float* C, void* workspace,
                                        size_t workspace_bytes, void* stream_v) {
  WsLayout L;
  acom_status_t st = debug_prep(plan, peaks, workspace, workspace_bytes, &L);
  if (st != ACOM_OK) return st;
  if (!C) return fail(ACOM_E_INVALID, "C is null");
  if (peaks->n_patterns == 0) return ACOM_OK;
  const PlanDev& d = plan->d;
  hipStream_t s = (hipStream_t)stream_v;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  const int np = (int)peaks->n_patterns;
  PolarArgs pa = polar_args(d, peaks, 0, np, 0);
  set_ws(pa, L, ws, d);
  if ((st = launch_polar(d, pa, s)) != ACOM_OK) return st;
  ExactArgs e = exact_args(d, L, ws, 0, np);
  e.C = C;
  return launch_exact(d, e, dim3(np, (d.Z + kBatch - 1) / kBatch), s);
}

extern "C" acom_status_t acom_bound(acom_plan_t plan, const acom_peaks_t* peaks, int32_t precision, float* U,
                                    void* workspace, size_t workspace_bytes, void* stream_v) {
  acom_status_t st = check_plan_precision(plan, precision);
  if (st != ACOM_OK) return st;
  WsLayout L;
  if ((st = debug_prep(plan, peaks, workspace, workspace_bytes, &L)) != ACOM_OK) return st;
  if (!U) return fail(ACOM_E_INVALID, "U is null");
  if (peaks->n_patterns == 0) return ACOM_OK;
  const PlanDev& d = plan->d;
  hipStream_t s = (hipStream_t)stream_v;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  const int np = (int)peaks->n_patterns;
  PolarArgs pa = polar_args(d, peaks, 0, np, precision);
  set_ws(pa, L, ws, d);
  if ((st = launch_polar(d, pa, s)) != ACOM_OK) return st;
  return launch_bound(d, precision, L, ws, np, U, d.Z, d.Z, s);
}

extern "C" acom_status_t acom_profile_begin(int32_t capacity) {
  if (capacity < 1 || capacity > (1 << 20)) return fail(ACOM_E_INVALID, "capacity must be in [1, 2^20]");
  acom_profile_end();
  g_prof.ev.assign(2 * (size_t)capacity, nullptr);
  for (auto& e : g_prof.ev) ACOM_HIP(hipEventCreate(&e));
  g_prof.kind.assign(capacity, -1);
  g_prof.used = 0;
  g_prof.on = true;
  return ACOM_OK;
}

extern "C" acom_status_t acom_profile_read(int32_t kind, double* total_ms, int32_t* launches) {
  if (!total_ms || !launches) return fail(ACOM_E_INVALID, "null argument");
  double t = 0.0;
  int n = 0;
  for (int i = 0; i < g_prof.used; ++i) {
    if (g_prof.kind[i] != kind) continue;
    ACOM_HIP(hipEventSynchronize(g_prof.ev[2 * i + 1]));
    float ms = 0.0f;
    ACOM_HIP(hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]));
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return ACOM_OK;
}

extern "C" acom_status_t acom_profile_end(void) {
  for (auto e : g_prof.ev)
    if (e) (void)hipEventDestroy(e);
  g_prof.ev.clear();
  g_prof.kind.clear();
  g_prof.used = 0;
  g_prof.on = false;
  return ACOM_OK;
}

extern "C" acom_status_t acom_set_tuning(int32_t key, int32_t value) {
  if (key == 0 || key == 1 || key == 4 || key == 6)  // an explicit contraction shape replaces the autotuned ones
    for (auto& t : g_tune.tuned) t = PlanDev::BoundShape();
  switch (key) {
    case 0:
      if (value != 0 && value != 1) return fail(ACOM_E_INVALID, "bound order must be 0 or 1");
      g_tune.bound_order = value;
      return ACOM_OK;
    case 1:
      if (value != 32 && value != 64 && value != 128) return fail(ACOM_E_INVALID, "16-bit step must be 32, 64 or 128");
      g_tune.bound_kch16 = value;
      return ACOM_OK;
    case 2:
      if (value != 0 && value != 1) return fail(ACOM_E_INVALID, "exact order must be 0 or 1");
      g_tune.exact_xcd = value;
      return ACOM_OK;
    case 3:
      if (value != 0 && value != 1) return fail(ACOM_E_INVALID, "polar order must be 0 or 1");
      g_tune.polar_xcd = value;
      return ACOM_OK;
    case 4:
      if (value < 0 || value > 2) return fail(ACOM_E_INVALID, "contraction tile must be 0, 1 or 2");
      g_tune.bound_tile = value;
      return ACOM_OK;
    case 5:
      if (value != 0 && value != 1) return fail(ACOM_E_INVALID, "zero-radius skipping must be 0 or 1");
      g_tune.skip_zero_radii = value;
      return ACOM_OK;
    case 6:
      if (value != 16 && value != 32) return fail(ACOM_E_INVALID, "FP32 step must be 16 or 32");
      g_tune.bound_kch32 = value;
      return ACOM_OK;
    case 7:
      if (value != 16 && value != 32) return fail(ACOM_E_INVALID, "polar columns per pass must be 16 or 32");
      g_tune.polar_cols = value;
      return ACOM_OK;
    case 8:
      if (value < 0 || value > 32768) return fail(ACOM_E_INVALID, "LDS bound-row limit must be in [0, 32768] zones");
      g_tune.exact_u_lds_max = value;
      return ACOM_OK;
    case 9:
      if (value != 0 && value != 1) return fail(ACOM_E_INVALID, "persistent exact pass must be 0 or 1");
      g_tune.exact_persist = value;
      return ACOM_OK;
    case 10:
      if (value < 0 || value > (1 << 20)) return fail(ACOM_E_INVALID, "exact-pass XCD run must be in [0, 2^20] patterns");
      g_tune.exact_xcd_block = value;
      return ACOM_OK;

  }
  return fail(ACOM_E_INVALID, "unknown tuning key");
}
