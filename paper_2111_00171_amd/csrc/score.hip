// Continuous correlation score, its backward, and gradient-ascent refinement.
//
// The continuous analogue of the paper's normalised polar correlation (an
// extension, not in the paper):
//   S = sum_m sum_g w_m v_g K_mg / sqrt(sum_g v_g^2)
//   w_m = q_m^gamma I_m^(omega/2)                               (Eq. image_polar)
//   v_g = |g|^gamma (|F_g|^2 exp(-s_g^2 / 2 sigma_e^2))^(omega/2) (Eq. excitation
//         error with the Gaussian shape factor of Eq. shape_gaussian)
//   K_mg = exp(-|q_m - (x_g, y_g)|^2 / (2 sigma_c^2)), sigma_c = delta / 2,
//   (x_g, y_g, z_g) = m^T g with m = base Exp(theta).
// dS/dtheta uses d(Exp(theta)^T u)/dtheta = [r]x J_r(theta) (SO(3) right Jacobian).
// One wavefront per pattern; lanes own reflections, peaks are streamed from
// LDS.  For omega > 0, reflections with |s_g| >= 10 sigma_e / sqrt(omega) + 0.035
// 1/A are left out: v_g is then below exp(-25) of |g|^gamma |F_g|^omega even
// after a 1 degree rotation (which moves s_g by at most 0.035 1/A for |g| < 2
// 1/A).  The set is taken at the orientation being scored (acom_score,
// acom_score_grad) and, in refinement, at the start orientation and again
// whenever the next trial could lie more than 1 degree from the orientation it
// was taken at (the bound: the accepted steps since then plus the trial's own,
// each a rotation by its step length).  For omega = 0
// all are kept.  At most kMaxKept reflections take part: a pattern whose set
// is larger is an error, reported as NaN (never truncated).
#include <cmath>
#include <type_traits>

#include "acom_internal.h"

namespace acom {
namespace {

constexpr int kW = 64;         // one wavefront per pattern
constexpr int kMaxKept = 1024;  // kept reflections per pattern
constexpr int kPeakChunk = 256;

struct ScoreArgs {
  const int64_t* offsets;
  const float *qx, *qy, *I;
  int64_t total_peaks;
  const float4* refl;
  const float* F2;
  const int* refl_off;
  int n_phases;
  float k0, delta, gamma, omega, sigma_e;
  int n;
  // score / grad
  const float* base;
  const float* theta;
  const int* phase;
  float* S;
  const float* dS;
  float* dtheta;
  float *dqx, *dqy;
  // refine
  int n_cand, max_iter;
  const float* init;
  const int* cand_phase;
  float* out_orient;
  float* out_score;
  int* out_cand;
  int* out_work;           // n x 2 or null: (peak, reflection) pairs evaluated for S alone and with its gradient
};

// v of the lane that DPP control CTRL selects within the same row of 16 lanes
template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the wavefront (every lane active), the same value in every lane:
// within each row of 16 lanes by DPP moves (lanes 2i <-> 2i + 1, the lane pairs
// of a quad, then the mirrored half-row and row, whose lanes hold equal sums by
// then), then the four row sums, read by scalar lane reads, in a fixed order.
__device__ __forceinline__ float wsum(float v) {
  v += dpp_row<0xB1>(v);
  v += dpp_row<0x4E>(v);
  v += dpp_row<0x141>(v);
  v += dpp_row<0x140>(v);
  const int b = __float_as_int(v);
  return (__int_as_float(__builtin_amdgcn_readlane(b, 0)) + __int_as_float(__builtin_amdgcn_readlane(b, 16))) +
         (__int_as_float(__builtin_amdgcn_readlane(b, 32)) + __int_as_float(__builtin_amdgcn_readlane(b, 48)));
}

__device__ __forceinline__ float powe(float x, float e) {
  if (e == 1.0f) return x;
  if (e == 0.5f) return sqrtf(x);
  if (e == 0.0f) return 1.0f;
  if (e == 2.0f) return x * x;
  return powf(x, e);
}

// Rodrigues Exp(theta) into E (row-major).
__device__ void expm3(const float* th, float* E) {
  const float t2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  const float t = sqrtf(t2);
  float a, b;
  if (t < 1e-4f) {
    a = 1.0f - t2 / 6.0f;
    b = 0.5f - t2 / 24.0f;
  } else {
    a = sinf(t) / t;
    b = (1.0f - cosf(t)) / t2;
  }
  const float K[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      float kk = 0.0f;
      for (int l = 0; l < 3; ++l) kk += K[3 * i + l] * K[3 * l + j];
      E[3 * i + j] = (i == j ? 1.0f : 0.0f) + a * K[3 * i + j] + b * kk;
    }
}

__device__ void right_jac(const float* th, float* J) {
  const float t2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  const float t = sqrtf(t2);
  float a, b;
  if (t < 1e-3f) {
    a = 0.5f - t2 / 24.0f;
    b = 1.0f / 6.0f - t2 / 120.0f;
  } else {
    a = (1.0f - cosf(t)) / t2;
    b = (t - sinf(t)) / (t2 * t);
  }
  const float K[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      float kk = 0.0f;
      for (int l = 0; l < 3; ++l) kk += K[3 * i + l] * K[3 * l + j];
      J[3 * i + j] = (i == j ? 1.0f : 0.0f) - a * K[3 * i + j] + b * kk;
    }
}

__device__ void matmul3(const float* A, const float* B, float* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

__device__ __forceinline__ float excitation(float x, float y, float z, float k0) {
  return -(2.0f * k0 * z + (x * x + y * y + z * z)) / (2.0f * sqrtf(x * x + y * y + (k0 + z) * (k0 + z)));
}

// LDS of one pattern: the kept reflections' indices and a chunk of peaks
// (position and weight); the score's peak gradient also keeps each kept
// reflection's projected position and value.
struct Shared {
  float qx[kPeakChunk], qy[kPeakChunk], w[kPeakChunk];
  int kept[kMaxKept];
  int nkept;
};
struct SharedKeep : Shared {
  float rx[kMaxKept], ry[kMaxKept], v[kMaxKept];
};

// Kept reflections of `ph` at orientation m (lane-cooperative, ascending order).
// Returns false (and keeps none) when more than kMaxKept pass the filter.
__device__ bool select_kept(const ScoreArgs& a, int ph, const float* m, Shared& sh) {
  const int lane = threadIdx.x;
  const int g0 = a.refl_off[ph], g1 = a.refl_off[ph + 1];
  const float lim = a.omega > 0.0f ? 10.0f * a.sigma_e / sqrtf(a.omega) + 0.035f : INFINITY;
  int base = 0;
  for (int c = g0; c < g1; c += kW) {
    const int g = c + lane;
    bool keep = false;
    if (g < g1) {
      const float4 r = a.refl[g];
      const float x = m[0] * r.x + m[3] * r.y + m[6] * r.z;
      const float y = m[1] * r.x + m[4] * r.y + m[7] * r.z;
      const float z = m[2] * r.x + m[5] * r.y + m[8] * r.z;
      keep = fabsf(excitation(x, y, z, a.k0)) < lim;
    }
    const unsigned long long bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (keep && base + before < kMaxKept) sh.kept[base + before] = g;
    base += __popcll(bal);
  }
  if (lane == 0) sh.nkept = base <= kMaxKept ? base : 0;
  __syncthreads();
  return base <= kMaxKept;
}

// S, and optionally dS/dtheta (theta-Jacobian J) and the per-reflection
// arrays needed for peak gradients, at orientation R = m (row-major).
struct Eval {
  float S, N, nv;
  float g[3];
};

// Peaks [c0, c0 + cnt) into LDS: position and weight w = q^gamma I^(omega/2).
// Every lane calls; ends with a barrier.
__device__ void load_peaks(const ScoreArgs& a, int64_t c0, int cnt, Shared& sh) {
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += kW) {
    const float x = a.qx[c0 + i], y = a.qy[c0 + i], in = a.I[c0 + i];
    const float q = sqrtf(x * x + y * y);
    sh.qx[i] = x;
    sh.qy[i] = y;
    sh.w[i] = powe(q, a.gamma) * powe(in, 0.5f * a.omega);
  }
  __syncthreads();
}

// The kept reflections are taken 64 at a time, one per lane: its projected
// position, excitation error and value v_g, then its sums over the peaks,
//   ag = sum_m w_m K_mg, (bx, by) = sum_m w_m K_mg (q_m - r_g),
// which it folds at once into N = sum_g ag v_g, sum_g v_g^2 and, for the
// gradient, the two parts of dS/dr_g = dN/dr_g / |v| - N v_g dv_g/dr_g / |v|^3
// (their cross products with r_g, times J, summed separately and combined
// with 1/|v| and N/|v|^3 at the end), so a lane holds one reflection's state.
// K = exp(-d^2 / 2 sigma_c^2) is taken as 2^(-d^2 log2(e) / 2 sigma_c^2) by the
// hardware base-2 exponential. peaks_cached: the pattern's peaks (m1 - m0 <=
// kPeakChunk) are already in LDS.
template <class SH>
__device__ Eval evaluate(const ScoreArgs& a, int64_t m0, int64_t m1, const float* R, const float* J, bool grad,
                         bool keep_arrays, bool peaks_cached, SH& sh) {
  const int lane = threadIdx.x;
  const float sig2 = 0.25f * a.delta * a.delta;
  const float kexp = 1.4426950408889634f / (2.0f * sig2);  // log2(e) / (2 sigma_c^2)
  const float inv2se = 1.0f / (2.0f * a.sigma_e * a.sigma_e);
  const float inv_se2 = 1.0f / (a.sigma_e * a.sigma_e);
  const int nk = sh.nkept;
  float Np = 0.0f, V2 = 0.0f;
  float ga[3] = {0.0f, 0.0f, 0.0f}, gb[3] = {0.0f, 0.0f, 0.0f};
  for (int j0 = 0; j0 < nk; j0 += kW) {
    const int j = j0 + lane;
    const bool act = j < nk;
    float rx = 0.0f, ry = 0.0f, rz = 0.0f, st = 0.0f, v = 0.0f;
    if (act) {
      const int g = sh.kept[j];
      const float4 r = a.refl[g];
      rx = R[0] * r.x + R[3] * r.y + R[6] * r.z;
      ry = R[1] * r.x + R[4] * r.y + R[7] * r.z;
      rz = R[2] * r.x + R[5] * r.y + R[8] * r.z;
      st = excitation(rx, ry, rz, a.k0);
      v = powe(r.w, a.gamma) * powe(a.F2[g] * expf(-st * st * inv2se), 0.5f * a.omega);
    }
    float ag = 0.0f, bx = 0.0f, by = 0.0f;
    for (int64_t c0 = m0; c0 < m1; c0 += kPeakChunk) {
      const int cnt = (int)min((int64_t)kPeakChunk, m1 - c0);
      if (!peaks_cached) load_peaks(a, c0, cnt, sh);
      if (act) {
        if (grad) {
#pragma unroll 4
          for (int i = 0; i < cnt; ++i) {
            const float dx = sh.qx[i] - rx, dy = sh.qy[i] - ry;
            const float wk = sh.w[i] * __builtin_amdgcn_exp2f(-(dx * dx + dy * dy) * kexp);
            ag += wk;
            bx += wk * dx;
            by += wk * dy;
          }
        } else {
#pragma unroll 4
          for (int i = 0; i < cnt; ++i) {
            const float dx = sh.qx[i] - rx, dy = sh.qy[i] - ry;
            ag += sh.w[i] * __builtin_amdgcn_exp2f(-(dx * dx + dy * dy) * kexp);
          }
        }
      }
    }
    Np += ag * v;
    V2 += v * v;
    if constexpr (std::is_same<SH, SharedKeep>::value) {
      if (keep_arrays && act) {
        sh.rx[j] = rx;
        sh.ry[j] = ry;
        sh.v[j] = v;
      }
    }
    if (grad && act) {
      const float D = sqrtf(rx * rx + ry * ry + (a.k0 + rz) * (a.k0 + rz));
      const float f = v * 0.5f * a.omega * (-st * inv_se2);
      const float dvx = f * (-rx / D - st * rx / (D * D));
      const float dvy = f * (-ry / D - st * ry / (D * D));
      const float dvz = f * (-(a.k0 + rz) / D - st * (a.k0 + rz) / (D * D));
      // part 1: dN/dr; part 2: v dv/dr
      const float ax = ag * dvx + v * bx / sig2, ay = ag * dvy + v * by / sig2, az = ag * dvz;
      const float ux = v * dvx, uy = v * dvy, uz = v * dvz;
      // (d x r) J for d = part 1 and part 2
      const float c1x = ay * rz - az * ry, c1y = az * rx - ax * rz, c1z = ax * ry - ay * rx;
      const float c2x = uy * rz - uz * ry, c2y = uz * rx - ux * rz, c2z = ux * ry - uy * rx;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        ga[i] += c1x * J[i] + c1y * J[3 + i] + c1z * J[6 + i];
        gb[i] += c2x * J[i] + c2y * J[3 + i] + c2z * J[6 + i];
      }
    }
  }
  Eval e;
  e.N = wsum(Np);
  const float v2 = wsum(V2);
  e.nv = sqrtf(v2);
  e.S = e.nv > 0.0f ? e.N / e.nv : 0.0f;
  e.g[0] = e.g[1] = e.g[2] = 0.0f;
  if (!grad || !(e.nv > 0.0f)) return e;
  const float c1 = 1.0f / e.nv, c2 = e.N / (e.nv * e.nv * e.nv);
#pragma unroll
  for (int i = 0; i < 3; ++i) e.g[i] = c1 * wsum(ga[i]) - c2 * wsum(gb[i]);
  return e;
}

__global__ void __launch_bounds__(kW) score_kernel(ScoreArgs a) {
  __shared__ SharedKeep sh;
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t m0 = a.offsets[p], m1 = a.offsets[p + 1];
  const int ph = a.phase ? a.phase[p] : 0;
  float base[9], th[3], E[9], R[9], J[9];
  for (int i = 0; i < 9; ++i) base[i] = a.base[(size_t)p * 9 + i];
  for (int i = 0; i < 3; ++i) th[i] = a.theta[(size_t)p * 3 + i];
  if (ph < 0 || ph >= a.n_phases || m0 < 0 || m1 < m0 || m1 > a.total_peaks) {
    if (lane == 0) {
      if (a.S) a.S[p] = NAN;
      if (a.dtheta)
        for (int i = 0; i < 3; ++i) a.dtheta[(size_t)p * 3 + i] = NAN;
    }
    return;
  }
  expm3(th, E);
  matmul3(base, E, R);
  right_jac(th, J);
  const bool grad = a.dtheta != nullptr;
  const bool peak_grad = a.dqx != nullptr || a.dqy != nullptr;
  if (!select_kept(a, ph, R, sh)) {  // more reflections than the cap: an error, never a truncated sum
    if (lane == 0) {
      if (a.S) a.S[p] = NAN;
      if (a.dtheta)
        for (int i = 0; i < 3; ++i) a.dtheta[(size_t)p * 3 + i] = NAN;
    }
    for (int64_t m = m0 + lane; m < m1; m += kW) {
      if (a.dqx) a.dqx[m] = NAN;
      if (a.dqy) a.dqy[m] = NAN;
    }
    return;
  }
  const bool cached = m1 - m0 <= kPeakChunk;  // the pattern's peaks fit the LDS chunk: loaded once
  if (cached) load_peaks(a, m0, (int)(m1 - m0), sh);
  Eval e = evaluate(a, m0, m1, R, J, grad, peak_grad, cached, sh);
  if (!grad) {
    if (lane == 0) a.S[p] = e.S;
    return;
  }
  const float ds = a.dS ? a.dS[p] : 1.0f;
  if (lane == 0) {
    for (int i = 0; i < 3; ++i) a.dtheta[(size_t)p * 3 + i] = ds * e.g[i];
    if (a.S) a.S[p] = e.S;
  }
  if (!peak_grad) return;
  __syncthreads();
  // per-peak gradient: (dw/dq K.v - w sum_g K v d / sig2) / nv
  const float sig2 = 0.25f * a.delta * a.delta;
  const float inv2sc = 1.0f / (2.0f * sig2);
  const int nk = sh.nkept;
  for (int64_t m = m0 + lane; m < m1; m += kW) {
    const float x = a.qx[m], y = a.qy[m], in = a.I[m];
    const float q = sqrtf(x * x + y * y);
    const float w = powe(q, a.gamma) * powe(in, 0.5f * a.omega);
    float kv = 0.0f, kdx = 0.0f, kdy = 0.0f;
    for (int j = 0; j < nk; ++j) {
      const float dx = x - sh.rx[j], dy = y - sh.ry[j];
      const float kvj = expf(-(dx * dx + dy * dy) * inv2sc) * sh.v[j];
      kv += kvj;
      kdx += kvj * dx;
      kdy += kvj * dy;
    }
    float gx = 0.0f, gy = 0.0f;
    if (e.nv > 0.0f) {
      const float inv_q2 = q > 0.0f ? 1.0f / (q * q) : 0.0f;
      gx = (a.gamma * w * x * inv_q2 * kv - w * kdx / sig2) / e.nv;
      gy = (a.gamma * w * y * inv_q2 * kv - w * kdy / sig2) / e.nv;
    }
    if (a.dqx) a.dqx[m] = ds * gx;
    if (a.dqy) a.dqy[m] = ds * gy;
  }
}

__global__ void __launch_bounds__(kW) refine_kernel(ScoreArgs a) {
  __shared__ Shared sh;
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t m0 = a.offsets[p], m1 = a.offsets[p + 1];
  const float deg = 0.017453292519943295f;
  const float lmax = 0.5f * deg, lmin = 1e-4f * deg;
  const float reach = 1.0f * deg;  // rotation within which a kept set stays valid
  float best[9];
  float bestS = -INFINITY;
  int bestc = -1;
  bool overflow = false;
  const int npk = (int)max((int64_t)0, m1 - m0);
  int work_s = 0, work_g = 0;  // pair evaluations (reported when out_work is given)
  // the pattern's peaks, once, when they fit the LDS chunk (else every evaluation streams them)
  const bool range_ok = m0 >= 0 && m1 >= m0 && m1 <= a.total_peaks;
  const bool cached = range_ok && m1 - m0 <= kPeakChunk;
  if (cached) load_peaks(a, m0, npk, sh);
  for (int i = 0; i < 9; ++i) best[i] = 0.0f;
  const float I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int c = 0; c < a.n_cand; ++c) {
    const size_t ci = (size_t)p * a.n_cand + c;
    const int ph = a.cand_phase ? a.cand_phase[ci] : 0;
    float m[9];
    for (int i = 0; i < 9; ++i) m[i] = a.init[ci * 9 + i];
    bool ok = ph >= 0 && ph < a.n_phases && range_ok;
    for (int i = 0; i < 9; ++i) ok = ok && isfinite(m[i]);
    if (!ok) continue;
    __syncthreads();
    if (!select_kept(a, ph, m, sh)) {
      overflow = true;
      break;
    }
    Eval e = evaluate(a, m0, m1, m, I3, true, false, cached, sh);
    work_g += sh.nkept * npk;
    float S = e.S;
    float g[3] = {e.g[0], e.g[1], e.g[2]};
    float l = 0.25f * deg;
    float drift = 0.0f;  // bound on the rotation from where the kept set was taken to m
    int it = 0;
    while (it < a.max_iter && l >= lmin) {
      const float gn = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
      if (!(gn > 0.0f)) break;
      if (drift + l > reach) {  // the trial could leave the set's range: take it again at m
        __syncthreads();
        if (!select_kept(a, ph, m, sh)) {
          overflow = true;
          break;
        }
        drift = 0.0f;
      }
      float th[3] = {l * g[0] / gn, l * g[1] / gn, l * g[2] / gn};
      float E[9], mt[9];
      expm3(th, E);
      matmul3(m, E, mt);
      Eval et = evaluate(a, m0, m1, mt, I3, false, false, cached, sh);
      work_s += sh.nkept * npk;
      ++it;
      if (et.S > S) {
        for (int i = 0; i < 9; ++i) m[i] = mt[i];
        S = et.S;
        drift += l;  // within reach: checked before the trial
        l = fminf(2.0f * l, lmax);
        Eval eg = evaluate(a, m0, m1, m, I3, true, false, cached, sh);
        work_g += sh.nkept * npk;
        g[0] = eg.g[0];
        g[1] = eg.g[1];
        g[2] = eg.g[2];
      } else {
        l *= 0.5f;
      }
    }
    if (overflow) break;
    if (S > bestS) {
      bestS = S;
      bestc = c;
      for (int i = 0; i < 9; ++i) best[i] = m[i];
    }
  }
  if (lane == 0 && a.out_work) {
    a.out_work[2 * (size_t)p] = work_s;
    a.out_work[2 * (size_t)p + 1] = work_g;
  }
  if (overflow) {  // more reflections than the cap for some candidate: the pattern is an error
    if (lane == 0) {
      for (int i = 0; i < 9; ++i) a.out_orient[(size_t)p * 9 + i] = 0.0f;
      if (a.out_score) a.out_score[p] = NAN;
      if (a.out_cand) a.out_cand[p] = -2;
    }
    return;
  }
  if (lane == 0) {
    for (int i = 0; i < 9; ++i) a.out_orient[(size_t)p * 9 + i] = bestc >= 0 ? best[i] : 0.0f;
    if (a.out_score) a.out_score[p] = bestc >= 0 ? bestS : 0.0f;
    if (a.out_cand) a.out_cand[p] = bestc;
  }
}

acom_status_t common_args(acom_plan_t plan, const acom_peaks_t* pk, ScoreArgs* a) {
  if (!plan) return fail(ACOM_E_INVALID, "plan is null");
  if (!pk) return fail(ACOM_E_INVALID, "peaks is null");
  if (pk->n_patterns < 0 || pk->total_peaks < 0) return fail(ACOM_E_INVALID, "negative sizes");
  if (pk->n_patterns > INT_MAX) return fail(ACOM_E_UNSUPPORTED, "too many patterns");
  if (pk->n_patterns > 0 && !pk->offsets) return fail(ACOM_E_INVALID, "offsets is null");
  if (pk->total_peaks > 0 && (!pk->qx || !pk->qy || !pk->intensity)) return fail(ACOM_E_INVALID, "peak arrays are null");
  const PlanDev& d = plan->d;
  *a = ScoreArgs();
  a->offsets = pk->offsets;
  a->qx = pk->qx;
  a->qy = pk->qy;
  a->I = pk->intensity;
  a->total_peaks = pk->total_peaks;
  a->refl = d.d_refl;
  a->F2 = d.d_reflF2;
  a->refl_off = d.d_refl_off;
  a->n_phases = d.n_phases;
  a->k0 = (float)d.k0;
  a->delta = (float)d.delta;
  a->gamma = (float)d.gamma;
  a->omega = (float)d.omega;
  a->sigma_e = (float)d.sigma_exc;
  a->n = (int)pk->n_patterns;
  return ACOM_OK;
}

}  // namespace
}  // namespace acom

using namespace acom;

extern "C" acom_status_t acom_score(acom_plan_t plan, const acom_peaks_t* peaks, const float* base_orient,
                                    const float* theta, const int32_t* phase, float* S, void* stream) {
  ScoreArgs a;
  acom_status_t st = common_args(plan, peaks, &a);
  if (st != ACOM_OK) return st;
  if (a.n == 0) return ACOM_OK;
  if (!base_orient || !theta || !S) return fail(ACOM_E_INVALID, "acom_score: null argument");
  a.base = base_orient;
  a.theta = theta;
  a.phase = phase;
  a.S = S;
  score_kernel<<<a.n, kW, 0, (hipStream_t)stream>>>(a);
  ACOM_HIP(hipGetLastError());
  return ACOM_OK;
}

extern "C" acom_status_t acom_score_grad(acom_plan_t plan, const acom_peaks_t* peaks, const float* base_orient,
                                         const float* theta, const int32_t* phase, const float* dS, float* dtheta,
                                         float* dqx, float* dqy, void* stream) {
  ScoreArgs a;
  acom_status_t st = common_args(plan, peaks, &a);
  if (st != ACOM_OK) return st;
  if (a.n == 0) return ACOM_OK;
  if (!base_orient || !theta || !dtheta) return fail(ACOM_E_INVALID, "acom_score_grad: null argument");
  a.base = base_orient;
  a.theta = theta;
  a.phase = phase;
  a.dS = dS;
  a.dtheta = dtheta;
  a.dqx = dqx;
  a.dqy = dqy;
  score_kernel<<<a.n, kW, 0, (hipStream_t)stream>>>(a);
  ACOM_HIP(hipGetLastError());
  return ACOM_OK;
}

extern "C" acom_status_t acom_refine(acom_plan_t plan, const acom_peaks_t* peaks, int32_t n_cand,
                                     const float* init_orient, const int32_t* cand_phase, int32_t max_iter,
                                     float* out_orient, float* out_score, int32_t* out_cand, int32_t* out_work,
                                     void* stream) {
  ScoreArgs a;
  acom_status_t st = common_args(plan, peaks, &a);
  if (st != ACOM_OK) return st;
  if (n_cand < 1 || n_cand > 64) return fail(ACOM_E_INVALID, "n_cand must be in [1, 64]");
  if (max_iter < 0 || max_iter > 100000) return fail(ACOM_E_INVALID, "max_iter must be in [0, 100000]");
  if (a.n == 0) return ACOM_OK;
  if (!init_orient || !out_orient) return fail(ACOM_E_INVALID, "acom_refine: null argument");
  a.n_cand = n_cand;
  a.max_iter = max_iter;
  a.init = init_orient;
  a.cand_phase = cand_phase;
  a.out_orient = out_orient;
  a.out_score = out_score;
  a.out_cand = out_cand;
  a.out_work = out_work;
  refine_kernel<<<a.n, kW, 0, (hipStream_t)stream>>>(a);
  ACOM_HIP(hipGetLastError());
  return ACOM_OK;
}
