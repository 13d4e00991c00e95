// Forward kinematical diffraction patterns on the GPU (Methods > Calculation of
// Kinematical Diffraction Patterns): for orientation m (sample -> crystal) a
// reflection g of the phase (the plan's reflections, 0 < |g| < k_max) sits at
// the (x, y) of m^T g with intensity |F_g|^2 exp(-s_g^2 / 2 sigma^2) (Eq.
// excitation error with the Gaussian shape factor), and is kept when that
// intensity exceeds rel_cut times the phase's largest |F|^2.
//
// Two calls: acom_simulate_count writes each pattern's peak count and the
// exclusive prefix sum (CSR offsets); acom_simulate_fill writes the peaks in
// reflection order.  One wavefront per pattern, 64 reflections per step, wave
// ballots for the in-order compaction.
#include <cmath>

#include "acom_internal.h"

namespace acom {
namespace {

constexpr int kSimThreads = 256;
constexpr int kScanThreads = 1024;

struct SimArgs {
  int n;
  const float* orient;  // n x 9
  const int* phase;     // n, or null (phase 0)
  const float4* refl;
  const float* F2;
  const int* refl_off;
  int n_phases;
  float k0, sigma, rel_cut;
  int* counts;          // n (count pass)
  const int64_t* offsets;  // n + 1 (fill pass)
  float *qx, *qy, *I;
};

// Hardware square root and reciprocal (<= 1 ulp each) and the exp2-based
// exponential: the kept intensities stay within 1e-5 relative of the exact
// formula (s^2 / 2 sigma^2 < 5 for a kept reflection).
__device__ __forceinline__ float sim_excitation(float x, float y, float z, float k0) {
  const float den = 2.0f * __builtin_amdgcn_sqrtf(x * x + y * y + (k0 + z) * (k0 + z));
  return -(2.0f * k0 * z + (x * x + y * y + z * z)) * __builtin_amdgcn_rcpf(den);
}

// One wavefront per pattern (kSimThreads / 64 patterns per block), no
// barriers: the wave reduces the phase's largest |F|^2, then walks the
// reflections 64 at a time; a ballot and its popcount below the lane give
// every kept reflection its rank in reflection order.
// FILL = false: count the kept reflections; FILL = true: write them from offsets[p].
template <bool FILL>
__global__ void __launch_bounds__(kSimThreads) simulate_kernel(SimArgs a) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * (kSimThreads / 64) + (threadIdx.x >> 6);
  if (p >= a.n) return;
  int ph = a.phase ? a.phase[p] : 0;
  if (ph < 0 || ph >= a.n_phases) ph = -1;
  const int g0 = ph < 0 ? 0 : a.refl_off[ph], g1 = ph < 0 ? 0 : a.refl_off[ph + 1];
  float M[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) M[i] = a.orient[(size_t)p * 9 + i];
  float fm = 0.0f;
  for (int g = g0 + lane; g < g1; g += 64) fm = fmaxf(fm, a.F2[g]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) fm = fmaxf(fm, __shfl_xor(fm, off, 64));
  const float cut = a.rel_cut * fm;
  const float inv2s2 = 1.0f / (2.0f * a.sigma * a.sigma);
  int64_t o = FILL ? a.offsets[p] : 0;
  int kept = 0;
  for (int gb = g0; gb < g1; gb += 64) {
    const int g = gb + lane;
    bool keep = false;
    float x = 0.0f, y = 0.0f, Ig = 0.0f;
    if (g < g1) {
      const float4 r = a.refl[g];
      x = M[0] * r.x + M[3] * r.y + M[6] * r.z;
      y = M[1] * r.x + M[4] * r.y + M[7] * r.z;
      const float z = M[2] * r.x + M[5] * r.y + M[8] * r.z;
      const float sg = sim_excitation(x, y, z, a.k0);
      Ig = a.F2[g] * __expf(-sg * sg * inv2s2);
      keep = Ig > cut;
    }
    const unsigned long long bal = __ballot(keep);
    if (FILL && keep) {
      const int64_t q = o + __popcll(bal & ((1ull << lane) - 1ull));
      a.qx[q] = x;
      a.qy[q] = y;
      a.I[q] = Ig;
    }
    o += __popcll(bal);
    kept += __popcll(bal);
  }
  if (!FILL && lane == 0) a.counts[p] = kept;
}

// offsets[0] = 0, offsets[i + 1] = offsets[i] + counts[i]: one block walks the
// counts in slices of 1024 x kScanPer; each thread sums kScanPer consecutive
// counts, a block-wide scan of those sums gives each thread its base, and the
// thread writes its kScanPer offsets.
constexpr int kScanPer = 16;
__global__ void __launch_bounds__(kScanThreads) scan_counts_kernel(const int* counts, int n, int64_t* offsets) {
  __shared__ int64_t s_wsum[kScanThreads / 64];
  __shared__ int64_t s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    s_carry = 0;
    offsets[0] = 0;
  }
  __syncthreads();
  for (int b = 0; b < n; b += kScanThreads * kScanPer) {
    const int i0 = b + tid * kScanPer;
    int c[kScanPer];
    int64_t v = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
      c[e] = i0 + e < n ? counts[i0 + e] : 0;
      v += c[e];
    }
    // inclusive scan of the thread sums within the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t u = __shfl_up(v, off, 64);
      if (lane >= off) v += u;
    }
    if (lane == 63) s_wsum[wave] = v;
    __syncthreads();
    int64_t run = s_carry;
    for (int w = 0; w < wave; ++w) run += s_wsum[w];
    run += __shfl_up(v, 1, 64) * (lane > 0);  // exclusive within the wave
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
      run += c[e];
      if (i0 + e < n) offsets[i0 + e + 1] = run;
    }
    __syncthreads();
    if (tid == 0) {
      int64_t t = s_carry;
      for (int w = 0; w < kScanThreads / 64; ++w) t += s_wsum[w];
      s_carry = t;
    }
    __syncthreads();
  }
}

acom_status_t sim_args(acom_plan_t plan, int64_t n, const float* orient, const int32_t* phase, float rel_cut,
                       SimArgs* a) {
  if (!plan) return fail(ACOM_E_INVALID, "plan is null");
  if (n < 0 || n > (1 << 24)) return fail(ACOM_E_INVALID, "n must be in [0, 2^24]");
  if (n > 0 && !orient) return fail(ACOM_E_INVALID, "orient is null");
  if (!(rel_cut > 0.0f) || !(rel_cut <= 1.0f)) return fail(ACOM_E_INVALID, "rel_cut must be in (0, 1]");
  const PlanDev& d = plan->d;
  a->n = (int)n;
  a->orient = orient;
  a->phase = phase;
  a->refl = d.d_refl;
  a->F2 = d.d_reflF2;
  a->refl_off = d.d_refl_off;
  a->n_phases = d.n_phases;
  a->k0 = (float)d.k0;
  a->sigma = (float)d.sigma_exc;
  a->rel_cut = rel_cut;
  a->counts = nullptr;
  a->offsets = nullptr;
  a->qx = a->qy = a->I = nullptr;
  return ACOM_OK;
}

}  // namespace

// Exclusive prefix sum of n int32 counts into n + 1 int64 offsets (one block);
// also used by the disk detector.
hipError_t launch_scan_counts(const int32_t* counts, int n, int64_t* offsets, hipStream_t s) {
  scan_counts_kernel<<<1, kScanThreads, 0, s>>>(counts, n, offsets);
  return hipGetLastError();
}

}  // namespace acom

using namespace acom;

extern "C" acom_status_t acom_simulate_count(acom_plan_t plan, int64_t n, const float* orient, const int32_t* phase,
                                             float rel_cut, int32_t* counts, int64_t* offsets, void* stream) {
  SimArgs a;
  acom_status_t st = sim_args(plan, n, orient, phase, rel_cut, &a);
  if (st != ACOM_OK) return st;
  if (!counts || !offsets) return fail(ACOM_E_INVALID, "counts and offsets are required");
  hipStream_t s = (hipStream_t)stream;
  a.counts = counts;
  if (n > 0) {
    simulate_kernel<false><<<dim3((unsigned)((n + kSimThreads / 64 - 1) / (kSimThreads / 64))), kSimThreads, 0, s>>>(a);
    ACOM_HIP(hipGetLastError());
  }
  ACOM_HIP(launch_scan_counts(counts, (int)n, offsets, s));
  return ACOM_OK;
}

extern "C" acom_status_t acom_simulate_fill(acom_plan_t plan, int64_t n, const float* orient, const int32_t* phase,
                                            float rel_cut, const int64_t* offsets, float* qx, float* qy,
                                            float* intensity, void* stream) {
  SimArgs a;
  acom_status_t st = sim_args(plan, n, orient, phase, rel_cut, &a);
  if (st != ACOM_OK) return st;
  if (!offsets || (n > 0 && (!qx || !qy || !intensity))) return fail(ACOM_E_INVALID, "outputs are required");
  a.offsets = offsets;
  a.qx = qx;
  a.qy = qy;
  a.I = intensity;
  if (n > 0) {
    simulate_kernel<true><<<dim3((unsigned)((n + kSimThreads / 64 - 1) / (kSimThreads / 64))), kSimThreads, 0,
                           (hipStream_t)stream>>>(a);
    ACOM_HIP(hipGetLastError());
  }
  return ACOM_OK;
}
