// Orientation plan construction (FP64 on the GPU).
//
// Methods > Structure Factor Calculations: reciprocal basis a* = (b x c)/V etc.
// (no 2 pi), lattice points 0 < |g| < k_max, F_hkl = sum_n f_n exp(-2 pi i hkl.p_n).
// Methods > Generation of an Orientation Plan: SLERP grid of zone axes over
// the boundary triangle(s), rotation M12 = Rz(phi1) Rx(theta2) (first two
// factors of Eq. rotation_matrices, Rx as printed), g' = M12^T g, excitation
// error s_g (Eq. excitation error, beam along +z, alpha = 0), in-plane angle
// gamma_g = atan2(g'_y, g'_x), P0 = sum_g |g|^gamma |F|^omega K(d) with
// d^2 = s_g^2 + rho^2 + (wrap(phi_a - gamma_g) q_s)^2, normalisation
// A = 1/sqrt(sum P0^2), and the FFT of P along phi3.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "acom_internal.h"

namespace acom {
namespace {

constexpr int kPlanThreads = 256;
constexpr int kExcitedCap = 1024;

struct V3 {
  double x, y, z;
};
V3 v3(double x, double y, double z) { return {x, y, z}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
double norm(V3 a) { return std::sqrt(dot(a, a)); }
V3 unit(V3 a) { return scale(a, 1.0 / norm(a)); }

double angle_between(V3 a, V3 b) { return std::acos(std::max(-1.0, std::min(1.0, dot(a, b)))); }

V3 slerp(V3 p0, V3 p1, double t) {
  double om = angle_between(p0, p1);
  if (om < 1e-12) return p0;
  double s = std::sin(om);
  return add(scale(p0, std::sin((1.0 - t) * om) / s), scale(p1, std::sin(t * om) / s));
}

// SLERP grid over one spherical triangle: rows i = 0..N between v0->v1 and
// v0->v2, row i holding i+1 points (row 0 is v0), N = ceil(angle(v0,v1)/step).
void triangle_grid(V3 v0, V3 v1, V3 v2, double step_deg, std::vector<V3>* out) {
  v0 = unit(v0);
  v1 = unit(v1);
  v2 = unit(v2);
  const double deg = angle_between(v0, v1) * 180.0 / M_PI;
  int N = std::max(1, (int)std::ceil(deg / step_deg - 1e-6));
  for (int i = 0; i <= N; ++i) {
    if (i == 0) {
      out->push_back(v0);
      continue;
    }
    V3 a = slerp(v0, v1, (double)i / N), b = slerp(v0, v2, (double)i / N);
    for (int j = 0; j <= i; ++j) out->push_back(slerp(a, b, (double)j / i));
  }
}

// (cos, sin)(2 pi m / N) with exact values on the axes.
void exact_cs(long m, int N, double* c, double* s) {
  m %= N;
  if (m < 0) m += N;
  if ((4 * m) % N == 0) {
    int q = (int)(4 * m / N);
    const double cc[4] = {1, 0, -1, 0}, ss[4] = {0, 1, 0, -1};
    *c = cc[q];
    *s = ss[q];
    return;
  }
  long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)N;
  *c = (double)cosl(a);
  *s = (double)sinl(a);
}

// ------------------------------------------------------------- kernels ----

__global__ void structure_factor_kernel(int G, const int* hkl, const double* gq, int n_atoms,
                                        const double* frac, const int* species, int n_f,
                                        const double* f_q, const double* f_tab, double2* F) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  const double h = hkl[3 * i], k = hkl[3 * i + 1], l = hkl[3 * i + 2];
  const double q = gq[i];
  double re = 0.0, im = 0.0;
  for (int n = 0; n < n_atoms; ++n) {
    double f = 1.0;
    if (n_f > 0) {
      const double* row = f_tab + (size_t)species[n] * n_f;
      if (q <= f_q[0]) {
        f = row[0];
      } else if (q >= f_q[n_f - 1]) {
        f = row[n_f - 1];
      } else {
        int lo = 0, hi = n_f - 1;
        while (hi - lo > 1) {
          int mid = (lo + hi) / 2;
          if (f_q[mid] <= q) lo = mid; else hi = mid;
        }
        double t = (q - f_q[lo]) / (f_q[hi] - f_q[lo]);
        f = row[lo] + t * (row[hi] - row[lo]);
      }
    }
    double ph = -2.0 * M_PI * (h * frac[3 * n] + k * frac[3 * n + 1] + l * frac[3 * n + 2]);
    double sn, cs;
    sincos(ph, &sn, &cs);
    re += f * cs;
    im += f * sn;
  }
  F[i] = make_double2(re, im);
}

struct PlanKernelArgs {
  int Z, N, R;
  const double* zones;      // Z x 3
  const int* zone_phase;    // Z
  const int* refl_off;      // n_phases + 1
  const double* refl;       // G x 5: gx, gy, gz, |g|, amp = |g|^gamma |F|^omega
  const double* q_s;        // R
  double k0, delta, sigma, rk;
  int kernel, radial;
  double* P;                // Z x N x R (output, normalised)
  double* M12;              // Z x 9
  double* normA;            // Z
};

__device__ inline double wrap_pi(double x) {
  const double tp = 2.0 * M_PI;
  double y = x + M_PI;
  y -= tp * floor(y / tp);
  return y - M_PI;
}

__device__ inline double kern64(double d, double delta, double sigma, int kind) {
  if (kind == ACOM_KERNEL_CONE) return d < delta ? 1.0 - d / delta : 0.0;
  return d < 3.0 * sigma ? exp(-d * d / (2.0 * sigma * sigma)) : 0.0;
}

// One block per zone: excited reflections into LDS, then every thread owns
// radial columns and adds each reflection's window of angular bins, in
// reflection order; finally the block normalises the zone.
__global__ void __launch_bounds__(kPlanThreads) plan_zone_kernel(PlanKernelArgs a) {
  const int z = blockIdx.x;
  __shared__ double sq[kExcitedCap], sgam[kExcitedCap], ss[kExcitedCap], samp[kExcitedCap];
  __shared__ int s_count;
  __shared__ double red[kPlanThreads];
  __shared__ double Msh[9];
  double* Pz = a.P + (size_t)z * a.N * a.R;
  const int NR = a.N * a.R;
  for (int i = threadIdx.x; i < NR; i += blockDim.x) Pz[i] = 0.0;
  if (threadIdx.x == 0) {
    const double wx = a.zones[3 * z], wy = a.zones[3 * z + 1], wz = a.zones[3 * z + 2];
    const double th = acos(fmin(1.0, fmax(-1.0, wz)));
    const double ph = (hypot(wx, wy) < 1e-12) ? 0.0 : atan2(-wx, wy);
    const double C1 = cos(ph), S1 = sin(ph), C2 = cos(th), S2 = sin(th);
    const double M[9] = {C1, -S1 * C2, -S1 * S2, S1, C1 * C2, C1 * S2, 0.0, -S2, C2};
    for (int i = 0; i < 9; ++i) {
      Msh[i] = M[i];
      a.M12[(size_t)z * 9 + i] = M[i];
    }
  }
  __syncthreads();
  const int ph = a.zone_phase[z];
  const int g0 = a.refl_off[ph], g1 = a.refl_off[ph + 1];
  const double dphi = 2.0 * M_PI / a.N;
  for (int base = g0; base < g1; base += kExcitedCap) {
    const int gend = min(g1, base + kExcitedCap);
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    // excited set of this batch, kept in reflection order by a serial scan
    if (threadIdx.x == 0) {
      int c = 0;
      for (int g = base; g < gend; ++g) {
        const double* r = a.refl + (size_t)g * 5;
        const double gx = Msh[0] * r[0] + Msh[3] * r[1] + Msh[6] * r[2];
        const double gy = Msh[1] * r[0] + Msh[4] * r[1] + Msh[7] * r[2];
        const double gz = Msh[2] * r[0] + Msh[5] * r[1] + Msh[8] * r[2];
        const double q2 = gx * gx + gy * gy + gz * gz;
        const double sg = -(2.0 * a.k0 * gz + q2) /
                          (2.0 * sqrt(gx * gx + gy * gy + (a.k0 + gz) * (a.k0 + gz)));
        if (fabs(sg) < a.rk) {
          sq[c] = r[3];
          sgam[c] = atan2(gy, gx);
          ss[c] = sg;
          samp[c] = r[4];
          ++c;
        }
      }
      s_count = c;
    }
    __syncthreads();
    const int cnt = s_count;
    for (int s = threadIdx.x; s < a.R; s += blockDim.x) {
      const double qs = a.q_s[s];
      for (int e = 0; e < cnt; ++e) {
        double rho;
        if (a.radial == ACOM_RADIAL_SHELLS) {
          if (fabs(sq[e] - qs) > 1e-9) continue;
          rho = 0.0;
        } else {
          rho = sq[e] - qs;
          if (fabs(rho) >= a.rk) continue;
        }
        const double base2 = ss[e] * ss[e] + rho * rho;
        if (base2 >= a.rk * a.rk) continue;
        // angular window: |wrap(phi_a - gamma)| q_s < rk
        int hw;
        if (qs <= 0.0) {
          hw = a.N;
        } else {
          double w = a.rk / (qs * dphi) + 1.0;
          hw = w > a.N ? a.N : (int)ceil(w);
        }
        if (2 * hw + 1 >= a.N) {
          for (int ai = 0; ai < a.N; ++ai) {
            const double dp = wrap_pi(ai * dphi - sgam[e]) * qs;
            const double k = kern64(sqrt(base2 + dp * dp), a.delta, a.sigma, a.kernel);
            if (k > 0.0) Pz[(size_t)ai * a.R + s] += samp[e] * k;
          }
        } else {
          const int ac = (int)floor(sgam[e] / dphi + 0.5);
          for (int j = -hw; j <= hw; ++j) {
            int ai = (ac + j) % a.N;
            if (ai < 0) ai += a.N;
            const double dp = wrap_pi(ai * dphi - sgam[e]) * qs;
            const double k = kern64(sqrt(base2 + dp * dp), a.delta, a.sigma, a.kernel);
            if (k > 0.0) Pz[(size_t)ai * a.R + s] += samp[e] * k;
          }
        }
      }
    }
    __syncthreads();
  }
  // normalisation A = 1 / sqrt(sum P0^2)
  double acc = 0.0;
  for (int i = threadIdx.x; i < NR; i += blockDim.x) acc += Pz[i] * Pz[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double tot = red[0];
  const double A = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
  for (int i = threadIdx.x; i < NR; i += blockDim.x) Pz[i] *= A;
  if (threadIdx.x == 0) a.normA[z] = A;
}

// FFT{P} along phi3 by a direct FP64 DFT: block (z, k), threads over s.
// Writes the FP32 spectrum zone-major [Z][Nk][Rp] (the exact pass's layout).
__global__ void plan_dft_kernel(int Z, int N, int Nk, int R, int Rp, const double* P, const double2* tw64,
                                float* PRz, float* PIz) {
  const int z = blockIdx.x;
  const int k = blockIdx.y;
  const double* Pz = P + (size_t)z * N * R;
  for (int s = threadIdx.x; s < R; s += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int a = 0; a < N; ++a) {
      const double v = Pz[(size_t)a * R + s];
      const double2 w = tw64[(int)(((long)k * a) % N)];
      re += v * w.x;
      im -= v * w.y;
    }
    const size_t oz = ((size_t)z * Nk + k) * Rp + s;
    PRz[oz] = (float)re;
    PIz[oz] = (float)im;
  }
}

// 16-bit conversions; the _up forms round a nonnegative value up (to the
// next representable value when round-to-nearest went below it), so that the
// block norms of the split bound never shrink.
__device__ __forceinline__ uint16_t bf16_bits(float v) {
  __hip_bfloat16 b = __float2bfloat16(v);
  return *reinterpret_cast<uint16_t*>(&b);
}
__device__ __forceinline__ uint16_t f16_bits(float v) {
  __half h = __float2half(v);
  return *reinterpret_cast<uint16_t*>(&h);
}
__device__ __forceinline__ uint16_t bf16_bits_up(float v) {
  uint16_t b = bf16_bits(v);
  __hip_bfloat16 t;
  *reinterpret_cast<uint16_t*>(&t) = b;
  return __bfloat162float(t) < v ? (uint16_t)(b + 1) : b;
}
__device__ __forceinline__ uint16_t f16_bits_up(float v) {
  uint16_t b = f16_bits(v);
  __half t;
  *reinterpret_cast<uint16_t*>(&t) = b;
  return __half2float(t) < v ? (uint16_t)(b + 1) : b;
}
__device__ __forceinline__ float f32_up(double v) {
  const float f = (float)v;
  return (double)f < v ? nextafterf(f, INFINITY) : f;
}

// Contraction operands, tile-major (64-row zone tiles), from the zone-major
// FP32 spectrum: block (z, row), threads over the row's Rp slots.
//   row < Nk:  FFT{P} at frequency row (FP32, tile stride rows32), and for
//              row < Kc[1] the 16-bit copies (tile stride rows16);
//   row >= Nk: norm row j = row - Nk of the split bound of each precision c
//              (0: FP32, 1: 16-bit) that has one: entry
//              v = (k - Kc[c]) nb + b = ||FFT{P}[z][k][b bb .. b bb + bb)||
//              at slot r0 + v mod Sp of the real (v mod 2Sp < Sp) or
//              imaginary array, FP32 row Nk + j or 16-bit row Kc[1] + j;
//              rounded up (norms of the FP32 values, taken in FP64).
struct TileArgs {
  int Z, Nk, Rp, bb, nb, Sp, r0, rows32, rows16;
  int Kc[2], npseudo[2];
  int64_t L[2];
  const float *PRz, *PIz;
  float *PR, *PI;
  uint16_t *PRb, *PIb, *PRh, *PIh;
};
__global__ void plan_tile_kernel(TileArgs a) {
  const int z = blockIdx.x;
  const int row = blockIdx.y;
  if (row < a.Nk) {
    const int k = row;
    for (int s = threadIdx.x; s < a.Rp; s += blockDim.x) {
      const size_t oz = ((size_t)z * a.Nk + k) * a.Rp + s;
      const float re = a.PRz[oz], im = a.PIz[oz];
      const size_t o = tile_off(z, k, s, a.rows32, a.Rp);
      a.PR[o] = re;
      a.PI[o] = im;
      if (k < a.Kc[1]) {
        const size_t o16 = tile_off(z, k, s, a.rows16, a.Rp);
        if (a.PRb) {
          a.PRb[o16] = bf16_bits(re);
          a.PIb[o16] = bf16_bits(im);
        }
        if (a.PRh) {
          a.PRh[o16] = f16_bits(re);
          a.PIh[o16] = f16_bits(im);
        }
      }
    }
    return;
  }
  const int j = row - a.Nk;
  for (int c = 0; c < 2; ++c) {
    if (j >= a.npseudo[c] || (c == 1 && !a.PRb && !a.PRh)) continue;
    for (int e = threadIdx.x; e < 2 * a.Sp; e += blockDim.x) {
      const int64_t v = (int64_t)j * 2 * a.Sp + e;
      if (v >= a.L[c]) break;
      const int k = a.Kc[c] + (int)(v / a.nb), b = (int)(v % a.nb);
      double n2 = 0.0;
      for (int s = b * a.bb; s < (b + 1) * a.bb; ++s) {
        const size_t oz = ((size_t)z * a.Nk + k) * a.Rp + s;
        const double re = a.PRz[oz], im = a.PIz[oz];
        n2 += re * re + im * im;
      }
      const float nrm = f32_up(sqrt(n2) * (1.0 + 1e-15));
      const int part = e / a.Sp, slot = a.r0 + e % a.Sp;
      if (c == 0) {
        (part ? a.PI : a.PR)[tile_off(z, a.Nk + j, slot, a.rows32, a.Rp)] = nrm;
      } else {
        const size_t o16 = tile_off(z, a.Kc[1] + j, slot, a.rows16, a.Rp);
        if (a.PRb) (part ? a.PIb : a.PRb)[o16] = bf16_bits_up(nrm);
        if (a.PRh) (part ? a.PIh : a.PRh)[o16] = f16_bits_up(nrm);
      }
    }
  }
}

// Radial columns that carry a nonzero FFT{P} value in some zone: block z,
// threads over s, one byte per (z, s); then one thread per s ORs over zones.
__global__ void plan_colnz_kernel(int Z, int Nk, int Rp, const float* PRz, const float* PIz, uint8_t* nz) {
  const int z = blockIdx.x;
  for (int s = threadIdx.x; s < Rp; s += blockDim.x) {
    bool any = false;
    for (int k = 0; k < Nk && !any; ++k) {
      const size_t o = ((size_t)z * Nk + k) * Rp + s;
      any = PRz[o] != 0.0f || PIz[o] != 0.0f;
    }
    nz[(size_t)z * Rp + s] = any ? 1 : 0;
  }
}

__global__ void plan_colany_kernel(int Z, int Rp, const uint8_t* nz, int32_t* colany) {
  for (int s = threadIdx.x; s < Rp; s += blockDim.x) {
    int any = 0;
    for (int z = 0; z < Z && !any; ++z) any = nz[(size_t)z * Rp + s];
    colany[s] = any;
  }
}

template <class T>
acom_status_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return ACOM_OK;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(ACOM_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  return ACOM_OK;
}

void free_plan(PlanDev& d) {
  (void)hipFree(d.d_qs);
  (void)hipFree(d.d_tw);
  (void)hipFree(d.d_rev);
  (void)hipFree(d.d_M12);
  (void)hipFree(d.d_zone_phase);
  (void)hipFree(d.d_PR);
  (void)hipFree(d.d_PI);
  (void)hipFree(d.d_PRz);
  (void)hipFree(d.d_PIz);
  for (int i = 0; i < 3; ++i) {
    (void)hipFree(d.d_PR16[i]);
    (void)hipFree(d.d_PI16[i]);
  }
  (void)hipFree(d.d_Pang);
  (void)hipFree(d.d_refl);
  (void)hipFree(d.d_reflF2);
  (void)hipFree(d.d_refl_off);
}

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  acom_status_t get(T** p, size_t n) {
    acom_status_t s = dalloc(p, n);
    if (s == ACOM_OK && *p) ptrs.push_back(*p);
    return s;
  }
};

acom_status_t validate(const acom_phase_t* phases, int n_phases, const acom_plan_params_t* p) {
  if (!phases || !p) return fail(ACOM_E_INVALID, "acom_build_plan: null phases or params");
  if (n_phases < 1 || n_phases > 127) return fail(ACOM_E_INVALID, "acom_build_plan: n_phases must be in [1, 127]");
  if (!(p->k_max > 0) || !std::isfinite(p->k_max)) return fail(ACOM_E_INVALID, "k_max must be > 0");
  if (!(p->delta > 0) || !std::isfinite(p->delta)) return fail(ACOM_E_INVALID, "delta must be > 0");
  if (!std::isfinite(p->gamma) || !std::isfinite(p->omega)) return fail(ACOM_E_INVALID, "gamma/omega must be finite");
  if (!(p->accel_kV > 0)) return fail(ACOM_E_INVALID, "accel_kV must be > 0");
  const int N = p->n_angular;
  Radices r;
  if (N < 8 || N > kMaxAngular || (N % 2) || !factor_angular(N, &r))
    return fail(ACOM_E_INVALID, "n_angular must be even, in [8, 1024], with prime factors 2, 3, 5 only");
  if (p->radial != ACOM_RADIAL_UNIFORM && p->radial != ACOM_RADIAL_SHELLS)
    return fail(ACOM_E_INVALID, "radial must be ACOM_RADIAL_UNIFORM or ACOM_RADIAL_SHELLS");
  if (p->radial == ACOM_RADIAL_UNIFORM && (p->n_radial < 1 || p->n_radial > 4096))
    return fail(ACOM_E_INVALID, "n_radial must be in [1, 4096]");
  if (p->kernel != ACOM_KERNEL_CONE && p->kernel != ACOM_KERNEL_GAUSS)
    return fail(ACOM_E_INVALID, "kernel must be ACOM_KERNEL_CONE or ACOM_KERNEL_GAUSS");
  if (p->precisions & ~7) return fail(ACOM_E_INVALID, "precisions: unknown bits");
  if (p->bound_exact_freqs < 0 || p->bound_exact_freqs_16bit < 0)
    return fail(ACOM_E_INVALID, "bound_exact_freqs(_16bit) must be >= 0 (0: default)");
  if (p->bound_block_radii != 0 && p->bound_block_radii != 2 && p->bound_block_radii != 4 &&
      p->bound_block_radii != 8 && p->bound_block_radii != 16)
    return fail(ACOM_E_INVALID, "bound_block_radii must be 2, 4, 8 or 16 (0: default 8)");
  for (int i = 0; i < n_phases; ++i) {
    const acom_phase_t& ph = phases[i];
    if (ph.n_atoms < 1 || !ph.frac_xyz) return fail(ACOM_E_INVALID, "phase needs n_atoms >= 1 and frac_xyz");
    if (ph.n_f < 0 || (ph.n_f > 0 && (!ph.f_q || !ph.f_tab)))
      return fail(ACOM_E_INVALID, "phase: n_f > 0 needs f_q and f_tab");
    if (ph.n_f > 0 && !ph.species) return fail(ACOM_E_INVALID, "phase: a scattering-factor table needs species");
    if (ph.n_zones_explicit > 0) {
      if (!ph.zones_explicit) return fail(ACOM_E_INVALID, "phase: zones_explicit is null");
    } else {
      if (ph.n_triangles < 1 || ph.n_triangles > 2) return fail(ACOM_E_INVALID, "phase: n_triangles must be 1 or 2");
      if (!(p->zone_step_deg > 0)) return fail(ACOM_E_INVALID, "zone_step_deg must be > 0");
    }
  }
  return ACOM_OK;
}

}  // namespace
}  // namespace acom

using namespace acom;

extern "C" acom_status_t acom_build_plan(const acom_phase_t* phases, int32_t n_phases,
                                         const acom_plan_params_t* prm, void* stream_v,
                                         acom_plan_t* out) {
  if (!out) return fail(ACOM_E_INVALID, "acom_build_plan: out is null");
  *out = nullptr;
  acom_status_t st = validate(phases, n_phases, prm);
  if (st != ACOM_OK) return st;
  hipStream_t stream = (hipStream_t)stream_v;
  const double kV = prm->accel_kV * 1e3;
  const double hP = 6.62607015e-34, m0 = 9.1093837015e-31, qe = 1.602176634e-19, cL = 299792458.0;
  const double lambda = hP / std::sqrt(2.0 * m0 * qe * kV * (1.0 + qe * kV / (2.0 * m0 * cL * cL))) * 1e10;

  auto* plan = new acom_plan_s();
  PlanDev& d = plan->d;
  d.N = prm->n_angular;
  d.Nk = d.N / 2 + 1;
  factor_angular(d.N, &d.rad);
  d.k_max = prm->k_max;
  d.delta = prm->delta;
  d.gamma = prm->gamma;
  d.omega = prm->omega;
  d.k0 = 1.0 / lambda;
  d.gauss_sigma = prm->gauss_sigma > 0 ? prm->gauss_sigma : 0.5 * prm->delta;
  d.sigma_exc = prm->sigma_exc > 0 ? prm->sigma_exc : 0.02;
  d.kernel = prm->kernel;
  d.radial = prm->radial;
  d.precisions = prm->precisions | 1;
  d.n_phases = n_phases;
  const double rk = d.kernel == ACOM_KERNEL_CONE ? d.delta : 3.0 * d.gauss_sigma;

  Scratch scratch;
  auto bail = [&](acom_status_t s) {
    free_plan(d);
    delete plan;
    return s;
  };

  // ---- reflections per phase (host enumeration; F on the GPU in FP64)
  std::vector<double> refl_all;  // G x 5
  std::vector<float> F2_all;
  std::vector<float4> refl_f;
  d.refl_off.assign(1, 0);
  for (int ip = 0; ip < n_phases; ++ip) {
    const acom_phase_t& ph = phases[ip];
    V3 A = v3(ph.lattice[0][0], ph.lattice[0][1], ph.lattice[0][2]);
    V3 B = v3(ph.lattice[1][0], ph.lattice[1][1], ph.lattice[1][2]);
    V3 C = v3(ph.lattice[2][0], ph.lattice[2][1], ph.lattice[2][2]);
    const double V = dot(A, cross(B, C));
    if (V == 0.0 || !std::isfinite(V)) return bail(fail(ACOM_E_INVALID, "degenerate lattice"));
    V3 As = scale(cross(B, C), 1.0 / V), Bs = scale(cross(C, A), 1.0 / V), Cs = scale(cross(A, B), 1.0 / V);
    const int hm = (int)std::ceil(prm->k_max * norm(A));
    const int km = (int)std::ceil(prm->k_max * norm(B));
    const int lm = (int)std::ceil(prm->k_max * norm(C));
    std::vector<int> hkl;
    std::vector<double> gv, gq;
    for (int h = -hm; h <= hm; ++h)
      for (int k = -km; k <= km; ++k)
        for (int l = -lm; l <= lm; ++l) {
          V3 g = add(add(scale(As, h), scale(Bs, k)), scale(Cs, l));
          double q = norm(g);
          if (q > 0.0 && q < prm->k_max) {
            hkl.insert(hkl.end(), {h, k, l});
            gv.insert(gv.end(), {g.x, g.y, g.z});
            gq.push_back(q);
          }
        }
    const int G = (int)gq.size();
    std::vector<double2> F(G);
    if (G > 0) {
      int *d_hkl = nullptr, *d_sp = nullptr;
      double *d_q = nullptr, *d_frac = nullptr, *d_fq = nullptr, *d_ft = nullptr;
      double2* d_F = nullptr;
      int n_species = 1;
      std::vector<int> sp(ph.n_atoms, 0);
      if (ph.species)
        for (int n = 0; n < ph.n_atoms; ++n) {
          sp[n] = ph.species[n];
          if (sp[n] < 0) return bail(fail(ACOM_E_INVALID, "species must be >= 0"));
          n_species = std::max(n_species, sp[n] + 1);
        }
      if ((st = scratch.get(&d_hkl, 3 * G)) || (st = scratch.get(&d_q, G)) ||
          (st = scratch.get(&d_frac, 3 * ph.n_atoms)) || (st = scratch.get(&d_sp, ph.n_atoms)) ||
          (st = scratch.get(&d_F, G)))
        return bail(st);
      if (ph.n_f > 0) {
        if ((st = scratch.get(&d_fq, ph.n_f)) || (st = scratch.get(&d_ft, (size_t)n_species * ph.n_f))) return bail(st);
        if (hipMemcpy(d_fq, ph.f_q, sizeof(double) * ph.n_f, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_ft, ph.f_tab, sizeof(double) * n_species * ph.n_f, hipMemcpyHostToDevice) != hipSuccess)
          return bail(fail(ACOM_E_HIP, "copy scattering-factor table"));
      }
      if (hipMemcpy(d_hkl, hkl.data(), sizeof(int) * 3 * G, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d_q, gq.data(), sizeof(double) * G, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d_frac, ph.frac_xyz, sizeof(double) * 3 * ph.n_atoms, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d_sp, sp.data(), sizeof(int) * ph.n_atoms, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(ACOM_E_HIP, "copy crystal to device"));
      structure_factor_kernel<<<(G + 255) / 256, 256, 0, stream>>>(G, d_hkl, d_q, ph.n_atoms, d_frac, d_sp, ph.n_f,
                                                                  d_fq, d_ft, d_F);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
        return bail(fail(ACOM_E_HIP, "structure factor kernel"));
      if (hipMemcpy(F.data(), d_F, sizeof(double2) * G, hipMemcpyDeviceToHost) != hipSuccess)
        return bail(fail(ACOM_E_HIP, "copy structure factors"));
    }
    double Imax = 0.0;
    for (int i = 0; i < G; ++i) Imax = std::max(Imax, F[i].x * F[i].x + F[i].y * F[i].y);
    for (int i = 0; i < G; ++i) {
      const double I = F[i].x * F[i].x + F[i].y * F[i].y;
      if (!(I > 1e-12 * Imax)) continue;  // forbidden reflection: round-off only
      const double amp = std::pow(gq[i], prm->gamma) * std::pow(std::sqrt(I), prm->omega);
      refl_all.insert(refl_all.end(), {gv[3 * i], gv[3 * i + 1], gv[3 * i + 2], gq[i], amp});
      F2_all.push_back((float)I);
      refl_f.push_back(make_float4((float)gv[3 * i], (float)gv[3 * i + 1], (float)gv[3 * i + 2], (float)gq[i]));
    }
    d.refl_off.push_back((int)F2_all.size());
  }
  d.G = (int)F2_all.size();

  // ---- zones
  std::vector<double> zl;
  for (int ip = 0; ip < n_phases; ++ip) {
    const acom_phase_t& ph = phases[ip];
    std::vector<V3> pts;
    if (ph.n_zones_explicit > 0) {
      for (int i = 0; i < ph.n_zones_explicit; ++i) {
        V3 w = v3(ph.zones_explicit[3 * i], ph.zones_explicit[3 * i + 1], ph.zones_explicit[3 * i + 2]);
        if (!(norm(w) > 0) || !std::isfinite(norm(w))) return bail(fail(ACOM_E_INVALID, "zero or non-finite zone axis"));
        pts.push_back(unit(w));
      }
    } else {
      std::vector<V3> raw;
      for (int t = 0; t < ph.n_triangles; ++t) {
        V3 c[3];
        for (int i = 0; i < 3; ++i) {
          c[i] = v3(ph.triangles[t][i][0], ph.triangles[t][i][1], ph.triangles[t][i][2]);
          if (!(norm(c[i]) > 0)) return bail(fail(ACOM_E_INVALID, "zero triangle corner"));
        }
        triangle_grid(c[0], c[1], c[2], prm->zone_step_deg, &raw);
      }
      for (const V3& p : raw) {
        bool dup = false;
        for (const V3& q : pts)
          if (norm(add(p, scale(q, -1.0))) <= 1e-9) {
            dup = true;
            break;
          }
        if (!dup) pts.push_back(p);
      }
    }
    for (const V3& p : pts) {
      zl.insert(zl.end(), {p.x, p.y, p.z});
      d.zone_phase.push_back(ip);
    }
  }
  d.Z = (int)d.zone_phase.size();
  if (d.Z < 1) return bail(fail(ACOM_E_INVALID, "no zone axes"));
  d.zones = zl;
  d.Zp = (int)align_up(d.Z, kTileZ);

  // ---- radial axis
  if (d.radial == ACOM_RADIAL_UNIFORM) {
    d.R = prm->n_radial;
    for (int s = 0; s < d.R; ++s) d.q_s.push_back((s + 0.5) * prm->k_max / d.R);
  } else {
    std::vector<double> qs;
    for (int g = 0; g < d.G; ++g) qs.push_back(refl_all[5 * g + 3]);
    std::sort(qs.begin(), qs.end());
    for (double q : qs)
      if (d.q_s.empty() || q - d.q_s.back() > 1e-9) d.q_s.push_back(q);
    d.R = (int)d.q_s.size();
    if (d.R < 1) return bail(fail(ACOM_E_INVALID, "no reflections below k_max"));
  }
  d.Rp = (int)align_up(d.R, kSChunk);

  // ---- device buffers
  const size_t NR = (size_t)d.N * d.R;
  double *d_zones = nullptr, *d_refl = nullptr, *d_qs64 = nullptr, *d_P = nullptr, *d_M12 = nullptr, *d_A = nullptr;
  int *d_zph = nullptr, *d_roff = nullptr;
  double2* d_tw64 = nullptr;
  if ((st = scratch.get(&d_zones, 3 * (size_t)d.Z)) || (st = scratch.get(&d_refl, std::max<size_t>(1, refl_all.size()))) ||
      (st = scratch.get(&d_qs64, d.R)) || (st = scratch.get(&d_M12, 9 * (size_t)d.Z)) ||
      (st = scratch.get(&d_A, d.Z)) || (st = scratch.get(&d_zph, d.Z)) || (st = scratch.get(&d_roff, n_phases + 1)) ||
      (st = scratch.get(&d_tw64, d.N)))
    return bail(st);
  if ((st = dalloc(&d_P, NR * d.Z))) return bail(st);
  d.d_Pang = d_P;  // owned by the plan (freed below unless kept)

  std::vector<double2> tw64(d.N);
  std::vector<float2> tw32(d.N);
  for (int m = 0; m < d.N; ++m) {
    double c, s;
    exact_cs(m, d.N, &c, &s);
    tw64[m] = make_double2(c, s);
    tw32[m] = make_float2((float)c, (float)s);
  }
  if (hipMemcpy(d_zones, zl.data(), sizeof(double) * zl.size(), hipMemcpyHostToDevice) != hipSuccess ||
      (refl_all.size() && hipMemcpy(d_refl, refl_all.data(), sizeof(double) * refl_all.size(), hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(d_qs64, d.q_s.data(), sizeof(double) * d.R, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_zph, d.zone_phase.data(), sizeof(int) * d.Z, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_roff, d.refl_off.data(), sizeof(int) * (n_phases + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_tw64, tw64.data(), sizeof(double2) * d.N, hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(ACOM_E_HIP, "copy plan inputs"));

  PlanKernelArgs ka;
  ka.Z = d.Z;
  ka.N = d.N;
  ka.R = d.R;
  ka.zones = d_zones;
  ka.zone_phase = d_zph;
  ka.refl_off = d_roff;
  ka.refl = d_refl;
  ka.q_s = d_qs64;
  ka.k0 = d.k0;
  ka.delta = d.delta;
  ka.sigma = d.gauss_sigma;
  ka.rk = rk;
  ka.kernel = d.kernel;
  ka.radial = d.radial;
  ka.P = d_P;
  ka.M12 = d_M12;
  ka.normA = d_A;
  plan_zone_kernel<<<d.Z, kPlanThreads, 0, stream>>>(ka);
  if (hipGetLastError() != hipSuccess) return bail(fail(ACOM_E_HIP, "plan_zone_kernel launch"));

  // frequency-domain plan, zone-major FP32 (the exact pass's operand)
  const size_t nfz = (size_t)d.Nk * d.Z * d.Rp;
  if ((st = dalloc(&d.d_PRz, nfz)) || (st = dalloc(&d.d_PIz, nfz))) return bail(st);
  if (hipMemsetAsync(d.d_PRz, 0, nfz * 4, stream) != hipSuccess || hipMemsetAsync(d.d_PIz, 0, nfz * 4, stream) != hipSuccess)
    return bail(fail(ACOM_E_HIP, "memset plan"));
  dim3 gdft(d.Z, d.Nk);
  plan_dft_kernel<<<gdft, 128, 0, stream>>>(d.Z, d.N, d.Nk, d.R, d.Rp, d_P, d_tw64, d.d_PRz, d.d_PIz);
  if (hipGetLastError() != hipSuccess) return bail(fail(ACOM_E_HIP, "plan_dft_kernel launch"));
  // leading radii where every zone's FFT{P} is exactly zero: the contraction
  // may skip them (their terms are exact zeros)
  {
    uint8_t* d_nz = nullptr;
    int32_t* d_colany = nullptr;
    if ((st = dalloc(&d_nz, (size_t)d.Z * d.Rp)) || (st = dalloc(&d_colany, d.Rp))) {
      (void)hipFree(d_nz);
      return bail(st);
    }
    plan_colnz_kernel<<<d.Z, 128, 0, stream>>>(d.Z, d.Nk, d.Rp, d.d_PRz, d.d_PIz, d_nz);
    plan_colany_kernel<<<1, 256, 0, stream>>>(d.Z, d.Rp, d_nz, d_colany);
    std::vector<int32_t> colany(d.Rp, 1);
    const bool ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(stream) == hipSuccess &&
                    hipMemcpy(colany.data(), d_colany, sizeof(int32_t) * d.Rp, hipMemcpyDeviceToHost) == hipSuccess;
    (void)hipFree(d_nz);
    (void)hipFree(d_colany);
    if (!ok) return bail(fail(ACOM_E_HIP, "plan column scan"));
    d.r0 = 0;
    while (d.r0 < d.R && !colany[d.r0]) ++d.r0;
  }
  // ---- split bound and the contraction operands (tile-major over zones)
  d.bb = prm->bound_block_radii > 0 ? prm->bound_block_radii : 16;
  d.nb = d.Rp / d.bb;
  d.Sp = d.Rp - d.r0;
  {
    const int want[2] = {prm->bound_exact_freqs > 0 ? prm->bound_exact_freqs : kDefaultExactFreqs[0],
                         prm->bound_exact_freqs_16bit > 0 ? prm->bound_exact_freqs_16bit : kDefaultExactFreqs[1]};
    for (int c = 0; c < 2; ++c) {
      d.Kc[c] = std::min(want[c], d.Nk);
      if (d.r0 >= d.R) d.Kc[c] = d.Nk;  // a plan that is zero everywhere: nothing to split
      d.L[c] = (int64_t)(d.Nk - d.Kc[c]) * d.nb;
      d.npseudo[c] = d.L[c] > 0 ? (int)((d.L[c] + 2 * d.Sp - 1) / (2 * d.Sp)) : 0;
    }
  }
  d.rows32 = d.Nk + d.npseudo[0];
  d.rows16 = d.Kc[1] + d.npseudo[1];
  // the polar pass addresses one 64-pattern tile of spectrum rows with 32-bit byte offsets
  if ((size_t)d.rows32 * 64 * d.Rp * 4 > (size_t)INT_MAX)
    return bail(fail(ACOM_E_UNSUPPORTED, "plan too large: a 64-pattern tile of spectrum rows exceeds 2 GiB"));
  {
    const size_t n32 = (size_t)d.rows32 * d.Zp * d.Rp, n16 = (size_t)d.rows16 * d.Zp * d.Rp;
    if ((st = dalloc(&d.d_PR, n32)) || (st = dalloc(&d.d_PI, n32))) return bail(st);
    if (hipMemsetAsync(d.d_PR, 0, n32 * 4, stream) != hipSuccess || hipMemsetAsync(d.d_PI, 0, n32 * 4, stream) != hipSuccess)
      return bail(fail(ACOM_E_HIP, "memset plan operands"));
    for (int p = 1; p <= 2; ++p)
      if (d.precisions & (1 << p)) {
        if ((st = dalloc(&d.d_PR16[p], n16)) || (st = dalloc(&d.d_PI16[p], n16))) return bail(st);
        if (hipMemsetAsync(d.d_PR16[p], 0, n16 * 2, stream) != hipSuccess ||
            hipMemsetAsync(d.d_PI16[p], 0, n16 * 2, stream) != hipSuccess)
          return bail(fail(ACOM_E_HIP, "memset plan16"));
      }
    TileArgs ta;
    ta.Z = d.Z;
    ta.Nk = d.Nk;
    ta.Rp = d.Rp;
    ta.bb = d.bb;
    ta.nb = d.nb;
    ta.Sp = d.Sp;
    ta.r0 = d.r0;
    ta.rows32 = d.rows32;
    ta.rows16 = d.rows16;
    for (int c = 0; c < 2; ++c) {
      ta.Kc[c] = d.Kc[c];
      ta.npseudo[c] = d.npseudo[c];
      ta.L[c] = d.L[c];
    }
    ta.PRz = d.d_PRz;
    ta.PIz = d.d_PIz;
    ta.PR = d.d_PR;
    ta.PI = d.d_PI;
    ta.PRb = d.d_PR16[ACOM_BF16];
    ta.PIb = d.d_PI16[ACOM_BF16];
    ta.PRh = d.d_PR16[ACOM_FP16];
    ta.PIh = d.d_PI16[ACOM_FP16];
    plan_tile_kernel<<<dim3(d.Z, d.Nk + std::max(d.npseudo[0], d.npseudo[1])), 128, 0, stream>>>(ta);
    if (hipGetLastError() != hipSuccess) return bail(fail(ACOM_E_HIP, "plan_tile_kernel launch"));
  }

  // small tables
  std::vector<double> M12(9 * (size_t)d.Z);
  d.normA.resize(d.Z);
  if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(ACOM_E_HIP, "plan build kernels"));
  if (hipMemcpy(M12.data(), d_M12, sizeof(double) * M12.size(), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(d.normA.data(), d_A, sizeof(double) * d.Z, hipMemcpyDeviceToHost) != hipSuccess)
    return bail(fail(ACOM_E_HIP, "copy zone tables"));
  std::vector<float> M12f(M12.begin(), M12.end());
  std::vector<int32_t> rev(d.N);
  for (int n = 0; n < d.N; ++n) {
    int pos = 0, S = d.N, m = n;
    for (int i = 0; i < d.rad.n; ++i) {
      S /= d.rad.r[i];
      pos += S * (m % d.rad.r[i]);
      m /= d.rad.r[i];
    }
    rev[n] = pos;
  }
  // q_s as FP32 pairs: hi (padding columns -1) then lo = q_s - hi, so that the
  // polar pass forms q_m - q_s to FP32 precision of the difference itself
  std::vector<float> qsf(2 * (size_t)d.Rp, 0.0f);
  for (int s = 0; s < d.Rp; ++s) qsf[s] = -1.0f;
  for (int s = 0; s < d.R; ++s) {
    qsf[s] = (float)d.q_s[s];
    qsf[d.Rp + s] = (float)(d.q_s[s] - (double)qsf[s]);
  }
  if ((st = dalloc(&d.d_M12, M12f.size())) || (st = dalloc(&d.d_zone_phase, d.Z)) || (st = dalloc(&d.d_qs, 2 * (size_t)d.Rp)) ||
      (st = dalloc(&d.d_tw, d.N)) || (st = dalloc(&d.d_rev, d.N)) || (st = dalloc(&d.d_refl, std::max(1, d.G))) ||
      (st = dalloc(&d.d_reflF2, std::max(1, d.G))) || (st = dalloc(&d.d_refl_off, n_phases + 1)))
    return bail(st);
  if (hipMemcpy(d.d_M12, M12f.data(), sizeof(float) * M12f.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d.d_zone_phase, d.zone_phase.data(), sizeof(int) * d.Z, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d.d_qs, qsf.data(), sizeof(float) * qsf.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d.d_tw, tw32.data(), sizeof(float2) * d.N, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d.d_rev, rev.data(), sizeof(int32_t) * d.N, hipMemcpyHostToDevice) != hipSuccess ||
      (d.G && hipMemcpy(d.d_refl, refl_f.data(), sizeof(float4) * d.G, hipMemcpyHostToDevice) != hipSuccess) ||
      (d.G && hipMemcpy(d.d_reflF2, F2_all.data(), sizeof(float) * d.G, hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(d.d_refl_off, d.refl_off.data(), sizeof(int) * (n_phases + 1), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(ACOM_E_HIP, "copy plan tables"));
  if (!prm->keep_f64) {
    (void)hipFree(d.d_Pang);
    d.d_Pang = nullptr;
  }
  *out = plan;
  return ACOM_OK;
}

extern "C" acom_status_t acom_plan_info(acom_plan_t plan, int32_t* n_zones, int32_t* n_radial,
                                        int32_t* n_angular, int32_t* n_phases, double* q_s, double* zones,
                                        int32_t* zone_phase, double* norm_A) {
  if (!plan) return fail(ACOM_E_INVALID, "acom_plan_info: null plan");
  const PlanDev& d = plan->d;
  if (n_zones) *n_zones = d.Z;
  if (n_radial) *n_radial = d.R;
  if (n_angular) *n_angular = d.N;
  if (n_phases) *n_phases = d.n_phases;
  if (q_s) std::memcpy(q_s, d.q_s.data(), sizeof(double) * d.R);
  if (zones) std::memcpy(zones, d.zones.data(), sizeof(double) * 3 * d.Z);
  if (zone_phase) std::memcpy(zone_phase, d.zone_phase.data(), sizeof(int32_t) * d.Z);
  if (norm_A) std::memcpy(norm_A, d.normA.data(), sizeof(double) * d.Z);
  return ACOM_OK;
}

extern "C" acom_status_t acom_plan_bound_split(acom_plan_t plan, int32_t precision, int32_t* exact_freqs,
                                              int32_t* block_radii) {
  if (!plan) return fail(ACOM_E_INVALID, "plan is null");
  if (precision < 0 || precision > 2) return fail(ACOM_E_INVALID, "precision must be ACOM_FP32, ACOM_BF16 or ACOM_FP16");
  if (exact_freqs) *exact_freqs = plan->d.Kc[precision == ACOM_FP32 ? 0 : 1];
  if (block_radii) *block_radii = plan->d.bb;
  return ACOM_OK;
}

extern "C" acom_status_t acom_plan_copy_f64(acom_plan_t plan, double* host_P) {
  if (!plan || !host_P) return fail(ACOM_E_INVALID, "acom_plan_copy_f64: null argument");
  const PlanDev& d = plan->d;
  if (!d.d_Pang) return fail(ACOM_E_UNSUPPORTED, "plan was built without keep_f64");
  ACOM_HIP(hipMemcpy(host_P, d.d_Pang, sizeof(double) * (size_t)d.Z * d.N * d.R, hipMemcpyDeviceToHost));
  return ACOM_OK;
}

extern "C" acom_status_t acom_plan_destroy(acom_plan_t plan) {
  if (!plan) return ACOM_OK;
  free_plan(plan->d);
  delete plan;
  return ACOM_OK;
}

// Fiber-texture zone sets (Orientation plans of other types: fiber texture).
// The zone axes w within theta_max of the fiber axis f, on rings of polar angle
// theta_i = i step about f (i = 0 .. floor(theta_max / step)), each ring with
// azimuths spaced at most `step` of arc: for a full circle n_i =
// ceil(360 sin theta_i / step) points phi0 + j 360 / n_i; for a wedge
// [phi0, phi1] n_i = ceil((phi1 - phi0) sin theta_i / step) intervals with both
// ends included.  Azimuth 0 is the direction u = unit(f x e), e the coordinate
// axis least aligned with f (ties to the lower index), and 90 degrees is f x u;
// w = cos theta f + sin theta (cos phi u + sin phi v).  Host memory only.
extern "C" acom_status_t acom_fiber_zones(const double* axis, double theta_max_deg, double phi0_deg,
                                          double phi1_deg, double step_deg, double* zones, int32_t capacity,
                                          int32_t* count) {
  if (!axis || !count) return fail(ACOM_E_INVALID, "acom_fiber_zones: axis and count are required");
  if (!(step_deg > 0.0) || !(theta_max_deg >= 0.0) || !(theta_max_deg <= 180.0))
    return fail(ACOM_E_INVALID, "acom_fiber_zones: step > 0 and theta_max in [0, 180] degrees");
  if (!(phi1_deg > phi0_deg) || phi1_deg - phi0_deg > 360.0 + 1e-9)
    return fail(ACOM_E_INVALID, "acom_fiber_zones: need phi0 < phi1 <= phi0 + 360");
  const double nf = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
  if (!(nf > 0.0) || !std::isfinite(nf)) return fail(ACOM_E_INVALID, "acom_fiber_zones: zero or invalid axis");
  const V3 f = v3(axis[0] / nf, axis[1] / nf, axis[2] / nf);
  const double af[3] = {std::fabs(f.x), std::fabs(f.y), std::fabs(f.z)};
  int ie = 0;
  for (int i = 1; i < 3; ++i)
    if (af[i] < af[ie]) ie = i;
  const V3 e = v3(ie == 0 ? 1.0 : 0.0, ie == 1 ? 1.0 : 0.0, ie == 2 ? 1.0 : 0.0);
  const V3 u = unit(cross(f, e));
  const V3 v = cross(f, u);
  const double d2r = 3.14159265358979323846 / 180.0;
  const bool full = phi1_deg - phi0_deg >= 360.0 - 1e-9;
  const int rings = (int)std::floor(theta_max_deg / step_deg + 1e-9);
  int n = 0;
  auto put = [&](V3 w) {
    if (zones && n < capacity) {
      zones[3 * n] = w.x;
      zones[3 * n + 1] = w.y;
      zones[3 * n + 2] = w.z;
    }
    ++n;
  };
  put(f);
  for (int i = 1; i <= rings; ++i) {
    const double th = i * step_deg * d2r;
    const double st = std::sin(th), ct = std::cos(th);
    if (full) {
      const int m = std::max(1, (int)std::ceil(360.0 * st / step_deg - 1e-9));
      for (int j = 0; j < m; ++j) {
        const double ph = (phi0_deg + j * 360.0 / m) * d2r;
        put(add(scale(f, ct), scale(add(scale(u, std::cos(ph)), scale(v, std::sin(ph))), st)));
      }
    } else {
      const int m = std::max(1, (int)std::ceil((phi1_deg - phi0_deg) * st / step_deg - 1e-9));
      for (int j = 0; j <= m; ++j) {
        const double ph = (phi0_deg + j * (phi1_deg - phi0_deg) / m) * d2r;
        put(add(scale(f, ct), scale(add(scale(u, std::cos(ph)), scale(v, std::sin(ph))), st)));
      }
    }
  }
  *count = n;
  if (zones && n > capacity) return fail(ACOM_E_INVALID, "acom_fiber_zones: capacity too small (count holds the need)");
  return ACOM_OK;
}
