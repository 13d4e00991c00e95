// Internal declarations shared by the HIP translation units of libacom.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/acom.h"

namespace acom {

// ------------------------------------------------------------------ errors --
acom_status_t fail(acom_status_t s, const std::string& msg);
acom_status_t hip_fail(hipError_t e, const char* what);
#define ACOM_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return acom::hip_fail(e_, #call); \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Tile-major layout of a set of spectra [rows][Nk][Rp]: rows (patterns or
// zones) grouped in tiles of 64, so that the 64 x Rp block a contraction tile
// reads for one frequency k is contiguous and every row of a tile lies in one
// Nk x 64 x Rp slab:  ((i / 64) * Nk + k) * 64 * Rp + (i % 64) * Rp + s.
__host__ __device__ inline size_t tile_off(int i, int k, int s, int Nk, int Rp) {
  return ((size_t)(i >> 6) * Nk + k) * (size_t)(64 * Rp) + (size_t)(i & 63) * Rp + s;
}

// Tile sizes of the contraction pass (patterns x zones per workgroup) and the
// radial padding unit (one s-chunk of the MFMA K loop).
constexpr int kTileP = 64;
constexpr int kTileZ = 64;
constexpr int kSChunk = 32;
constexpr int kMaxRadices = 12;
constexpr int kMaxAngular = 1024;
constexpr int kMaxTopK = 16;
// default exact frequencies of the split bound, FP32 / 16-bit operands
constexpr int kDefaultExactFreqs[2] = {28, 48};

// Mixed-radix factorisation of the angular length (radices 8, 9, 4, 2, 3, 5, greedily).
struct Radices {
  int n = 0;
  int r[kMaxRadices] = {0};
};
bool factor_angular(int N, Radices* out);

// Device-resident plan.
struct PlanDev {
  // sizes
  int Z = 0, Zp = 0;        // zones, zones padded to kTileZ
  int R = 0, Rp = 0;        // radial bins, padded to kSChunk
  int r0 = 0;               // leading radial bins where FFT{P} is zero in every zone
  // Split bound of the contraction pass: frequencies k < Kc are bounded by the
  // larger modulus of the two correlogram spectra, k >= Kc by Cauchy-Schwarz on
  // blocks of bb radii.  Kc is set per operand precision (index 0: FP32, 1:
  // the 16-bit copies).  The block norms form a vector of L = (Nk - Kc) nb
  // entries per zone (and per pattern) that the operand arrays carry in
  // npseudo extra rows after the spectrum rows, Sp = Rp - r0 entries in the
  // real and Sp in the imaginary array of each row (slots r0 .. Rp-1; slots
  // below r0 hold zeros).  Rows per 64-row tile: rows32 = Nk + npseudo[0] for
  // the FP32 operands (the exact pass reads rows < Nk), rows16 = Kc[1] +
  // npseudo[1] for the 16-bit copies.
  int Kc[2] = {0, 0}, npseudo[2] = {0, 0};
  int64_t L[2] = {0, 0};
  int bb = 8, nb = 0, Sp = 0, rows32 = 0, rows16 = 0;
  int N = 0, Nk = 0;        // angular bins, N/2 + 1
  int n_phases = 0;
  Radices rad;
  // parameters
  double k_max = 0, delta = 0, gamma = 1, omega = 1, k0 = 0, gauss_sigma = 0, sigma_exc = 0.02;
  int kernel = 0, radial = 0;
  int precisions = 1;
  // host copies
  std::vector<double> q_s, zones, normA;  // R, Z*3, Z
  std::vector<int32_t> zone_phase;        // Z
  std::vector<int32_t> refl_off;          // n_phases + 1
  // device arrays
  float* d_qs = nullptr;        // 2 Rp: q_s rounded to FP32 (padding columns -1: no peak reaches them), then q_s - that
  float2* d_tw = nullptr;       // N twiddles (cos, sin)(2 pi m / N)
  int32_t* d_rev = nullptr;     // N: digit-reversed position of index n (in-place FFT input order)
  float* d_M12 = nullptr;       // Z x 9 (row-major, float)
  int32_t* d_zone_phase = nullptr;
  float* d_PR = nullptr;        // FFT{P} real part, FP32, tile-major over Zp zones
  float* d_PI = nullptr;        // imaginary part
  float* d_PRz = nullptr;       // FP32 real part, zone-major [Z][Nk][Rp] (exact pass)
  float* d_PIz = nullptr;
  uint16_t* d_PR16[3] = {nullptr, nullptr, nullptr};  // tile-major 16-bit copies (index = acom_precision_t)
  uint16_t* d_PI16[3] = {nullptr, nullptr, nullptr};
  double* d_Pang = nullptr;     // optional FP64 angular plan Z x N x R
  // a contraction launch shape (block tile, radii per LDS step, block order)
  struct BoundShape {
    int set = 0, tile = 0, kch = 64, order = 1;
    float ms = 0.0f;
  };
  // reflections for the continuous score (all phases concatenated)
  int G = 0;
  float4* d_refl = nullptr;     // (gx, gy, gz, |g|)
  float* d_reflF2 = nullptr;    // |F|^2
  int32_t* d_refl_off = nullptr;
};

}  // namespace acom

struct acom_plan_s {
  acom::PlanDev d;
};
