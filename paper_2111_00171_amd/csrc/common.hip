// Error reporting and small host helpers of libacom.
#include <cstdio>
#include <string>

#include "acom_internal.h"

namespace acom {

static thread_local std::string g_last_error;

acom_status_t fail(acom_status_t s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

acom_status_t hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return ACOM_E_HIP;
}

bool factor_angular(int N, Radices* out) {
  Radices r;
  int m = N;
  while (m % 8 == 0 && r.n < kMaxRadices) { r.r[r.n++] = 8; m /= 8; }
  while (m % 9 == 0 && r.n < kMaxRadices) { r.r[r.n++] = 9; m /= 9; }
  while (m % 4 == 0 && r.n < kMaxRadices) { r.r[r.n++] = 4; m /= 4; }
  while (m % 2 == 0 && r.n < kMaxRadices) { r.r[r.n++] = 2; m /= 2; }
  while (m % 3 == 0 && r.n < kMaxRadices) { r.r[r.n++] = 3; m /= 3; }
  while (m % 5 == 0 && r.n < kMaxRadices) { r.r[r.n++] = 5; m /= 5; }
  if (m != 1) return false;
  *out = r;
  return true;
}

}  // namespace acom

extern "C" const char* acom_status_string(acom_status_t s) {
  switch (s) {
    case ACOM_OK: return "ok";
    case ACOM_E_INVALID: return "invalid argument";
    case ACOM_E_NOMEM: return "out of device memory";
    case ACOM_E_HIP: return "HIP runtime error";
    case ACOM_E_UNSUPPORTED: return "unsupported";
    case ACOM_E_WORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

extern "C" const char* acom_last_error(void) { return acom::g_last_error.c_str(); }
