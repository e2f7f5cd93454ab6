// Host-side definitions shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>

#include "gw_physics.hpp"
#include "../../include/gwgen.h"

struct gw_ctx {
  gw_config cfg;
  gw::DevCfg dc;
  double* kcbrt = nullptr;    // [F]  k^(1/3)
  double* lnk3 = nullptr;     // [F]  ln(k)/3
  double* k53 = nullptr;      // [F]  k^(-5/3) (0 at k = 0)
  void* tw_win = nullptr;     // cpx<T>[N/2]
  void* twr_win = nullptr;    // cpx<T>[N/4 + 1]
  void* tw_welch = nullptr;   // cpx<T>[L]
  void* tw_long = nullptr;    // cpx<float>[N2][N1]: W_NC^(m1 k2), windows longer than 32768 samples
  // windows longer than 32768 samples: k^(1/3), ln(k)/3 (double[N/2] each) and
  // exp(-2 pi i k / N) (cpx<float>[N/2]) for k < N/2, stored at the position
  // (k mod N2) N1 + k / N2 of bin k in the transposed four-step spectrum
  void* long_tabs = nullptr;
  int device = 0;             // HIP device the context was created on
  void* scratch = nullptr;    // that device's copy of the library's static scratch area
  std::string err;
};

// A captured batch pipeline; each launch advances the device batch counter.
struct gw_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t* batch = nullptr;  // device batch index inside the caller's workspace
  std::string err;
};

namespace gw {
// Autotuners time every variant once per round and keep each one's best round.
constexpr int kTuneRounds = 3;
struct WinArgs;
gw_status ctx_fail(gw_ctx* c, gw_status s, const std::string& msg);
// Window stage of windows longer than 32768 samples (four-step transforms
// in the output buffer): src 0 whiten, 1 fused batch, 2 inject.
gw_status long_window(gw_ctx* c, int src, const WinArgs& w, const float* x, const float* hdet, int64_t items,
                      hipStream_t st);
// Row length N1 of the four-step split NC = N1 x N2 of those windows.
int long_row_length(int NC);
gw_status ctx_check_launch(gw_ctx* c, const char* what);
// Host validation of a configuration into device constants (nothing launched).
gw_status validate_config(const gw_config* g, DevCfg* dc, std::string* why);
gw_status capture_graph(const std::function<gw_status(hipStream_t)>& enqueue, uint64_t* batch, uint64_t first,
                        gw_graph** out, std::string* why);
}  // namespace gw
