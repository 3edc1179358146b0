// Per-kernel HIP-event timing (see Profiler in internal.h).
#include "internal.h"

namespace sdpm {

const char* const kKernelNames[K_NKERNELS] = {
    "fill", "drift_deposit", "rhs", "residual_fp64", "correct", "reduce_final", "sum_phi",
    "add_const", "smooth_red_zero_guess", "smooth_color", "resid_red", "restrict_fw", "prolong_black",
    "coarse_lds", "interp_kick_drift", "interp_force", "count_kept", "scan_counts", "scatter",
    "copy_back", "morton_radix_sort", "gather", "conv3d_mfma", "conv3d_wgrad_mfma", "net_misc", "force_mesh", "lightcone",
    "smooth_color_coarse", "ade_sweep", "fft_3d", "fft_divide", "power_spectrum", "sweep4_fused",
    "sweep4_fused_zero_guess", "sweep4_fused_coarse", "sweep4_fused_resid", "correct_est", "rhs_force",
};

thread_local Profiler* g_prof = nullptr;

void Profiler::reset() {
  used = 0;
  pend_id.clear();
  pend_bytes.clear();
  pend_launches.clear();
  for (int k = 0; k < K_NKERNELS; ++k) {
    ms[k] = 0.0;
    bytes[k] = 0.0;
    launches[k] = 0;
  }
}

void Profiler::begin(hipStream_t st) {
  if (used + 2 > ev.size()) {
    for (int k = 0; k < 256; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      ev.push_back(e);
    }
  }
  (void)hipEventRecord(ev[used], st);
}

void Profiler::end(hipStream_t st, int id, double b, int nl) {
  if (used + 2 > ev.size()) return;
  (void)hipEventRecord(ev[used + 1], st);
  used += 2;
  pend_id.push_back(id);
  pend_bytes.push_back(b);
  pend_launches.push_back(nl);
}

void Profiler::collect() {
  for (size_t q = 0; q < pend_id.size(); ++q) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ev[2 * q], ev[2 * q + 1]) == hipSuccess) {
      ms[pend_id[q]] += t;
      bytes[pend_id[q]] += pend_bytes[q];
      launches[pend_id[q]] += pend_launches[q];
    }
  }
  used = 0;
  pend_id.clear();
  pend_bytes.clear();
  pend_launches.clear();
}

void Profiler::release() {
  for (auto e : ev) (void)hipEventDestroy(e);
  ev.clear();
  used = 0;
}

}  // namespace sdpm
