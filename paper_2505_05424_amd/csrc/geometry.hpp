// Grid geometry and the device-side control block shared by every kernel.
//
// Layout ("padded box"): every plane has nb = N0*N1*...*ND entries with
// N0 = n0+1 (time nodes) and Nd = n_d+1 (spatial nodes), time slowest and the
// last spatial axis fastest. Cell planes (q0, alpha0, cone components) use
// the time slices 0..n0-1; G^s_d planes (q_d, alpha_d) use x_d = 0..n_d-1.
// Unused entries stay zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dot {

constexpr int kMaxAxes = 4;   // time + up to 3 spatial axes
constexpr int kNumSums = 20;  // residual partial sums (see kernels_update.hpp)

struct Geo {
  int D;                     // spatial dimensions
  int K;                     // cone dimension 4D+2
  int N[kMaxAxes];           // nodes per axis (1 for unused axes)
  int n[kMaxAxes];           // segments per axis
  int64_t stride[kMaxAxes];  // plane strides per axis (in elements)
  int64_t nb;                // elements per plane
  int64_t nx;                // spatial nodes per time slice
  double inv_h[kMaxAxes];    // n_d
};

// Device-resident control block: penalty, counters, stop flag and the last
// residuals. Kernels read sigma and stop at entry; the finalize kernel writes.
struct Ctl {
  double sigma;
  double tau;
  double tol;
  double eta[8];   // eta_dot, eta_p, eta_d, eta_c, eta_p_soc, eta_d_soc, c1, c2
  double objective;
  double dual_objective;
  int32_t iter;          // iterations done
  int32_t stop;          // 0 running, 1 converged, 2 iteration limit, 3 diverged
  int32_t checks;
  int32_t sigma_changes;
  int32_t next_update;   // iteration count of the next sigma decision
  int32_t gap;           // current gap of the sigma schedule
  int32_t adapt;         // apply the sigma rule
  int32_t cadence;       // residual-check cadence
  int32_t iter_limit;    // stop (2) at the first check with iter >= iter_limit
  double growth;         // growth factor of the sigma schedule gaps
};

}  // namespace dot
