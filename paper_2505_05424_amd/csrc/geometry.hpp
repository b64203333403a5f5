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
constexpr int kBlock = 256;   // lanes per workgroup of the node sweeps

// Pointers into device memory qualified as global, so that loads and stores
// through them compile to global (not flat) memory instructions.
template <typename T>
using gp = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gp<T> glob(T* p) {
  return (gp<T>)p;
}

struct Geo {
  int D;                     // spatial dimensions
  int K;                     // cone dimension 4D+2
  int N[kMaxAxes];           // nodes per axis (1 for unused axes)
  int n[kMaxAxes];           // segments per axis
  int64_t stride[kMaxAxes];  // plane strides per axis (in elements)
  int64_t nb;                // elements per plane
  int64_t nx;                // spatial nodes per time slice
  double inv_h[kMaxAxes];    // n_d
  // node sweeps: a workgroup takes kBlock consecutive spatial nodes and tc
  // consecutive time slices (its lanes march through time); workgroup b of an
  // instance covers spatial block b % nxb and time chunk b / nxb
  uint32_t nxb;              // spatial blocks, ceil(nx / kBlock)
  int32_t tc;                // time slices per workgroup
  uint32_t nsweep;           // workgroups per sweep, nxb * ceil(N0 / tc)
};

// Workgroup b of a launch of G workgroups runs on XCD b % 8; remap so that
// each XCD receives one contiguous range of the logical index (neighbouring
// tiles then share that XCD's L2).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G) {
  const uint32_t q = G >> 3, r = G & 7, x = b & 7, p = b >> 3;
  return x * q + (x < r ? x : r) + p;
}

// Device-resident control block: penalty, counters, stop flag and the last
// residuals. Kernels read sigma and stop at entry; the finalize kernel writes.
constexpr int kSigmaHist = 32;  // sigma changes kept in the control block

// The scalar part, which the finalize step keeps in registers.
struct CtlState {
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

struct Ctl : CtlState {
  // the last kSigmaHist sigma changes (a ring: change j sits at j % kSigmaHist):
  // the new sigma and the iteration count of the check that made it
  double hist_sigma[kSigmaHist];
  int32_t hist_iter[kSigmaHist];
};

}  // namespace dot
