// Descriptor-driven launches: every kernel of an iteration is one launch over
// all instances of a batch (a single solve is a batch of one). Workgroup b of
// a launch takes the logical index L = xcd_remap(b) and serves instance
// map[L]; its block index inside that instance is L minus the instance's
// first block in that launch's grid. Instances may
// have different grids; each carries its own geometry, state pointers,
// constant tables and control block (sigma, stop flag), so each converges and
// stops on its own.
#pragma once
#include "geometry.hpp"
#include "kernels_dct.hpp"
#include "kernels_update.hpp"

namespace dot {

template <typename T>
struct Inst {
  Geo g;
  double* phi;      // FP64 potential
  T* work;          // transform work plane: phi itself (FP64) or the FP32 scratch
  T* q[2];          // q and q_new, swapped every iteration (parity argument)
  double* alpha;    // multipliers alpha (FP64 in both modes: they accumulate updates)
  T* beta;
  T* W;             // 4D weighted w planes of the z-step
  double* dw;       // w_{K-1} - w_0 of the z-step (FP64)
  Ctl* ctl;         // nullptr for step-level calls (sigma from the argument)
  double* partials;
  const double* sw;
  const double* om;
  const double* c_lo;
  const double* c_hi;
  const T* lam_other;
  const T* lam_last;
  AxisTab<T> tab[kMaxAxes];
  FinArgs fa;
  uint32_t blk0;             // first block in the per-node grid
  uint32_t tile0[kMaxAxes];  // first tile in each axis-pass grid
  int32_t tri;               // last axis solved by tridiagonal elimination (else transform, 1/Lambda, transform)
};

// Instance of logical block L: map[L], or 0 without a map (an executor of
// one instance launches without one, saving the map load at every entry).
__device__ __forceinline__ uint32_t inst_of_block(const uint16_t* __restrict__ map, uint32_t L) {
  return map ? glob(map)[L] : 0u;
}

template <typename T>
__device__ __forceinline__ bool stopped(const Inst<T>& s) {
  return s.ctl && glob(s.ctl)->stop;
}

// z-step of iteration par's parity: cone gather and projection from q[par]
// and beta into the W planes.
template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_cone(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  cone_body<T, D>(s.g, s.q[par], s.beta, s.sw, s.W, s.dw, s.ctl, L - s.blk0);
}

// q-step and alpha update: q[par ^ 1] from phi, alpha and the W planes.
template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_q(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  q_body<T, D>(s.g, s.phi, s.alpha, s.om, s.q[par ^ 1], s.W, s.dw, s.ctl, L - s.blk0);
}

template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_beta(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par, int check) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  beta_body<T, D>(s.g, s.q[par], s.q[par ^ 1], s.beta, s.sw, s.ctl, s.partials, check, L - s.blk0);
}

// beta update of iteration it (no residual check) and the right-hand side of
// iteration it + 1 in one launch: both are sweeps over the same workgroups
// and neither reads what the other writes (rhs reads the new q and alpha, and
// phi for the defect; beta reads q, q_new and beta). sigma does not change
// between them (no check).
template <typename T, int D, bool DEFECT>
__global__ void __launch_bounds__(256)
kb_beta_rhs(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  const double inv_sigma = 1.0 / glob(s.ctl)->sigma;
  beta_body<T, D>(s.g, s.q[par], s.q[par ^ 1], s.beta, s.sw, s.ctl, s.partials, 0, L - s.blk0);
  rhs_body<T, D, DEFECT>(s.g, s.q[par ^ 1], s.alpha, s.phi, s.c_lo, s.c_hi, s.work, inv_sigma, L - s.blk0);
}

// beta update of iteration it (parity par, no residual check) and the z-step
// of iteration it + 1 (parity par ^ 1) in one sweep.
template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_beta_cone(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  beta_cone_body<T, D>(s.g, s.q[par], s.q[par ^ 1], s.beta, s.sw, s.W, s.dw, s.ctl, L - s.blk0);
}

// kb_beta_cone and the right-hand side of iteration it + 1 in one launch (the
// right-hand side reads the new q, alpha and phi, none of which the other
// two steps write).
template <typename T, int D, bool DEFECT>
__global__ void __launch_bounds__(256)
kb_beta_cone_rhs(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  const double inv_sigma = 1.0 / glob(s.ctl)->sigma;
  beta_cone_body<T, D>(s.g, s.q[par], s.q[par ^ 1], s.beta, s.sw, s.W, s.dw, s.ctl, L - s.blk0);
  rhs_body<T, D, DEFECT>(s.g, s.q[par ^ 1], s.alpha, s.phi, s.c_lo, s.c_hi, s.work, inv_sigma, L - s.blk0);
}

// z-step and right-hand side of one iteration in one launch, where neither
// can join the previous beta update (after a residual check, whose sigma
// decision they must see, and at the start of a run): both read q[par] and
// write disjoint planes (W and dw; the transform work plane), and neither
// reads what the other writes.
template <typename T, int D, bool DEFECT>
__global__ void __launch_bounds__(256)
kb_cone_rhs(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  const double inv_sigma = 1.0 / glob(s.ctl)->sigma;
  cone_body<T, D>(s.g, s.q[par], s.beta, s.sw, s.W, s.dw, s.ctl, L - s.blk0);
  rhs_body<T, D, DEFECT>(s.g, s.q[par], s.alpha, s.phi, s.c_lo, s.c_hi, s.work, inv_sigma, L - s.blk0);
}

// Right-hand side (or its defect against phi) of the Poisson solve into the
// transform work plane, from (q[par], alpha).
template <typename T, int D, bool DEFECT>
__global__ void __launch_bounds__(256)
kb_rhs(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par, double sigma_arg) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  const double inv_sigma = 1.0 / (s.ctl ? glob(s.ctl)->sigma : sigma_arg);
  rhs_body<T, D, DEFECT>(s.g, s.q[par], s.alpha, s.phi, s.c_lo, s.c_hi, s.work, inv_sigma, L - s.blk0);
}

// Residual partials at the iterate held in q[par] (the newest q).
template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_resid(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int par) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  resid_body<T, D>(s.g, s.phi, s.q[par], s.alpha, s.beta, s.om, s.sw, s.c_lo, s.c_hi, s.partials, L - s.blk0);
}

// First stage of the residual reduction: kFinChunks blocks per instance
// (block b: instance b / kFinChunks, chunk b % kFinChunks); instances below
// kFinStageMinRows rows return at once.
template <typename T>
__global__ void __launch_bounds__(256)
kb_fin_stage(const Inst<T>* __restrict__ I) {
  const Inst<T>& s = I[blockIdx.x / kFinChunks];
  if (!s.fa.staged || stopped(s)) return;
  fin_stage_body(s.fa, s.partials, (int)(blockIdx.x % kFinChunks));
}

// One block of 256 threads per instance.
template <typename T>
__global__ void __launch_bounds__(256)
kb_finalize(const Inst<T>* __restrict__ I, int update_ctl) {
  const Inst<T>& s = I[blockIdx.x];
  finalize_body(s.fa, s.partials, s.ctl, update_ctl);  // returns before the update if the instance stopped
}

template <typename T, int D, int KIND, int SRC, int DST, int CW>
__global__ void __launch_bounds__(kMaxWaves * 64)
kb_axis_pass(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int axis) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s)) return;
  if (KIND == kFwdScaleInv && s.tri) return;  // this instance's last axis takes kb_tri_pass
  PassArgs pa;
  pa.inner = s.g.stride[axis];
  pa.ncols = s.g.nb / s.g.N[axis];
  axis_pass_body<T, D, KIND, SRC, DST, CW>(s.g, pa, s.tab[axis], s.work, s.phi, s.lam_other, s.lam_last,
                                           (int64_t)(L - s.tile0[axis]));
}

// Last-axis tridiagonal solve over the tiles of the last-axis grid (CW lines
// each); the c' checkpoints go to W plane 0 (an executor with such an
// instance runs the cone step after the phi-step, not beside it).
template <typename T, int D, int CW>
__global__ void __launch_bounds__(kTriThreads)
kb_tri_pass(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s) || !s.tri || s.g.N[D] <= kTriPartMaxNodes) return;  // shorter lines: kb_tri_part
  tri_pass_body<T, CW>(s.g, s.work, s.W, s.lam_other, (int64_t)(L - s.tile0[D]));
}

// Partitioned last-axis solve (lines of up to kTriPartMaxNodes nodes) over the
// same tile grid: tile t of an instance holds its lines [t cw, (t + 1) cw).
template <typename T, int D>
__global__ void __launch_bounds__(kTriThreads, 2)
kb_tri_part(const Inst<T>* __restrict__ I, const uint16_t* __restrict__ map, int cw) {
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const Inst<T>& s = I[inst_of_block(map, L)];
  if (stopped(s) || !s.tri || s.g.N[D] > kTriPartMaxNodes) return;
  tri_part_body<T>(s.g, s.work, s.lam_other, (int64_t)(L - s.tile0[D]), cw);
}

// ---- step-level kernels (single instance, caller pointers) ----------------

// Zero n 32-bit words (one workgroup).
__global__ void __launch_bounds__(256) kb_clear_words(uint32_t* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_cone_out(const Inst<T>* __restrict__ I, double inv_sigma, T* __restrict__ z) {
  const Inst<T>& s = I[0];
  cone_out_body<T, D>(s.g, s.q[0], s.beta, s.sw, inv_sigma, z, blockIdx.x);
}

template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_zres(const Inst<T>* __restrict__ I, const T* __restrict__ z) {
  const Inst<T>& s = I[0];
  zres_body<T, D>(s.g, z, s.q[0], s.sw, s.partials, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_divergence(const Inst<T>* __restrict__ I, double inv_sigma, double* __restrict__ b) {
  const Inst<T>& s = I[0];
  const Geo& g = s.g;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nb) return;
  const int t = (int)(i / g.stride[0]);
  const uint32_t xs = (uint32_t)(i % g.stride[0]);
  int x[kMaxAxes];
  spatial_coords<D>(g, xs, x);
  b[i] = divergence_at<T, D>(g, s.q[0], s.alpha, s.c_lo, s.c_hi, inv_sigma, t, xs, x);
}

}  // namespace dot
