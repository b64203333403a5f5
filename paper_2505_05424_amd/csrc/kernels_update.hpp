// Cone gather + projection, proximal q update, multiplier updates and the
// KKT-residual reductions of Algorithm 2 (z-step, q-step, multiplier steps)
// and Sec. 5.3.
//
// Every kernel is a coalesced sweep over the padded box: one lane per node
// (or per cell), neighbours along axis d at +-stride[d]. The four maps F^d_v
// of eq. fdetails read, for cell (t, x):
//   v=1: q_d[t,   x - e_d] (x_d >= 1)    v=2: q_d[t,   x] (x_d <= n_d - 1)
//   v=3: q_d[t+1, x - e_d] (x_d >= 1)    v=4: q_d[t+1, x] (x_d <= n_d - 1)
// and the adjoint sends the value of component (d, v) of a cell back to the
// same q_d entry, so q_d[t, s] collects v=1 from cell (t, s+1), v=2 from
// (t, s), v=3 from (t-1, s+1) and v=4 from (t-1, s).
#pragma once
#include "geometry.hpp"

namespace dot {

template <int D>
__device__ __forceinline__ void node_coords(const Geo& g, int64_t i, int (&x)[kMaxAxes]) {
  int64_t r = i;
#pragma unroll
  for (int d = D; d >= 1; --d) {
    x[d] = (int)(r % g.N[d]);
    r /= g.N[d];
  }
  x[0] = (int)r;
}

// u = B_omega F q + d - beta/sigma at cell i (argument of the z-step
// projection of Algorithm 2), in double.
// sw = sqrt(omega/2) of the cell.
template <typename T, int D>
__device__ __forceinline__ void cone_input(const Geo& g, const T* __restrict__ q, const T* __restrict__ beta,
                                           int64_t i, const int (&x)[kMaxAxes], double sw, double inv_sigma,
                                           double (&u)[4 * D + 2]) {
  constexpr int K = 4 * D + 2;
  const int64_t nb = g.nb;
  const double q0 = (double)q[i];
  u[0] = 1.0 - q0 - (double)beta[i] * inv_sigma;
  u[K - 1] = 1.0 + q0 - (double)beta[(K - 1) * nb + i] * inv_sigma;
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    const T* qd = q + d * nb;
    const bool lo = x[d] >= 1;
    const bool hi = x[d] < g.n[d];
    const int64_t sd = g.stride[d], s0 = g.stride[0];
    const double f1 = lo ? (double)qd[i - sd] : 0.0;
    const double f2 = hi ? (double)qd[i] : 0.0;
    const double f3 = lo ? (double)qd[i + s0 - sd] : 0.0;
    const double f4 = hi ? (double)qd[i + s0] : 0.0;
    const int k = 1 + 4 * (d - 1);
    u[k + 0] = sw * f1 - (double)beta[(k + 0) * nb + i] * inv_sigma;
    u[k + 1] = sw * f2 - (double)beta[(k + 1) * nb + i] * inv_sigma;
    u[k + 2] = sw * f3 - (double)beta[(k + 2) * nb + i] * inv_sigma;
    u[k + 3] = sw * f4 - (double)beta[(k + 3) * nb + i] * inv_sigma;
  }
}

// Projection onto the second-order cone {y0 >= |ybar|} (eq. app-proj), in
// place, in double: y if |ybar| <= y0; 0 if |ybar| <= -y0; otherwise
// 1/2 (y0 + |ybar|) (1; ybar/|ybar|).
template <int K>
__device__ __forceinline__ void soc_project(double (&y)[K]) {
  double n2 = 0.0;
#pragma unroll
  for (int k = 1; k < K; ++k) n2 = fma(y[k], y[k], n2);
  const double nrm = sqrt(n2);
  const double y0 = y[0];
  if (nrm <= y0) return;
  if (nrm <= -y0) {
#pragma unroll
    for (int k = 0; k < K; ++k) y[k] = 0.0;
    return;
  }
  const double a = 0.5 * (y0 + nrm);
  const double s = a / nrm;
  y[0] = a;
#pragma unroll
  for (int k = 1; k < K; ++k) y[k] *= s;
}

// ---- node sweeps ------------------------------------------------------------
// A workgroup owns kBlock consecutive spatial nodes and the time slices
// [t0, t1) of one chunk; each lane walks its spatial node through those slices,
// so the values at slice t+1 that the cell at t needs (q_d, phi) are loaded
// once and carried to the next slice in registers.
struct Column {
  uint32_t xs;          // spatial index of the lane
  bool live;            // xs < nx
  int x[kMaxAxes];      // spatial coordinates x[1..D]
  int t0, t1;           // time slices of the workgroup
};

template <int D>
__device__ __forceinline__ Column column_of(const Geo& g, uint32_t blk) {
  Column c;
  const uint32_t tci = blk / g.nxb;
  const uint32_t xb = blk - tci * g.nxb;
  c.xs = xb * kBlock + threadIdx.x;
  c.live = c.xs < (uint32_t)g.nx;
  uint32_t r = c.live ? c.xs : 0u;
#pragma unroll
  for (int d = D; d >= 1; --d) {
    const uint32_t Nd = (uint32_t)g.N[d];
    const uint32_t qd = r / Nd;
    c.x[d] = (int)(r - qd * Nd);
    r = qd;
  }
  c.t0 = (int)tci * g.tc;
  c.t1 = min(c.t0 + g.tc, g.N[0]);
  return c;
}

// Values of F^d_v q at one cell that come from one time slice: for each d,
// [0] = q_d[t, x - e_d] (x_d >= 1, else 0) and [1] = q_d[t, x] (x_d < n_d),
// kept in the storage type (they are widened to double where used).
template <typename T, int D>
__device__ __forceinline__ void load_fq(const Geo& g, gp<const T> q, uint32_t i, const Column& c,
                                        T (&f)[kMaxAxes][2]) {
  const uint32_t nb = (uint32_t)g.nb;
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    gp<const T> qd = q + (size_t)d * nb;
    const uint32_t sd = (uint32_t)g.stride[d];
    f[d][0] = c.x[d] >= 1 ? qd[i - sd] : T(0);
    f[d][1] = c.x[d] < g.n[d] ? qd[i] : T(0);
  }
}

template <typename T, int D>
__device__ __forceinline__ void shift_fq(T (&a)[kMaxAxes][2], const T (&b)[kMaxAxes][2]) {
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    a[d][0] = b[d][0];
    a[d][1] = b[d][1];
  }
}

// u = B_omega F q + d - beta/sigma at a cell from its beta values bt, q0 and
// the F q values of slices t (fa) and t+1 (fb), in double.
template <typename T, int D>
__device__ __forceinline__ void cone_arg(const T (&bt)[4 * D + 2], double q0, const T (&fa)[kMaxAxes][2],
                                         const T (&fb)[kMaxAxes][2], double sw, double inv_sigma,
                                         double (&u)[4 * D + 2]) {
  constexpr int K = 4 * D + 2;
  u[0] = 1.0 - q0 - (double)bt[0] * inv_sigma;
  u[K - 1] = 1.0 + q0 - (double)bt[K - 1] * inv_sigma;
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    const int k = 1 + 4 * (d - 1);
    u[k + 0] = sw * (double)fa[d][0] - (double)bt[k + 0] * inv_sigma;
    u[k + 1] = sw * (double)fa[d][1] - (double)bt[k + 1] * inv_sigma;
    u[k + 2] = sw * (double)fb[d][0] - (double)bt[k + 2] * inv_sigma;
    u[k + 3] = sw * (double)fb[d][1] - (double)bt[k + 3] * inv_sigma;
  }
}

// z-step output of one cell from its projected u = Pi(...) and the beta
// values bt the argument was formed with: w = z - d + beta/sigma; the
// weighted components sqrt(omega/2) w_{d,v} go to the W planes (for the q_d
// update) and w_{K-1} - w_0 to the FP64 plane DW (for the q0 update: in the
// storage type its rounding would enter every alpha0 increment, which near
// convergence are smaller than that rounding).
template <typename T, int D>
__device__ __forceinline__ void cone_store(const double (&u)[4 * D + 2], const T (&bt)[4 * D + 2], double sw,
                                           double inv_sigma, gp<T> W, gp<double> DW, uint32_t nb, uint32_t i) {
  constexpr int K = 4 * D + 2;
  const double w0 = u[0] - 1.0 + (double)bt[0] * inv_sigma;
  const double wl = u[K - 1] - 1.0 + (double)bt[K - 1] * inv_sigma;
#pragma unroll
  for (int k = 1; k < K - 1; ++k) W[(size_t)(k - 1) * nb + i] = (T)(sw * (u[k] + (double)bt[k] * inv_sigma));
  DW[i] = wl - w0;
}

// a1 + a2 per cell (the z-step of Algorithm 2): z = Pi(u), then cone_store.
// Reads only q and beta, so it may run while the phi-step is being solved.
template <typename T, int D>
__device__ __forceinline__ void cone_body(const Geo& g, const T* __restrict__ q_, const T* __restrict__ beta_,
                                          const double* __restrict__ sw_sp, T* __restrict__ W_,
                                          double* __restrict__ DW_, const Ctl* __restrict__ ctl, uint32_t blk) {
  constexpr int K = 4 * D + 2;
  const Column c = column_of<D>(g, blk);
  const int tend = min(c.t1, g.n[0]);
  if (!c.live || c.t0 >= tend) return;
  gp<const T> q = glob(q_);
  gp<const T> beta = glob(beta_);
  gp<T> W = glob(W_);
  gp<double> DW = glob(DW_);
  const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx;
  const double inv_sigma = 1.0 / glob(ctl)->sigma;
  const double sw = glob(sw_sp)[c.xs];
  uint32_t i = (uint32_t)c.t0 * nx + c.xs;
  T fa[kMaxAxes][2], fb[kMaxAxes][2];
  load_fq<T, D>(g, q, i, c, fa);
  for (int t = c.t0; t < tend; ++t, i += nx) {
    load_fq<T, D>(g, q, i + nx, c, fb);
    T bt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) bt[k] = beta[(size_t)k * nb + i];
    const double q0 = (double)q[i];
    double u[K];
    cone_arg<T, D>(bt, q0, fa, fb, sw, inv_sigma, u);
    soc_project<K>(u);
    cone_store<T, D>(u, bt, sw, inv_sigma, W, DW, nb, i);
    shift_fq<T, D>(fa, fb);
  }
}

// q_d update (d >= 1) of a5 per node: rhs = A_d phi + alpha_d/sigma + the four
// adjacent cells' weighted w components; diagonal 1 + 1/2 sum of omega over
// the adjacent cells (Prop. 3.2 with weights); alpha_d update; q0 as in the
// paper's diagonal 3. The loads of slice t+1 are issued before slice t is
// computed (two slices in flight).
template <typename T, int D>
struct QdSlice {
  double ph;
  double phd[kMaxAxes];  // phi[i + e_d]
  T w[kMaxAxes][4];      // W_{d,v} of the adjacent cells (0 where absent)
  double ad[kMaxAxes];   // alpha_d
  double a0;             // alpha0 of the cell (t < n0)
  double dw;             // w_{K-1} - w_0 of the cell (t < n0)
};

template <typename T, int D>
__device__ __forceinline__ void qd_load(const Geo& g, const Column& c, int t, uint32_t i, gp<const double> phi,
                                        gp<const double> alpha, gp<const T> W, gp<const double> DW,
                                        QdSlice<T, D>& s) {
  const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx;
  const bool has_now = t < g.n[0], has_prev = t >= 1;
  s.ph = phi[i];
  s.a0 = has_now ? alpha[i] : 0.0;
  s.dw = has_now ? DW[i] : 0.0;
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    const bool in = c.x[d] < g.n[d];
    const uint32_t sd = (uint32_t)g.stride[d];
    gp<const T> Wd = W + (size_t)(4 * (d - 1)) * nb;
    s.phd[d] = in ? phi[i + sd] : 0.0;
    s.ad[d] = in ? alpha[(size_t)d * nb + i] : 0.0;
    s.w[d][0] = in && has_now ? Wd[(size_t)0 * nb + i + sd] : T(0);
    s.w[d][1] = in && has_now ? Wd[(size_t)1 * nb + i] : T(0);
    s.w[d][2] = in && has_prev ? Wd[(size_t)2 * nb + i - nx + sd] : T(0);
    s.w[d][3] = in && has_prev ? Wd[(size_t)3 * nb + i - nx] : T(0);
  }
}

// q update of a5 per node (the q-step of Algorithm 2 with the diagonal of
// Prop. 3.2) and the alpha update: q0 and alpha0 at the cell (t < n0) from
// A_0 phi, alpha0 and w_{K-1} - w_0; q_d and alpha_d (d >= 1) from A_d phi,
// alpha_d and the adjacent cells' weighted w components.
template <typename T, int D>
__device__ __forceinline__ void q_body(const Geo& g, const double* __restrict__ phi_, double* __restrict__ alpha_,
                                       const double* __restrict__ om_sp, T* __restrict__ qn_,
                                       const T* __restrict__ W_, const double* __restrict__ DW_,
                                       const Ctl* __restrict__ ctl, uint32_t blk) {
  const Column c = column_of<D>(g, blk);
  if (!c.live) return;
  gp<const double> phi = glob(phi_);
  gp<double> alpha = glob(alpha_);
  gp<T> qn = glob(qn_);
  gp<const T> W = glob(W_);
  gp<const double> DW = glob(DW_);
  gp<const double> om = glob(om_sp);
  const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx;
  const double sigma = glob(ctl)->sigma, tau = glob(ctl)->tau, inv_sigma = 1.0 / sigma;
  double om_a = om[c.xs], om_b[kMaxAxes];
#pragma unroll
  for (int d = 1; d <= D; ++d) om_b[d] = c.x[d] < g.n[d] ? om[c.xs + (uint32_t)g.stride[d]] : 0.0;
  uint32_t i = (uint32_t)c.t0 * nx + c.xs;
  QdSlice<T, D> cur, nxt;
  qd_load<T, D>(g, c, c.t0, i, phi, alpha, W, DW, cur);
  for (int t = c.t0; t < c.t1; ++t, i += nx) {
    const bool more = t + 1 < c.t1;
    if (more) qd_load<T, D>(g, c, t + 1, i + nx, phi, alpha, W, DW, nxt);
    const bool has_now = t < g.n[0];
    const bool has_prev = t >= 1;
    const double ct = (double)has_now + (double)has_prev;
    if (has_now) {
      const double ph1 = more ? nxt.ph : phi[i + nx];
      const double g0 = (ph1 - cur.ph) * g.inv_h[0];
      const double q0n = (g0 + cur.a0 * inv_sigma + cur.dw) * (1.0 / 3.0);
      qn[i] = (T)q0n;
      alpha[i] = cur.a0 + tau * sigma * (g0 - q0n);
    }
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      if (c.x[d] >= g.n[d]) continue;
      double acc = 0.0;
      if (has_now) acc += (double)cur.w[d][0] + (double)cur.w[d][1];
      if (has_prev) acc += (double)cur.w[d][2] + (double)cur.w[d][3];
      const double diag = 1.0 + 0.5 * ct * (om_a + om_b[d]);
      const double gd = (cur.phd[d] - cur.ph) * g.inv_h[d];
      const double ad = cur.ad[d];
      const double qdn = (gd + ad * inv_sigma + acc) / diag;
      qn[(size_t)d * nb + i] = (T)qdn;
      alpha[(size_t)d * nb + i] = ad + tau * sigma * (gd - qdn);
    }
    cur = nxt;
  }
}

// Right-hand side of the phi-step of Algorithm 2 per node, written to the
// transform work plane: b = A^*(q - alpha/sigma) - c/sigma (zero extension
// outside each staggered set) or, with DEFECT, the defect b - A^*A phi of the
// FP64 phi (path-graph Laplacian / h_d^2 per axis, Neumann ends). The time
// neighbours (q0 - alpha0/sigma at t-1, phi at t-1 and t) are carried, and
// the loads of slice t+1 are issued before slice t is computed.
template <typename T, int D>
struct RhsSlice {
  T q0;                     // q0 at the cell t (t < n0)
  double a0;                // alpha0 at the cell t (t < n0)
  T qd[kMaxAxes][2];        // q_d at x - e_d and x
  double ad[kMaxAxes][2];   // alpha_d at x - e_d and x
  double phn;               // phi at t+1 (DEFECT)
  double phs[kMaxAxes][2];  // phi at x - e_d and x + e_d (DEFECT)
  double cb;                // c~ on the boundary slices
};

template <typename T, int D, bool DEFECT>
__device__ __forceinline__ void rhs_load(const Geo& g, const Column& c, int t, uint32_t i, gp<const T> q,
                                         gp<const double> al, gp<const double> phi, const double* c_lo,
                                         const double* c_hi, RhsSlice<T, D>& s) {
  const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx;
  const int n0 = g.n[0];
  s.q0 = t < n0 ? q[i] : T(0);
  s.a0 = t < n0 ? al[i] : 0.0;
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    const uint32_t sd = (uint32_t)g.stride[d];
    gp<const T> qd = q + (size_t)d * nb;
    gp<const double> ad = al + (size_t)d * nb;
    const bool lo = c.x[d] >= 1, hi = c.x[d] < g.n[d];
    s.qd[d][0] = lo ? qd[i - sd] : T(0);
    s.ad[d][0] = lo ? ad[i - sd] : 0.0;
    s.qd[d][1] = hi ? qd[i] : T(0);
    s.ad[d][1] = hi ? ad[i] : 0.0;
    if (DEFECT) {
      s.phs[d][0] = lo ? phi[i - sd] : 0.0;
      s.phs[d][1] = hi ? phi[i + sd] : 0.0;
    }
  }
  if (DEFECT) s.phn = t < n0 ? phi[i + nx] : 0.0;
  s.cb = t == 0 ? glob(c_lo)[c.xs] : (t == n0 ? glob(c_hi)[c.xs] : 0.0);
}

template <typename T, int D, bool DEFECT>
__device__ __forceinline__ void rhs_body(const Geo& g, const T* __restrict__ q_, const double* __restrict__ al_,
                                         const double* __restrict__ phi_, const double* __restrict__ c_lo_,
                                         const double* __restrict__ c_hi_, T* __restrict__ out_, double inv_sigma,
                                         uint32_t blk) {
  const Column c = column_of<D>(g, blk);
  if (!c.live) return;
  gp<const T> q = glob(q_);
  gp<const double> al = glob(al_);
  gp<const double> phi = glob(phi_);
  gp<T> out = glob(out_);
  const uint32_t nx = (uint32_t)g.nx, xs = c.xs;
  const int n0 = g.n[0];
  const double w0 = g.inv_h[0] * g.inv_h[0];
  uint32_t i = (uint32_t)c.t0 * nx + xs;
  double y0m = 0.0, phm = 0.0, ph = 0.0;
  if (c.t0 >= 1) {
    y0m = (double)q[i - nx] - al[i - nx] * inv_sigma;
    if (DEFECT) phm = phi[i - nx];
  }
  if (DEFECT) ph = phi[i];
  RhsSlice<T, D> cur, nxt;
  rhs_load<T, D, DEFECT>(g, c, c.t0, i, q, al, phi, c_lo_, c_hi_, cur);
  for (int t = c.t0; t < c.t1; ++t, i += nx) {
    if (t + 1 < c.t1) rhs_load<T, D, DEFECT>(g, c, t + 1, i + nx, q, al, phi, c_lo_, c_hi_, nxt);
    double b = 0.0;
    if (t >= 1) b += y0m * g.inv_h[0];
    double y0 = 0.0;
    if (t < n0) {
      y0 = (double)cur.q0 - cur.a0 * inv_sigma;
      b -= y0 * g.inv_h[0];
    }
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      if (c.x[d] >= 1) b += ((double)cur.qd[d][0] - cur.ad[d][0] * inv_sigma) * g.inv_h[d];
      if (c.x[d] < g.n[d]) b -= ((double)cur.qd[d][1] - cur.ad[d][1] * inv_sigma) * g.inv_h[d];
    }
    if (t == 0 || t == n0) b -= cur.cb * inv_sigma;
    if (DEFECT) {
      double r = 0.0;
      if (t >= 1) r += (ph - phm) * w0;
      if (t < n0) r -= (cur.phn - ph) * w0;
#pragma unroll
      for (int d = 1; d <= D; ++d) {
        const double wd = g.inv_h[d] * g.inv_h[d];
        if (c.x[d] >= 1) r += (ph - cur.phs[d][0]) * wd;
        if (c.x[d] < g.n[d]) r -= (cur.phs[d][1] - ph) * wd;
      }
      b -= r;
      phm = ph;
      ph = cur.phn;
    }
    out[i] = (T)b;
    y0m = y0;
    cur = nxt;
  }
}

// Block-wide sum of NS doubles in a fixed order (wave shuffles, then LDS
// across waves); the first NS threads write the block's partials, except
// slot `skip`, which another kernel owns.
template <int NS>
__device__ __forceinline__ void wave_sums(double (&s)[NS]) {
  // butterfly over the 64 lanes; the NS sums advance together, so their
  // cross-lane exchanges overlap instead of forming NS serial chains
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] += __shfl_xor(s[k], off, 64);
  }
}

// The partials of an instance are slot-major: slot k of workgroup b at
// partials[k * nsweep + b], so the finalize reads each slot coalesced.
template <int NS>
__device__ __forceinline__ void block_partials(double (&s)[NS], double* __restrict__ partials, uint32_t blk,
                                               uint32_t nsweep, int skip) {
  __shared__ double red[16][NS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  wave_sums<NS>(s);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) red[w][k] = s[k];
  }
  __syncthreads();
  if (threadIdx.x < NS && (int)threadIdx.x != skip) {
    double v = 0.0;
    for (int j = 0; j < nw; ++j) v += red[j][threadIdx.x];
    glob(partials)[(size_t)threadIdx.x * nsweep + blk] = v;
  }
}

// Block sum of one double into partials slot 11.
__device__ __forceinline__ void block_slot11(double v, double* __restrict__ partials, uint32_t blk,
                                             uint32_t nsweep) {
  __shared__ double red1[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) red1[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int j = 0; j < nw; ++j) tot += red1[j];
    glob(partials)[(size_t)11 * nsweep + blk] = tot;
  }
}

// beta update of a5 at one cell: z = Pi(u) from the old q (q0o, F q values
// fa / fb of slices t and t+1) and the old beta bt, then
// beta += tau sigma (z - B F q_new - d) with the new q (q0n, ga / gb) into bn;
// ssq accumulates |z - B F q_new - d|^2.
template <typename T, int D>
__device__ __forceinline__ void beta_cell(const T (&bt)[4 * D + 2], double q0o, const T (&fa)[kMaxAxes][2],
                                          const T (&fb)[kMaxAxes][2], double q0n, const T (&ga)[kMaxAxes][2],
                                          const T (&gb)[kMaxAxes][2], double sw, double sigma, double tau,
                                          double inv_sigma, double& ssq, T (&bn)[4 * D + 2]) {
  constexpr int K = 4 * D + 2;
  double u[K];
  cone_arg<T, D>(bt, q0o, fa, fb, sw, inv_sigma, u);
  soc_project<K>(u);
  auto upd = [&](int k, double bq) {
    const double r = u[k] - bq;
    ssq = fma(r, r, ssq);
    bn[k] = (T)((double)bt[k] + tau * sigma * r);
  };
  upd(0, 1.0 - q0n);
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    const int k = 1 + 4 * (d - 1);
    upd(k + 0, sw * (double)ga[d][0]);
    upd(k + 1, sw * (double)ga[d][1]);
    upd(k + 2, sw * (double)gb[d][0]);
    upd(k + 3, sw * (double)gb[d][1]);
  }
  upd(K - 1, 1.0 + q0n);
}

// beta update of a5 per cell (z recomputed from the old q and beta); at
// residual checks the block sums of |z - B F q_new - d|^2 go to partials
// slot 11. Block 0 counts the iteration.
template <typename T, int D>
__device__ __forceinline__ void beta_body(const Geo& g, const T* __restrict__ q_, const T* __restrict__ qn_,
                                          T* __restrict__ beta_, const double* __restrict__ sw_sp, Ctl* __restrict__ ctl,
                                          double* __restrict__ partials, int check, uint32_t blk) {
  constexpr int K = 4 * D + 2;
  const Column c = column_of<D>(g, blk);
  const int tend = min(c.t1, g.n[0]);
  const double sigma = glob(ctl)->sigma, tau = glob(ctl)->tau, inv_sigma = 1.0 / sigma;
  double ssq = 0.0;
  if (c.live && c.t0 < tend) {
    gp<const T> q = glob(q_);
    gp<const T> qn = glob(qn_);
    gp<T> beta = glob(beta_);
    const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx;
    const double sw = glob(sw_sp)[c.xs];
    uint32_t i = (uint32_t)c.t0 * nx + c.xs;
    T fa[kMaxAxes][2], fb[kMaxAxes][2], ga[kMaxAxes][2], gb[kMaxAxes][2];
    load_fq<T, D>(g, q, i, c, fa);
    load_fq<T, D>(g, qn, i, c, ga);
    for (int t = c.t0; t < tend; ++t, i += nx) {
      load_fq<T, D>(g, q, i + nx, c, fb);
      load_fq<T, D>(g, qn, i + nx, c, gb);
      T bt[K], bn[K];
#pragma unroll
      for (int k = 0; k < K; ++k) bt[k] = beta[(size_t)k * nb + i];
      beta_cell<T, D>(bt, (double)q[i], fa, fb, (double)qn[i], ga, gb, sw, sigma, tau, inv_sigma, ssq, bn);
#pragma unroll
      for (int k = 0; k < K; ++k) beta[(size_t)k * nb + i] = bn[k];
      shift_fq<T, D>(fa, fb);
      shift_fq<T, D>(ga, gb);
    }
  }
  if (check) block_slot11(ssq, partials, blk, g.nsweep);
  if (blk == 0 && threadIdx.x == 0) glob(ctl)->iter += 1;
}

// beta update of one iteration (old q in q_, new q in qn_) and the z-step of
// the next, which reads exactly the new q and the new beta, in one sweep: the
// new beta values and the F q_new values are still in registers when the
// cone argument of the next iteration is formed, so neither is read again.
// Used between iterations without a residual check (sigma is the same for
// both steps). Computes the values of beta_body followed by cone_body.
template <typename T, int D>
__device__ __forceinline__ void beta_cone_body(const Geo& g, const T* __restrict__ q_, const T* __restrict__ qn_,
                                               T* __restrict__ beta_, const double* __restrict__ sw_sp,
                                               T* __restrict__ W_, double* __restrict__ DW_, Ctl* __restrict__ ctl,
                                               uint32_t blk) {
  constexpr int K = 4 * D + 2;
  const Column c = column_of<D>(g, blk);
  const int tend = min(c.t1, g.n[0]);
  const double sigma = glob(ctl)->sigma, tau = glob(ctl)->tau, inv_sigma = 1.0 / sigma;
  if (c.live && c.t0 < tend) {
    gp<const T> q = glob(q_);
    gp<const T> qn = glob(qn_);
    gp<T> beta = glob(beta_);
    gp<T> W = glob(W_);
    gp<double> DW = glob(DW_);
    const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx;
    const double sw = glob(sw_sp)[c.xs];
    uint32_t i = (uint32_t)c.t0 * nx + c.xs;
    T fa[kMaxAxes][2], fb[kMaxAxes][2], ga[kMaxAxes][2], gb[kMaxAxes][2];
    load_fq<T, D>(g, q, i, c, fa);
    load_fq<T, D>(g, qn, i, c, ga);
    double ssq = 0.0;
    for (int t = c.t0; t < tend; ++t, i += nx) {
      load_fq<T, D>(g, q, i + nx, c, fb);
      load_fq<T, D>(g, qn, i + nx, c, gb);
      T bt[K], bn[K];
#pragma unroll
      for (int k = 0; k < K; ++k) bt[k] = beta[(size_t)k * nb + i];
      const double q0n = (double)qn[i];
      beta_cell<T, D>(bt, (double)q[i], fa, fb, q0n, ga, gb, sw, sigma, tau, inv_sigma, ssq, bn);
#pragma unroll
      for (int k = 0; k < K; ++k) beta[(size_t)k * nb + i] = bn[k];
      double u[K];
      cone_arg<T, D>(bn, q0n, ga, gb, sw, inv_sigma, u);
      soc_project<K>(u);
      cone_store<T, D>(u, bn, sw, inv_sigma, W, DW, nb, i);
      shift_fq<T, D>(fa, fb);
      shift_fq<T, D>(ga, gb);
    }
  }
  if (blk == 0 && threadIdx.x == 0) glob(ctl)->iter += 1;
}

// Partial sums for the residuals of Sec. 5.3 at (phi, q, alpha, beta), one
// lane per spatial node over the workgroup's time slices. Slots:
// 0 |A phi - q|^2, 1 |A phi|^2, 2 |q|^2, 3 |A^* alpha + c|^2,
// 5 |alpha0 - max(0, f + alpha0)|^2, 6 |alpha0|^2, 7 |f|^2,
// 8 |alpha_bar - g|^2, 9 |alpha_bar|^2, 10 |g|^2, 13 |F^*B^*beta + alpha|^2,
// 14 |F^*B^*beta|^2, 15 |alpha|^2, 16 <c, phi>, 17 sum m^2 / r over r > 0.
// (4, 11, 12 are filled elsewhere.) Values of node slice t that slice t+1
// needs again (alpha0, phi, q_d on the time node, the cell's last two beta
// components of each axis, alpha0 at x + e_d) are carried, and the loads of
// slice t+1 are issued before slice t is summed.
template <typename T, int D>
struct ResSlice {
  double a0;               // alpha0 at the cell t (t < n0)
  double ad_lo[kMaxAxes];  // alpha_d at x - e_d (x_d >= 1)
  double ad[kMaxAxes];     // alpha_d at x (x_d < n_d)
  double cc;               // c~ on the boundary slices
  double ph1;              // phi at t+1 (t < n0)
  double phd[kMaxAxes];    // phi at x + e_d (x_d < n_d)
  T q0, bK, b0;            // q0, beta_{K-1}, beta_0 at the cell t (t < n0)
  T fq1[kMaxAxes][2];      // q_d at node t+1: x - e_d (x_d >= 1), x (x_d < n_d); t < n0
  T b01[kMaxAxes][2];      // beta_{k}[x + e_d], beta_{k+1}[x] of the cell t (t < n0, x_d < n_d)
  T b23[kMaxAxes][2];      // beta_{k+2}[x + e_d], beta_{k+3}[x] of the cell t (t < n0, x_d < n_d)
  double a0s[kMaxAxes];    // alpha0 at x + e_d of the cell t (t < n0, x_d < n_d)
};

template <typename T, int D>
__device__ __forceinline__ void res_load(const Geo& g, const Column& c, int t, uint32_t i, gp<const double> phi,
                                         gp<const T> q, gp<const double> alpha, gp<const T> beta,
                                         const double* c_lo, const double* c_hi, ResSlice<T, D>& s) {
  constexpr int K = 4 * D + 2;
  const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx;
  const int n0 = g.n[0];
  const bool cell = t < n0;
  s.a0 = cell ? alpha[i] : 0.0;
  s.cc = t == 0 ? glob(c_lo)[c.xs] : (t == n0 ? glob(c_hi)[c.xs] : 0.0);
  s.ph1 = cell ? phi[i + nx] : 0.0;
  s.q0 = cell ? q[i] : T(0);
  s.bK = cell ? beta[(size_t)(K - 1) * nb + i] : T(0);
  s.b0 = cell ? beta[i] : T(0);
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    const uint32_t sd = (uint32_t)g.stride[d];
    const bool lo = c.x[d] >= 1, hi = c.x[d] < g.n[d];
    gp<const double> ad = alpha + (size_t)d * nb;
    gp<const T> qd = q + (size_t)d * nb;
    const int k = 1 + 4 * (d - 1);
    s.ad_lo[d] = lo ? ad[i - sd] : 0.0;
    s.ad[d] = hi ? ad[i] : 0.0;
    s.phd[d] = hi ? phi[i + sd] : 0.0;
    s.fq1[d][0] = cell && lo ? qd[i + nx - sd] : T(0);
    s.fq1[d][1] = cell && hi ? qd[i + nx] : T(0);
    s.b01[d][0] = cell && hi ? beta[(size_t)(k + 0) * nb + i + sd] : T(0);
    s.b01[d][1] = cell && hi ? beta[(size_t)(k + 1) * nb + i] : T(0);
    s.b23[d][0] = cell && hi ? beta[(size_t)(k + 2) * nb + i + sd] : T(0);
    s.b23[d][1] = cell && hi ? beta[(size_t)(k + 3) * nb + i] : T(0);
    s.a0s[d] = cell && hi ? alpha[i + sd] : 0.0;
  }
}

template <typename T, int D>
__device__ __forceinline__ void resid_body(const Geo& g, const double* phi_, const T* q_, const double* alpha_,
                                           const T* beta_, const double* om_sp, const double* sw_sp,
                                           const double* c_lo_, const double* c_hi_, double* __restrict__ partials,
                                           uint32_t blk) {
  double s[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) s[k] = 0.0;
  const Column c = column_of<D>(g, blk);
  if (c.live) {
    gp<const double> phi = glob(phi_);
    gp<const T> q = glob(q_);
    gp<const double> alpha = glob(alpha_);
    gp<const T> beta = glob(beta_);
    gp<const double> om = glob(om_sp);
    gp<const double> swp = glob(sw_sp);
    const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx, xs = c.xs;
    const int n0 = g.n[0];
    const double oma = om[xs], swa = swp[xs];
    double omb[kMaxAxes], swb[kMaxAxes];
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      const bool in = c.x[d] < g.n[d];
      omb[d] = in ? om[xs + (uint32_t)g.stride[d]] : 0.0;
      swb[d] = in ? swp[xs + (uint32_t)g.stride[d]] : 0.0;
    }
    uint32_t i = (uint32_t)c.t0 * nx + xs;
    // carried values of node slice t: alpha0 at t-1, phi at t, q_d at node t,
    // the last two beta components of cell t-1, alpha0 at x + e_d of cell t-1
    double a0p = 0.0, ph = phi[i];
    T fq0[kMaxAxes][2], b23p[kMaxAxes][2];
    double a0sp[kMaxAxes];
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      const uint32_t sd = (uint32_t)g.stride[d];
      const bool lo = c.x[d] >= 1, hi = c.x[d] < g.n[d];
      gp<const T> qd = q + (size_t)d * nb;
      const int k = 1 + 4 * (d - 1);
      fq0[d][0] = lo ? qd[i - sd] : T(0);
      fq0[d][1] = hi ? qd[i] : T(0);
      const bool prev = c.t0 >= 1 && hi;
      b23p[d][0] = prev ? beta[(size_t)(k + 2) * nb + i - nx + sd] : T(0);
      b23p[d][1] = prev ? beta[(size_t)(k + 3) * nb + i - nx] : T(0);
      a0sp[d] = prev ? alpha[i - nx + sd] : 0.0;
    }
    if (c.t0 >= 1) a0p = alpha[i - nx];
    ResSlice<T, D> cur, nxt;
    res_load<T, D>(g, c, c.t0, i, phi, q, alpha, beta, c_lo_, c_hi_, cur);
    for (int t = c.t0; t < c.t1; ++t, i += nx) {
      if (t + 1 < c.t1) res_load<T, D>(g, c, t + 1, i + nx, phi, q, alpha, beta, c_lo_, c_hi_, nxt);
      // divergence residual at the node
      double div = 0.0;
      if (t >= 1) div += a0p * g.inv_h[0];
      if (t < n0) div -= cur.a0 * g.inv_h[0];
#pragma unroll
      for (int d = 1; d <= D; ++d) {
        if (c.x[d] >= 1) div += cur.ad_lo[d] * g.inv_h[d];
        if (c.x[d] < g.n[d]) div -= cur.ad[d] * g.inv_h[d];
      }
      div += cur.cc;
      s[3] += div * div;
      s[16] += cur.cc * ph;
      if (t < n0) {
        // q0, alpha0 at the cell
        const double g0 = (cur.ph1 - ph) * g.inv_h[0];
        const double q0 = (double)cur.q0, a0 = cur.a0;
        s[0] += (g0 - q0) * (g0 - q0);
        s[1] += g0 * g0;
        s[2] += q0 * q0;
        const double fb = (double)cur.bK - (double)cur.b0;
        s[13] += (fb + a0) * (fb + a0);
        s[14] += fb * fb;
        s[15] += a0 * a0;
        // f(q) = q0 + omega/8 sum_{d,v} (F^d_v q_d)^2
        double sq = 0.0;
#pragma unroll
        for (int d = 1; d <= D; ++d) {
          if (c.x[d] >= 1) {
            const double f1 = (double)fq0[d][0], f3 = (double)cur.fq1[d][0];
            sq += f1 * f1 + f3 * f3;
          }
          if (c.x[d] < g.n[d]) {
            const double f2 = (double)fq0[d][1], f4 = (double)cur.fq1[d][1];
            sq += f2 * f2 + f4 * f4;
          }
        }
        const double f = q0 + 0.125 * oma * sq;
        const double cr = a0 - fmax(0.0, f + a0);
        s[5] += cr * cr;
        s[6] += a0 * a0;
        s[7] += f * f;
      }
#pragma unroll
      for (int d = 1; d <= D; ++d) {
        if (c.x[d] >= g.n[d]) continue;
        const double gd = (cur.phd[d] - ph) * g.inv_h[d];
        const double qd = (double)fq0[d][1];
        const double ad = cur.ad[d];
        s[0] += (gd - qd) * (gd - qd);
        s[1] += gd * gd;
        s[2] += qd * qd;
        s[15] += ad * ad;
        // F^*B^* beta at this point, and r_d = L_X^d L_T^*(omega alpha0)
        double fb = 0.0, r = 0.0;
        if (t < n0) {
          fb += swb[d] * (double)cur.b01[d][0] + swa * (double)cur.b01[d][1];
          r += omb[d] * cur.a0s[d] + oma * cur.a0;
        }
        if (t >= 1) {
          fb += swb[d] * (double)b23p[d][0] + swa * (double)b23p[d][1];
          r += omb[d] * a0sp[d] + oma * a0p;
        }
        r *= 0.25;
        s[13] += (fb + ad) * (fb + ad);
        s[14] += fb * fb;
        const double gg = r * qd;
        s[8] += (ad - gg) * (ad - gg);
        s[9] += ad * ad;
        s[10] += gg * gg;
        if (r > 0.0) s[17] += ad * ad / r;
      }
      // carry to slice t+1
      a0p = cur.a0;
      ph = cur.ph1;
#pragma unroll
      for (int d = 1; d <= D; ++d) {
        fq0[d][0] = cur.fq1[d][0];
        fq0[d][1] = cur.fq1[d][1];
        b23p[d][0] = cur.b23[d][0];
        b23p[d][1] = cur.b23[d][1];
        a0sp[d] = cur.a0s[d];
      }
      cur = nxt;
    }
  }
  block_partials<kNumSums>(s, partials, blk, g.nsweep, 11);
}

// Scalars the finalize step needs besides the partials.
struct FinArgs {
  double vol;      // h0 h1 ... hD
  double c_norm2;  // sum c~^2
  double d_norm2;  // sum d^2 = 2 * number of cells
  int64_t nblocks;
  int32_t staged;  // the partials are reduced in two stages (nblocks >= kFinStageMinRows)
};

// The workgroup partials of a large instance are reduced in two stages:
// kFinChunks workgroups each sum a contiguous range of the rows into one
// stage row (one workgroup alone is bound by how many loads one CU keeps in
// flight: 8,547 rows took 35 us, 36,945 rows 133 us), then the finalize block
// sums the stage rows. The stage rows follow the partial rows: slot k of
// stage row c at partials[kNumSums * nblocks + k * kFinChunks + c]. Below
// kFinStageMinRows rows the finalize block sums the rows itself (the extra
// launch cost more than it saved there).
constexpr int kFinChunks = 64;
constexpr int64_t kFinStageMinRows = 8192;

__device__ __forceinline__ double* fin_stage_rows(const FinArgs& fa, double* partials) {
  return partials + (size_t)kNumSums * (size_t)fa.nblocks;
}

// First stage: rows [n c / kFinChunks, n (c + 1) / kFinChunks) of every slot,
// each thread adding its rows in order, then the wave and block sums.
__device__ __forceinline__ void fin_stage_body(const FinArgs& fa, double* __restrict__ partials, int chunk) {
  const int64_t n = fa.nblocks;
  const int64_t r0 = n * chunk / kFinChunks, r1 = n * (chunk + 1) / kFinChunks;
  gp<const double> pr = glob(partials);
  double v[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) v[k] = 0.0;
  for (int64_t j = r0 + threadIdx.x; j < r1; j += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) v[k] += pr[k * n + j];
  }
  block_partials<kNumSums>(v, fin_stage_rows(fa, partials), (uint32_t)chunk, (uint32_t)kFinChunks, -1);
}

__device__ __forceinline__ double eta_ratio(double num2, double a2, double b2, double vol) {
  return sqrt(vol * num2) / (1.0 + sqrt(vol * a2) + sqrt(vol * b2));
}

// Sums the block partials (their stage rows when staged) in a fixed order,
// forms the residuals, applies the sigma rule of Sec. 5.3 on its schedule and
// sets the stop flag. One block per instance, after fin_stage_body.
__device__ __forceinline__ void finalize_body(const FinArgs& fa, const double* __restrict__ partials,
                                              Ctl* __restrict__ ctl, int update_ctl) {
  __shared__ double acc[1024 / 64][kNumSums];
  __shared__ double tot[kNumSums];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // thread 0 requests the control block first, so that its latency overlaps
  // the partial sums
  CtlState c;
  if (threadIdx.x == 0) c = *static_cast<const CtlState*>(ctl);
  // one pass over the stage rows (or the workgroup rows): each thread sums
  // every slot of its rows (slot-major, read coalesced), then the slots are
  // reduced across the block; waves past the last row hold zeros and skip the
  // cross-lane sums
  const int64_t rows = fa.staged ? kFinChunks : fa.nblocks;
  gp<const double> pr = glob(fa.staged ? fin_stage_rows(fa, const_cast<double*>(partials)) : partials);
  double v[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) v[k] = 0.0;
  for (int64_t j = threadIdx.x; j < rows; j += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) v[k] += pr[k * rows + j];
  }
  if ((int64_t)w * 64 < rows) wave_sums<kNumSums>(v);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) acc[w][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < kNumSums) {
    double v = 0.0;
    for (int j = 0; j < nw; ++j) v += acc[j][threadIdx.x];
    tot[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (update_ctl && c.stop) return;  // a stopped instance keeps its last check
  const double vol = fa.vol;
  const double eta_p = eta_ratio(tot[0], tot[1], tot[2], vol);
  const double eta_d = sqrt(vol * tot[3]) / (1.0 + sqrt(vol * fa.c_norm2));
  const double c1 = eta_ratio(tot[5], tot[6], tot[7], vol);
  const double c2 = eta_ratio(tot[8], tot[9], tot[10], vol);
  const double eta_c = fmax(c1, c2);
  const double eta_dot = fmax(eta_p, fmax(eta_d, eta_c));
  const double p2 = sqrt(vol * tot[11]) / (1.0 + sqrt(vol * fa.d_norm2));
  const double d2 = eta_ratio(tot[13], tot[14], tot[15], vol);
  const double eps = fmax(eta_p, p2), eds = fmax(eta_d, d2);
  // the register copy of the control block is stored back once
  c.eta[0] = eta_dot;
  c.eta[1] = eta_p;
  c.eta[2] = eta_d;
  c.eta[3] = eta_c;
  c.eta[4] = eps;
  c.eta[5] = eds;
  c.eta[6] = c1;
  c.eta[7] = c2;
  c.objective = -vol * tot[16];
  c.dual_objective = 0.5 * vol * tot[17];
  if (update_ctl) {
    c.checks += 1;
    if (!(eta_dot == eta_dot) || isinf(eta_dot)) {
      c.stop = 3;
    } else if (eta_dot <= c.tol) {
      c.stop = 1;
    } else {
      if (c.adapt && c.iter >= c.next_update) {
        const double ratio = eds > 0.0 ? eps / eds : INFINITY;
        const int changes = c.sigma_changes;
        if (ratio > 2.0) {
          c.sigma *= 1.25;
          c.sigma_changes += 1;
        } else if (ratio < 0.5) {
          c.sigma /= 1.25;
          c.sigma_changes += 1;
        }
        if (c.sigma_changes != changes) {
          ctl->hist_sigma[changes % kSigmaHist] = c.sigma;
          ctl->hist_iter[changes % kSigmaHist] = c.iter;
        }
        while (c.next_update <= c.iter) {
          const int nxt = (int)floor(c.growth * (double)c.gap) + c.cadence;
          c.gap = nxt - nxt % c.cadence;
          c.next_update += c.gap;
        }
      }
      if (c.iter >= c.iter_limit) c.stop = 2;
    }
  }
  *static_cast<CtlState*>(ctl) = c;
}

// ---- standalone step kernels (step-level entry points) --------------------

template <typename T, int D>
__device__ __forceinline__ void cone_out_body(const Geo& g, const T* __restrict__ q, const T* __restrict__ beta,
                                              const double* __restrict__ sw_sp, double inv_sigma, T* __restrict__ z,
                                              int64_t blk) {
  constexpr int K = 4 * D + 2;
  const int64_t i = blk * blockDim.x + threadIdx.x;
  if (i >= g.nb) return;
  const int64_t nb = g.nb;
  if (i >= (int64_t)g.n[0] * g.stride[0]) {
#pragma unroll
    for (int k = 0; k < K; ++k) z[k * nb + i] = T(0);
    return;
  }
  int x[kMaxAxes];
  node_coords<D>(g, i, x);
  double u[K];
  cone_input<T, D>(g, q, beta, i, x, sw_sp[i % g.nx], inv_sigma, u);
  soc_project<K>(u);
#pragma unroll
  for (int k = 0; k < K; ++k) z[k * nb + i] = (T)u[k];
}

// |z - B F q - d|^2 block sums into partials slot 11 (z given), over the
// same workgroups as the residual sweep.
template <typename T, int D>
__device__ __forceinline__ void zres_body(const Geo& g, const T* z_, const T* q_, const double* sw_sp,
                                          double* __restrict__ partials, uint32_t blk) {
  constexpr int K = 4 * D + 2;
  const Column c = column_of<D>(g, blk);
  const int tend = min(c.t1, g.n[0]);
  double ssq = 0.0;
  if (c.live) {
    gp<const T> z = glob(z_);
    gp<const T> q = glob(q_);
    const uint32_t nb = (uint32_t)g.nb, nx = (uint32_t)g.nx;
    const double sw = glob(sw_sp)[c.xs];
    uint32_t i = (uint32_t)c.t0 * nx + c.xs;
    for (int t = c.t0; t < tend; ++t, i += nx) {
      T fa[kMaxAxes][2], fb[kMaxAxes][2];
      load_fq<T, D>(g, q, i, c, fa);
      load_fq<T, D>(g, q, i + nx, c, fb);
      const double q0 = (double)q[i];
      const double r0 = (double)z[i] - (1.0 - q0);
      const double rl = (double)z[(size_t)(K - 1) * nb + i] - (1.0 + q0);
      ssq += r0 * r0 + rl * rl;
#pragma unroll
      for (int d = 1; d <= D; ++d) {
        const int k = 1 + 4 * (d - 1);
        const double f[4] = {(double)fa[d][0], (double)fa[d][1], (double)fb[d][0], (double)fb[d][1]};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double r = (double)z[(size_t)(k + v) * nb + i] - sw * f[v];
          ssq += r * r;
        }
      }
    }
  }
  block_slot11(ssq, partials, blk, g.nsweep);
}

}  // namespace dot
