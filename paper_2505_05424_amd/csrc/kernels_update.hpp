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

// ---------------------------------------------------------------------------
// a1 + a2 + q0 part of a5: per cell, z = Pi(u); w = z - d + beta/sigma;
// q0_new = (A_0 phi + alpha0/sigma + w_{K-1} - w_0) / 3 and alpha0 update;
// the weighted components sqrt(omega/2) w_{d,v} go to W for the q_d update.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void cone_q0_body(const Geo& g, const double* __restrict__ phi, const T* __restrict__ q,
                                             T* __restrict__ alpha, const T* __restrict__ beta,
                                             const double* __restrict__ sw_sp, T* __restrict__ qn, T* __restrict__ W,
                                             const Ctl* __restrict__ ctl, int64_t blk) {
  constexpr int K = 4 * D + 2;
  const int64_t i = blk * blockDim.x + threadIdx.x;
  const int64_t ncell = (int64_t)g.n[0] * g.stride[0];
  if (i >= ncell) return;
  const double sigma = ctl->sigma, tau = ctl->tau, inv_sigma = 1.0 / sigma;
  int x[kMaxAxes];
  node_coords<D>(g, i, x);
  const int64_t xs = i % g.nx;
  const double sw = sw_sp[xs];
  double u[K];
  cone_input<T, D>(g, q, beta, i, x, sw, inv_sigma, u);
  soc_project<K>(u);
  const int64_t nb = g.nb;
  // w = z - d + beta/sigma
  const double w0 = u[0] - 1.0 + (double)beta[i] * inv_sigma;
  const double wl = u[K - 1] - 1.0 + (double)beta[(K - 1) * nb + i] * inv_sigma;
  const double g0 = ((double)phi[i + g.stride[0]] - (double)phi[i]) * g.inv_h[0];
  const double a0 = (double)alpha[i];
  const double q0n = (g0 + a0 * inv_sigma + wl - w0) * (1.0 / 3.0);
  qn[i] = (T)q0n;
  alpha[i] = (T)(a0 + tau * sigma * (g0 - q0n));
#pragma unroll
  for (int k = 1; k < K - 1; ++k) {
    const double wk = u[k] + (double)beta[k * nb + i] * inv_sigma;
    W[(k - 1) * nb + i] = (T)(sw * wk);
  }
}

// q_d update (d >= 1) of a5 per node: rhs = A_d phi + alpha_d/sigma + the four
// adjacent cells' weighted w components; diagonal 1 + 1/2 sum of omega over
// the adjacent cells (Prop. 3.2 with weights); alpha_d update.
template <typename T, int D>
__device__ __forceinline__ void qd_body(const Geo& g, const double* __restrict__ phi, T* __restrict__ alpha,
                                        const double* __restrict__ om_sp, T* __restrict__ qn, const T* __restrict__ W,
                                        const Ctl* __restrict__ ctl, int64_t blk) {
  const int64_t i = blk * blockDim.x + threadIdx.x;
  if (i >= g.nb) return;
  const double sigma = ctl->sigma, tau = ctl->tau, inv_sigma = 1.0 / sigma;
  int x[kMaxAxes];
  node_coords<D>(g, i, x);
  const int64_t nb = g.nb, s0 = g.stride[0];
  const int64_t xs = i % g.nx;
  const int t = x[0];
  const bool has_now = t < g.n[0];
  const bool has_prev = t >= 1;
  const double ct = (double)has_now + (double)has_prev;
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    if (x[d] >= g.n[d]) continue;
    const int64_t sd = g.stride[d];
    const T* Wd = W + (int64_t)(4 * (d - 1)) * nb;
    double acc = 0.0;
    if (has_now) acc += (double)Wd[0 * nb + i + sd] + (double)Wd[1 * nb + i];
    if (has_prev) acc += (double)Wd[2 * nb + i - s0 + sd] + (double)Wd[3 * nb + i - s0];
    const double diag = 1.0 + 0.5 * ct * (om_sp[xs] + om_sp[xs + sd]);
    const double gd = ((double)phi[i + sd] - (double)phi[i]) * g.inv_h[d];
    const double ad = (double)alpha[d * nb + i];
    const double qdn = (gd + ad * inv_sigma + acc) / diag;
    qn[d * nb + i] = (T)qdn;
    alpha[d * nb + i] = (T)(ad + tau * sigma * (gd - qdn));
  }
}

// Block-wide sum of NS doubles in a fixed order (wave shuffles, then LDS
// across waves); the first NS threads write the block's partials, except
// slot `skip`, which another kernel owns.
template <int NS>
__device__ __forceinline__ void block_partials(double (&s)[NS], double* __restrict__ out_block, int skip) {
  __shared__ double red[16][NS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double v = s[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[w][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < NS && (int)threadIdx.x != skip) {
    double v = 0.0;
    for (int j = 0; j < nw; ++j) v += red[j][threadIdx.x];
    out_block[threadIdx.x] = v;
  }
}

// beta update of a5 per cell: z recomputed from the old (q, beta),
// beta += tau sigma (z - B F q_new - d); at residual checks the block sums of
// |z - B F q_new - d|^2 go to partials slot 11. Block 0 counts the iteration.
template <typename T, int D>
__device__ __forceinline__ void beta_body(const Geo& g, const T* __restrict__ q, const T* __restrict__ qn,
                                          T* __restrict__ beta, const double* __restrict__ sw_sp,
                                          Ctl* __restrict__ ctl, double* __restrict__ partials, int check,
                                          int64_t blk) {
  constexpr int K = 4 * D + 2;
  const int64_t i = blk * blockDim.x + threadIdx.x;
  const int64_t ncell = (int64_t)g.n[0] * g.stride[0];
  const double sigma = ctl->sigma, tau = ctl->tau, inv_sigma = 1.0 / sigma;
  double ssq = 0.0;
  if (i < ncell) {
    int x[kMaxAxes];
    node_coords<D>(g, i, x);
    const double sw = sw_sp[i % g.nx];
    double u[K];
    cone_input<T, D>(g, q, beta, i, x, sw, inv_sigma, u);
    soc_project<K>(u);
    // B F q_new + d
    double bq[K];
    const int64_t nb = g.nb;
    const double q0 = (double)qn[i];
    bq[0] = 1.0 - q0;
    bq[K - 1] = 1.0 + q0;
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      const T* qd = qn + d * nb;
      const bool lo = x[d] >= 1, hi = x[d] < g.n[d];
      const int64_t sd = g.stride[d], s0 = g.stride[0];
      const int k = 1 + 4 * (d - 1);
      bq[k + 0] = lo ? sw * (double)qd[i - sd] : 0.0;
      bq[k + 1] = hi ? sw * (double)qd[i] : 0.0;
      bq[k + 2] = lo ? sw * (double)qd[i + s0 - sd] : 0.0;
      bq[k + 3] = hi ? sw * (double)qd[i + s0] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double r = u[k] - bq[k];
      ssq = fma(r, r, ssq);
      beta[k * nb + i] = (T)((double)beta[k * nb + i] + tau * sigma * r);
    }
  }
  if (check) {
    double s[1] = {ssq};
    __shared__ double red1[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double v = s[0];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red1[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int j = 0; j < nw; ++j) tot += red1[j];
      partials[blk * kNumSums + 11] = tot;
    }
  }
  if (blk == 0 && threadIdx.x == 0) ctl->iter += 1;
}

// Partial sums for the residuals of Sec. 5.3 at (phi, q, alpha, beta), one
// lane per node. Slots: 0 |A phi - q|^2, 1 |A phi|^2, 2 |q|^2,
// 3 |A^* alpha + c|^2, 5 |alpha0 - max(0, f + alpha0)|^2, 6 |alpha0|^2,
// 7 |f|^2, 8 |alpha_bar - g|^2, 9 |alpha_bar|^2, 10 |g|^2,
// 13 |F^*B^*beta + alpha|^2, 14 |F^*B^*beta|^2, 15 |alpha|^2, 16 <c, phi>,
// 17 sum m^2 / r over r > 0. (4, 11, 12 are filled elsewhere.)
template <typename T, int D>
__device__ __forceinline__ void resid_body(const Geo& g, const double* __restrict__ phi, const T* __restrict__ q,
                                           const T* __restrict__ alpha, const T* __restrict__ beta,
                                           const double* __restrict__ om_sp, const double* __restrict__ sw_sp,
                                           const double* __restrict__ c_lo, const double* __restrict__ c_hi,
                                           double* __restrict__ partials, int64_t blk) {
  constexpr int K = 4 * D + 2;
  double s[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) s[k] = 0.0;
  const int64_t i = blk * blockDim.x + threadIdx.x;
  if (i < g.nb) {
    int x[kMaxAxes];
    node_coords<D>(g, i, x);
    const int64_t nb = g.nb, s0 = g.stride[0];
    const int64_t xs = i % g.nx;
    const int t = x[0];
    const int n0 = g.n[0];
    // divergence residual at the node
    double div = 0.0;
    if (t >= 1) div += (double)alpha[i - s0] * g.inv_h[0];
    if (t < n0) div -= (double)alpha[i] * g.inv_h[0];
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      const T* ad = alpha + d * nb;
      if (x[d] >= 1) div += (double)ad[i - g.stride[d]] * g.inv_h[d];
      if (x[d] < g.n[d]) div -= (double)ad[i] * g.inv_h[d];
    }
    double cc = 0.0;
    if (t == 0) cc = c_lo[xs];
    if (t == n0) cc = c_hi[xs];
    div += cc;
    s[3] += div * div;
    s[16] += cc * (double)phi[i];
    if (t < n0) {
      // q0, alpha0 at the cell
      const double g0 = ((double)phi[i + s0] - (double)phi[i]) * g.inv_h[0];
      const double q0 = (double)q[i], a0 = (double)alpha[i];
      s[0] += (g0 - q0) * (g0 - q0);
      s[1] += g0 * g0;
      s[2] += q0 * q0;
      const double fb = (double)beta[(K - 1) * nb + i] - (double)beta[i];
      s[13] += (fb + a0) * (fb + a0);
      s[14] += fb * fb;
      s[15] += a0 * a0;
      // f(q) = q0 + omega/8 sum_{d,v} (F^d_v q_d)^2
      double sq = 0.0;
#pragma unroll
      for (int d = 1; d <= D; ++d) {
        const T* qd = q + d * nb;
        const int64_t sd = g.stride[d];
        if (x[d] >= 1) {
          const double f1 = (double)qd[i - sd], f3 = (double)qd[i + s0 - sd];
          sq += f1 * f1 + f3 * f3;
        }
        if (x[d] < g.n[d]) {
          const double f2 = (double)qd[i], f4 = (double)qd[i + s0];
          sq += f2 * f2 + f4 * f4;
        }
      }
      const double f = q0 + 0.125 * om_sp[xs] * sq;
      const double cr = a0 - fmax(0.0, f + a0);
      s[5] += cr * cr;
      s[6] += a0 * a0;
      s[7] += f * f;
    }
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      if (x[d] >= g.n[d]) continue;
      const int64_t sd = g.stride[d];
      const double gd = ((double)phi[i + sd] - (double)phi[i]) * g.inv_h[d];
      const double qd = (double)q[d * nb + i];
      const double ad = (double)alpha[d * nb + i];
      s[0] += (gd - qd) * (gd - qd);
      s[1] += gd * gd;
      s[2] += qd * qd;
      s[15] += ad * ad;
      // F^*B^* beta at this point, and r_d = L_X^d L_T^*(omega alpha0)
      const int k = 1 + 4 * (d - 1);
      const double swa = sw_sp[xs], swb = sw_sp[xs + sd];
      const double oma = om_sp[xs], omb = om_sp[xs + sd];
      double fb = 0.0, r = 0.0;
      if (t < n0) {
        fb += swb * (double)beta[(k + 0) * nb + i + sd] + swa * (double)beta[(k + 1) * nb + i];
        r += omb * (double)alpha[i + sd] + oma * (double)alpha[i];
      }
      if (t >= 1) {
        fb += swb * (double)beta[(k + 2) * nb + i - s0 + sd] + swa * (double)beta[(k + 3) * nb + i - s0];
        r += omb * (double)alpha[i - s0 + sd] + oma * (double)alpha[i - s0];
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
  }
  block_partials<kNumSums>(s, partials + blk * kNumSums, 11);
}

// Scalars the finalize step needs besides the partials.
struct FinArgs {
  double vol;      // h0 h1 ... hD
  double c_norm2;  // sum c~^2
  double d_norm2;  // sum d^2 = 2 * number of cells
  int64_t nblocks;
};

__device__ __forceinline__ double eta_ratio(double num2, double a2, double b2, double vol) {
  return sqrt(vol * num2) / (1.0 + sqrt(vol * a2) + sqrt(vol * b2));
}

// Sums the block partials in a fixed order, forms the residuals, applies the
// sigma rule of Sec. 5.3 on its schedule and sets the stop flag. One block
// per instance.
__device__ __forceinline__ void finalize_body(const FinArgs& fa, const double* __restrict__ partials,
                                              Ctl* __restrict__ ctl, int update_ctl) {
  __shared__ double acc[1024 / 64][kNumSums];
  __shared__ double tot[kNumSums];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = 0; k < kNumSums; ++k) {
    double v = 0.0;
    for (int64_t j = threadIdx.x; j < fa.nblocks; j += blockDim.x) v += partials[j * kNumSums + k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) acc[w][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNumSums) {
    double v = 0.0;
    for (int j = 0; j < nw; ++j) v += acc[j][threadIdx.x];
    tot[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
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
  ctl->eta[0] = eta_dot;
  ctl->eta[1] = eta_p;
  ctl->eta[2] = eta_d;
  ctl->eta[3] = eta_c;
  ctl->eta[4] = eps;
  ctl->eta[5] = eds;
  ctl->eta[6] = c1;
  ctl->eta[7] = c2;
  ctl->objective = -vol * tot[16];
  ctl->dual_objective = 0.5 * vol * tot[17];
  if (!update_ctl) return;
  ctl->checks += 1;
  if (!(eta_dot == eta_dot) || isinf(eta_dot)) {
    ctl->stop = 3;
    return;
  }
  if (eta_dot <= ctl->tol) {
    ctl->stop = 1;
    return;
  }
  if (ctl->adapt && ctl->iter >= ctl->next_update) {
    const double ratio = eds > 0.0 ? eps / eds : INFINITY;
    if (ratio > 2.0) {
      ctl->sigma *= 1.25;
      ctl->sigma_changes += 1;
    } else if (ratio < 0.5) {
      ctl->sigma /= 1.25;
      ctl->sigma_changes += 1;
    }
    while (ctl->next_update <= ctl->iter) {
      const int nxt = (int)floor(ctl->growth * (double)ctl->gap) + ctl->cadence;
      ctl->gap = nxt - nxt % ctl->cadence;
      ctl->next_update += ctl->gap;
    }
  }
  if (ctl->iter >= ctl->iter_limit) ctl->stop = 2;
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

// |z - B F q - d|^2 block sums into partials slot 11 (z given).
template <typename T, int D>
__device__ __forceinline__ void zres_body(const Geo& g, const T* __restrict__ z, const T* __restrict__ q,
                                          const double* __restrict__ sw_sp, double* __restrict__ partials,
                                          int64_t blk) {
  constexpr int K = 4 * D + 2;
  const int64_t i = blk * blockDim.x + threadIdx.x;
  double ssq = 0.0;
  if (i < (int64_t)g.n[0] * g.stride[0]) {
    int x[kMaxAxes];
    node_coords<D>(g, i, x);
    const int64_t nb = g.nb;
    const double sw = sw_sp[i % g.nx];
    const double q0 = (double)q[i];
    double r0 = (double)z[i] - (1.0 - q0);
    double rl = (double)z[(K - 1) * nb + i] - (1.0 + q0);
    ssq = r0 * r0 + rl * rl;
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      const T* qd = q + d * nb;
      const bool lo = x[d] >= 1, hi = x[d] < g.n[d];
      const int64_t sd = g.stride[d], s0 = g.stride[0];
      const int k = 1 + 4 * (d - 1);
      const double f[4] = {lo ? (double)qd[i - sd] : 0.0, hi ? (double)qd[i] : 0.0,
                           lo ? (double)qd[i + s0 - sd] : 0.0, hi ? (double)qd[i + s0] : 0.0};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double r = (double)z[(k + v) * nb + i] - sw * f[v];
        ssq += r * r;
      }
    }
  }
  double s[1] = {ssq};
  __shared__ double red1[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double v = s[0];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) red1[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int j = 0; j < nw; ++j) tot += red1[j];
    partials[blk * kNumSums + 11] = tot;
  }
}

}  // namespace dot
