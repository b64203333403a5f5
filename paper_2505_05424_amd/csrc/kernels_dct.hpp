// Cosine-transform passes of the space-time Poisson solve (Sec. 4, the
// phi-step of Algorithm 2): A^*A is the sum over axes of path-graph Laplacians / h_d^2, whose
// eigenvectors are the orthonormal DCT-II basis of length N_d = n_d + 1.
//
// One pass transforms every line of one axis. A workgroup stages a tile of
// kCW lines x L points in LDS (one line per lane), folds each line into its
// symmetric and antisymmetric halves (x_j +- x_{L-1-j}), and multiplies the
// halves by the even-row and odd-row halves of the transform matrix with
// register blocks of kR outputs per lane. The matrix rows are the same for
// all lanes of a wave, so they are read as wave-uniform (scalar) loads.
// Passes work in place: a tile holds whole lines, so each workgroup reads and
// writes only its own elements.
#pragma once
#include "geometry.hpp"

namespace dot {

constexpr int kCW = 64;       // lines per tile (one per lane)
constexpr int kR = 16;        // outputs per register block
constexpr int kDctWaves = 8;  // waves per workgroup
constexpr int kMaxBlk = 3;    // register blocks per wave

// Folded transform tables of one axis (device pointers).
//   fe[j][k'] = C[2k'][j]   (j < ne inputs: u_0..u_{M-1}, then the middle point if L odd)
//   fo[j][k'] = C[2k'+1][j] (j < M inputs v_j)
//   ie[k'][j] = C[2k'][j]   (k' < ne inputs X_{2k'}, j < ne outputs E_j)
//   io[k'][j] = C[2k'+1][j] (k' < M inputs X_{2k'+1}, j < M outputs O_j)
// C[k][j] = s_k cos(pi k (2j+1) / (2L)), s_0 = sqrt(1/L), s_k = sqrt(2/L).
// Rows are padded with zeros to ne_pad / no_pad columns (multiples of kR).
template <typename T>
struct AxisTab {
  const T* fe;
  const T* fo;
  const T* ie;
  const T* io;
  int L, M, ne, no, ne_pad, no_pad;
};

enum PassKind { kFwd = 0, kInv = 1, kFwdScaleInv = 2 };
enum PassSrc { kSrcPlane = 0, kSrcDivergence = 1 };

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Multiply the folded halves held in the tile by the tables of one direction.
// even_in(j) / odd_in(j) map an input index to its tile slot. Results stay in
// registers: res[b][r] is output (blk*kR + r) of the b-th block of this wave.
template <typename T, typename EvenSlot, typename OddSlot>
__device__ __forceinline__ void dct_blocks(const T* __restrict__ tile, const T* __restrict__ te,
                                           const T* __restrict__ to, int n_even_in, int n_odd_in,
                                           int ne_pad, int no_pad, EvenSlot even_in, OddSlot odd_in,
                                           T (&res)[kMaxBlk][kR]) {
  const int lane = threadIdx.x & 63;
  const int w = wave_id();
  const int nwaves = blockDim.x >> 6;
  const int nbe = ne_pad / kR;
  const int nbt = nbe + no_pad / kR;
#pragma unroll
  for (int b = 0; b < kMaxBlk; ++b) {
    const int blk = w + b * nwaves;
    T acc[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) acc[r] = T(0);
    if (blk < nbe) {
      const T* col0 = te + blk * kR;
      for (int j = 0; j < n_even_in; ++j) {
        const T xv = tile[even_in(j) * (kCW + 1) + lane];
        const T* c = col0 + (size_t)j * ne_pad;
#pragma unroll
        for (int r = 0; r < kR; ++r) acc[r] = fma(c[r], xv, acc[r]);
      }
    } else if (blk < nbt) {
      const T* col0 = to + (blk - nbe) * kR;
      for (int j = 0; j < n_odd_in; ++j) {
        const T xv = tile[odd_in(j) * (kCW + 1) + lane];
        const T* c = col0 + (size_t)j * no_pad;
#pragma unroll
        for (int r = 0; r < kR; ++r) acc[r] = fma(c[r], xv, acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) res[b][r] = acc[r];
  }
}

// Write the register results of dct_blocks to tile slots: even output k' of
// the even half goes to slot even_out(k'), odd output to odd_out(k').
template <typename T, typename EvenOut, typename OddOut>
__device__ __forceinline__ void dct_store(T* __restrict__ tile, int ne, int no, int ne_pad, int no_pad,
                                          EvenOut even_out, OddOut odd_out, const T (&res)[kMaxBlk][kR]) {
  const int lane = threadIdx.x & 63;
  const int w = wave_id();
  const int nwaves = blockDim.x >> 6;
  const int nbe = ne_pad / kR;
  const int nbt = nbe + no_pad / kR;
#pragma unroll
  for (int b = 0; b < kMaxBlk; ++b) {
    const int blk = w + b * nwaves;
    if (blk >= nbt) continue;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      if (blk < nbe) {
        const int k = blk * kR + r;
        if (k < ne) tile[even_out(k) * (kCW + 1) + lane] = res[b][r];
      } else {
        const int k = (blk - nbe) * kR + r;
        if (k < no) tile[odd_out(k) * (kCW + 1) + lane] = res[b][r];
      }
    }
  }
}

// Forward transform of the tile (input x in natural order, output X in
// natural order).
template <typename T>
__device__ __forceinline__ void tile_forward(T* tile, const AxisTab<T>& a) {
  const int L = a.L, M = a.M;
  for (int p = threadIdx.x; p < M * kCW; p += blockDim.x) {
    const int j = p / kCW, c = p % kCW;
    const T x0 = tile[j * (kCW + 1) + c];
    const T x1 = tile[(L - 1 - j) * (kCW + 1) + c];
    tile[j * (kCW + 1) + c] = x0 + x1;            // u_j
    tile[(L - 1 - j) * (kCW + 1) + c] = x0 - x1;  // v_j
  }
  __syncthreads();
  T res[kMaxBlk][kR];
  dct_blocks(tile, a.fe, a.fo, a.ne, a.no, a.ne_pad, a.no_pad,
             [](int j) { return j; }, [L](int j) { return L - 1 - j; }, res);
  __syncthreads();
  dct_store(tile, a.ne, a.no, a.ne_pad, a.no_pad,
            [](int k) { return 2 * k; }, [](int k) { return 2 * k + 1; }, res);
  __syncthreads();
}

// Inverse transform (DCT-III, the transpose) of the tile, natural order in
// and out.
template <typename T>
__device__ __forceinline__ void tile_inverse(T* tile, const AxisTab<T>& a) {
  const int L = a.L, M = a.M;
  T res[kMaxBlk][kR];
  dct_blocks(tile, a.ie, a.io, a.ne, a.no, a.ne_pad, a.no_pad,
             [](int k) { return 2 * k; }, [](int k) { return 2 * k + 1; }, res);
  __syncthreads();
  // E_j -> slot j (j < ne), O_j -> slot L-1-j (j < M)
  dct_store(tile, a.ne, a.no, a.ne_pad, a.no_pad,
            [](int j) { return j; }, [L](int j) { return L - 1 - j; }, res);
  __syncthreads();
  for (int p = threadIdx.x; p < M * kCW; p += blockDim.x) {
    const int j = p / kCW, c = p % kCW;
    const T e = tile[j * (kCW + 1) + c];
    const T o = tile[(L - 1 - j) * (kCW + 1) + c];
    tile[j * (kCW + 1) + c] = e + o;
    tile[(L - 1 - j) * (kCW + 1) + c] = e - o;
  }
  __syncthreads();
}

// Divergence b = A^*(q - alpha/sigma) - c/sigma at node (t, spatial index xs),
// the right-hand side of the phi-step of Algorithm 2 (zero extension outside each staggered set).
template <typename T, int D>
__device__ __forceinline__ T divergence_at(const Geo& g, const T* __restrict__ q, const T* __restrict__ al,
                                           const double* __restrict__ c_lo, const double* __restrict__ c_hi,
                                           double inv_sigma, int t, int64_t xs) {
  const int64_t nb = g.nb;
  const int64_t i = (int64_t)t * g.stride[0] + xs;
  double b = 0.0;
  // time axis: cells t-1 and t
  if (t >= 1) b += ((double)q[i - g.stride[0]] - (double)al[i - g.stride[0]] * inv_sigma) * g.inv_h[0];
  if (t < g.n[0]) b -= ((double)q[i] - (double)al[i] * inv_sigma) * g.inv_h[0];
  int64_t r = xs;
#pragma unroll
  for (int d = D; d >= 1; --d) {
    const int xd = (int)(r % g.N[d]);
    r /= g.N[d];
    const T* qd = q + d * nb;
    const T* ad = al + d * nb;
    if (xd >= 1) b += ((double)qd[i - g.stride[d]] - (double)ad[i - g.stride[d]] * inv_sigma) * g.inv_h[d];
    if (xd < g.n[d]) b -= ((double)qd[i] - (double)ad[i] * inv_sigma) * g.inv_h[d];
  }
  if (t == 0) b -= c_lo[xs] * inv_sigma;
  if (t == g.n[0]) b -= c_hi[xs] * inv_sigma;
  return (T)b;
}

struct PassArgs {
  int64_t inner;   // stride of the transformed axis
  int64_t ncols;   // number of lines = outer * inner
};

// One axis pass over a plane, in place. SRC = kSrcDivergence (time axis only,
// first pass) computes the divergence of (q, alpha) while loading. KIND =
// kFwdScaleInv (last axis only) applies forward, 1/Lambda, inverse.
template <typename T, int D, int KIND, int SRC>
__global__ void __launch_bounds__(kDctWaves * 64)
k_axis_pass(Geo g, PassArgs pa, AxisTab<T> a, T* __restrict__ plane,
            const T* __restrict__ q, const T* __restrict__ al,
            const double* __restrict__ c_lo, const double* __restrict__ c_hi,
            const T* __restrict__ lam_other, const T* __restrict__ lam_last,
            const Ctl* __restrict__ ctl, double sigma_arg) {
  extern __shared__ unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  if (ctl && ctl->stop) return;
  const int L = a.L;
  const int64_t c0 = (int64_t)blockIdx.x * kCW;
  const int64_t inner = pa.inner;
  const int64_t ncols = pa.ncols;
  double inv_sigma = 0.0;
  if (SRC == kSrcDivergence) inv_sigma = 1.0 / (ctl ? ctl->sigma : sigma_arg);

  // load
  if (inner == 1) {
    for (int e = threadIdx.x; e < L * kCW; e += blockDim.x) {
      const int cl = e / L, j = e % L;
      const int64_t c = c0 + cl;
      T v = T(0);
      if (c < ncols) v = plane[c * L + j];
      tile[j * (kCW + 1) + cl] = v;
    }
  } else {
    for (int e = threadIdx.x; e < L * kCW; e += blockDim.x) {
      const int j = e / kCW, cl = e % kCW;
      const int64_t c = c0 + cl;
      T v = T(0);
      if (c < ncols) {
        if (SRC == kSrcDivergence) {
          v = divergence_at<T, D>(g, q, al, c_lo, c_hi, inv_sigma, j, c);
        } else {
          const int64_t o = c / inner, ii = c % inner;
          v = plane[o * (int64_t)L * inner + (int64_t)j * inner + ii];
        }
      }
      tile[j * (kCW + 1) + cl] = v;
    }
  }
  __syncthreads();

  if (KIND == kFwd || KIND == kFwdScaleInv) tile_forward(tile, a);
  if (KIND == kFwdScaleInv) {
    for (int e = threadIdx.x; e < L * kCW; e += blockDim.x) {
      const int k = e / kCW, cl = e % kCW;
      const int64_t c = c0 + cl;
      T s = T(0);
      if (c < ncols) {
        const T lam = lam_other[c] + lam_last[k];
        s = lam > T(0) ? T(1) / lam : T(0);  // mode (0,...,0): phi in rge A^*
      }
      tile[k * (kCW + 1) + cl] *= s;
    }
    __syncthreads();
  }
  if (KIND == kInv || KIND == kFwdScaleInv) tile_inverse(tile, a);

  // store
  if (inner == 1) {
    for (int e = threadIdx.x; e < L * kCW; e += blockDim.x) {
      const int cl = e / L, j = e % L;
      const int64_t c = c0 + cl;
      if (c < ncols) plane[c * L + j] = tile[j * (kCW + 1) + cl];
    }
  } else {
    for (int e = threadIdx.x; e < L * kCW; e += blockDim.x) {
      const int j = e / kCW, cl = e % kCW;
      const int64_t c = c0 + cl;
      if (c < ncols) {
        const int64_t o = c / inner, ii = c % inner;
        plane[o * (int64_t)L * inner + (int64_t)j * inner + ii] = tile[j * (kCW + 1) + cl];
      }
    }
  }
}

}  // namespace dot
