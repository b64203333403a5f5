// Cosine-transform passes of the space-time Poisson solve (Sec. 4, the
// phi-step of Algorithm 2): A^*A is the sum over axes of path-graph Laplacians / h_d^2, whose
// eigenvectors are the orthonormal DCT-II basis of length N_d = n_d + 1.
//
// One pass transforms every line of one axis. A workgroup stages a tile of
// kCW lines x L points in LDS (one line per column), folds each line into its
// symmetric and antisymmetric halves (x_j +- x_{L-1-j}), which the even-row
// and odd-row halves of the transform matrix act on separately, and runs both
// half-size products on the matrix cores (16x16x4 MFMA, FP64 or FP32): the
// matrix is the A operand, streamed from a fragment-major table (one
// coalesced element per lane per k-step, prefetched one step ahead), and the
// folded lines are the B operand, read from LDS. Passes work in place: a tile
// holds whole lines, so a workgroup reads and writes only its own elements.
#pragma once
#include "geometry.hpp"

namespace dot {

constexpr int kCW = 64;        // lines per tile (launches with many tiles)
constexpr int kCWMid = 32;     // lines per tile where 64 lines do not fit the LDS or give too few tiles
constexpr int kCWNarrow = 16;  // lines per tile (launches with few tiles: 4x the workgroups)
constexpr int kMaxWaves = 16;  // waves per workgroup (upper bound)
constexpr int kU = 8;          // k-steps per prefetch chunk
constexpr int kLoadBatch = 8;  // rows a wave loads before writing them to the tile

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaOps;
template <> struct MfmaOps<double> {
  typedef dbl4 acc_t;
  typedef double chunk_t __attribute__((ext_vector_type(kU)));
  static constexpr int kItems = 3;  // work items per wave
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element v of lane l is row (l / 16) + 4 v, column l % 16 (gfx950)
  __device__ static int out_row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct MfmaOps<float> {
  typedef flt4 acc_t;
  typedef float chunk_t __attribute__((ext_vector_type(kU)));
  static constexpr int kItems = 5;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element v of lane l is row 4 (l / 16) + v, column l % 16 (gfx950)
  __device__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Folded transform tables of one axis, fragment-major in chunks of kU
// k-steps: for a half matrix H with rb row blocks and ks k-steps (a multiple
// of kU), element (m, s, lane) sits at
//   ((m * (ks / kU + 1) + s / kU) * 64 + lane) * kU + s % kU
// and holds H[16 m + lane % 16][4 s + lane / 16] (zero outside H), so one
// lane reads its kU fragments of a chunk as one contiguous vector; the extra
// zero chunk per row block lets the prefetch run past the end unguarded. With C[k][j] = s_k cos(pi k (2j+1) / (2L)) the halves are
//   forward even  H[k'][j] = C[2k'][j]    (j < ne: u_0..u_{M-1}, middle point)
//   forward odd   H[k'][j] = C[2k'+1][j]  (j < no: v_j)
//   inverse even  H[j][k'] = C[2k'][j]    (outputs E_j from X_{2k'})
//   inverse odd   H[j][k'] = C[2k'+1][j]  (outputs O_j from X_{2k'+1})
template <typename T>
struct AxisTab {
  const T* fe;
  const T* fo;
  const T* ie;
  const T* io;
  int L, M, ne, no;
  int rb_e, rb_o, ks_e, ks_o;
};

// Work items a wave may take in one pass: a narrow tile has one accumulator
// per item instead of two, so a wave holds twice as many items in the same
// registers.
template <typename T, int CW>
constexpr int items_per_wave() {
  return MfmaOps<T>::kItems * (CW >= 32 ? 1 : 2);
}

enum PassKind { kFwd = 0, kInv = 1, kFwdScaleInv = 2 };
// What the first (time-axis forward) pass loads: the work plane itself (in
// place), or an FP64 right-hand side plane (mixed-precision step call).
enum PassSrc { kSrcPlane = 0, kSrcPlaneF64 = 3 };
// Where the last (time-axis inverse) pass stores: the work plane, phi += result
// (FP64), or phi = result (FP64).
enum PassDst { kDstPlane = 0, kDstPhiAdd = 1, kDstPhiSet = 2 };

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Tile slot of input k of a half: forward even u_k / middle at k; forward odd
// v_k at L-1-k; inverse even X_{2k} at 2k; inverse odd X_{2k+1} at 2k+1.
__device__ __forceinline__ int in_slot(bool inv, bool odd, int L, int k) {
  return inv ? (odd ? 2 * k + 1 : 2 * k) : (odd ? L - 1 - k : k);
}
// Tile slot of output r of a half: forward X_{2r} / X_{2r+1}; inverse E_r at r,
// O_r at L-1-r.
__device__ __forceinline__ int out_slot(bool inv, bool odd, int L, int r) {
  return inv ? (odd ? L - 1 - r : r) : (odd ? 2 * r + 1 : 2 * r);
}

// Both half-size products of one direction on a tile of CW columns; results
// are written back into the tile (natural order after a forward pass; E/O
// slots after an inverse pass, combined by the caller). A work item is one
// 16-row block of a half matrix times 16 * NACC columns (NACC accumulators
// sharing the coefficient fragments).
template <typename T, int CW>
__device__ __forceinline__ void tile_mfma(T* tile, const AxisTab<T>& a, bool inv) {
  typedef typename MfmaOps<T>::acc_t acc_t;
  constexpr int KI = items_per_wave<T, CW>();
  constexpr int NACC = CW >= 32 ? 2 : 1;
  constexpr int NG = CW / (16 * NACC);  // column groups per row block
  const int lane = threadIdx.x & 63;
  const int w = wave_id();
  const int nwaves = blockDim.x >> 6;
  const int nitems = NG * (a.rb_e + a.rb_o);
  const int L = a.L;
  acc_t acc[KI][NACC];
#pragma unroll
  for (int b = 0; b < KI; ++b) {
#pragma unroll
    for (int h = 0; h < NACC; ++h) acc[b][h] = acc_t{0, 0, 0, 0};
    const int it = w + b * nwaves;
    if (it >= nitems) continue;
    const int rbi = it / NG, g = it % NG;
    const bool odd = rbi >= a.rb_e;
    const int m = odd ? rbi - a.rb_e : rbi;
    const int ks = odd ? a.ks_o : a.ks_e;
    const int nin = odd ? a.no : a.ne;
    typedef typename MfmaOps<T>::chunk_t chunk_t;
    gp<const chunk_t> tp = (gp<const chunk_t>)reinterpret_cast<const chunk_t*>(inv ? (odd ? a.io : a.ie)
                                                                                  : (odd ? a.fo : a.fe)) +
                           (size_t)m * (ks / kU + 1) * 64 + lane;
    const int col = g * 16 * NACC + (lane & 15);
    const int kr = (nin + 3) >> 2;  // k-steps holding inputs (the rest of the last chunk is zero padding)
    // coefficient fragments are prefetched one chunk of kU k-steps ahead
    chunk_t cur = tp[0];
    for (int st = 0; st < ks; st += kU) {
      const chunk_t nxt = tp[(st / kU + 1) * 64];
      // keep the prefetch ahead of this chunk's LDS reads and MFMAs
      __builtin_amdgcn_sched_barrier(0);
      T bv[NACC][kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        int k = (st + u) * 4 + (lane >> 4);
        k = k < nin ? k : nin - 1;  // padded inputs: zero coefficient, any finite value
        const int sl = in_slot(inv, odd, L, k) * (CW + 1) + col;
#pragma unroll
        for (int h = 0; h < NACC; ++h) bv[h][u] = tile[sl + 16 * h];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (st + u >= kr) break;  // zero coefficients only
#pragma unroll
        for (int h = 0; h < NACC; ++h) acc[b][h] = MfmaOps<T>::mma(cur[u], bv[h][u], acc[b][h]);
      }
      cur = nxt;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < KI; ++b) {
    const int it = w + b * nwaves;
    if (it >= nitems) continue;
    const int rbi = it / NG, g = it % NG;
    const bool odd = rbi >= a.rb_e;
    const int m = odd ? rbi - a.rb_e : rbi;
    const int nout = odd ? a.no : a.ne;
    const int col = g * 16 * NACC + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = m * 16 + MfmaOps<T>::out_row(lane, v);
      if (r < nout) {
        const int sl = out_slot(inv, odd, L, r) * (CW + 1) + col;
#pragma unroll
        for (int h = 0; h < NACC; ++h) tile[sl + 16 * h] = acc[b][h][v];
      }
    }
  }
  __syncthreads();
}

// Forward transform of the tile (input x in natural order, output X in
// natural order).
template <typename T, int CW>
__device__ __forceinline__ void tile_forward(T* tile, const AxisTab<T>& a) {
  const int L = a.L, M = a.M;
  for (int p = threadIdx.x; p < M * CW; p += blockDim.x) {
    const int j = p / CW, c = p % CW;
    const T x0 = tile[j * (CW + 1) + c];
    const T x1 = tile[(L - 1 - j) * (CW + 1) + c];
    tile[j * (CW + 1) + c] = x0 + x1;            // u_j
    tile[(L - 1 - j) * (CW + 1) + c] = x0 - x1;  // v_j
  }
  __syncthreads();
  tile_mfma<T, CW>(tile, a, false);
}

// Inverse transform (DCT-III, the transpose) of the tile, natural order in
// and out: E_j = sum_k' C[2k'][j] X_{2k'}, O_j = sum_k' C[2k'+1][j] X_{2k'+1},
// x_j = E_j + O_j, x_{L-1-j} = E_j - O_j.
template <typename T, int CW>
__device__ __forceinline__ void tile_inverse(T* tile, const AxisTab<T>& a) {
  const int L = a.L, M = a.M;
  tile_mfma<T, CW>(tile, a, true);
  for (int p = threadIdx.x; p < M * CW; p += blockDim.x) {
    const int j = p / CW, c = p % CW;
    const T e = tile[j * (CW + 1) + c];
    const T o = tile[(L - 1 - j) * (CW + 1) + c];
    tile[j * (CW + 1) + c] = e + o;
    tile[(L - 1 - j) * (CW + 1) + c] = e - o;
  }
  __syncthreads();
}

// Divergence b = A^*(q - alpha/sigma) - c/sigma at node (t, spatial index xs
// with spatial coordinates x[1..D]), the right-hand side of the phi-step of
// Algorithm 2 (zero extension outside each staggered set).
template <typename T, int D>
__device__ __forceinline__ double divergence_at(const Geo& g, const T* q_, const double* al_,
                                           const double* __restrict__ c_lo, const double* __restrict__ c_hi,
                                           double inv_sigma, int t, uint32_t xs, const int (&x)[kMaxAxes]) {
  const uint32_t nb = (uint32_t)g.nb;
  const uint32_t s0 = (uint32_t)g.stride[0];
  const uint32_t i = (uint32_t)t * s0 + xs;
  gp<const T> q = glob(q_);
  gp<const double> al = glob(al_);
  double b = 0.0;
  // time axis: cells t-1 and t
  if (t >= 1) b += ((double)q[i - s0] - (double)al[i - s0] * inv_sigma) * g.inv_h[0];
  if (t < g.n[0]) b -= ((double)q[i] - (double)al[i] * inv_sigma) * g.inv_h[0];
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    const uint32_t sd = (uint32_t)g.stride[d];
    gp<const T> qd = q + (size_t)d * nb;
    gp<const double> ad = al + (size_t)d * nb;
    if (x[d] >= 1) b += ((double)qd[i - sd] - (double)ad[i - sd] * inv_sigma) * g.inv_h[d];
    if (x[d] < g.n[d]) b -= ((double)qd[i] - (double)ad[i] * inv_sigma) * g.inv_h[d];
  }
  if (t == 0) b -= glob(c_lo)[xs] * inv_sigma;
  if (t == g.n[0]) b -= glob(c_hi)[xs] * inv_sigma;
  return b;
}

// Spatial coordinates x[1..D] of spatial flat index xs.
template <int D>
__device__ __forceinline__ void spatial_coords(const Geo& g, uint32_t xs, int (&x)[kMaxAxes]) {
  uint32_t r = xs;
#pragma unroll
  for (int d = D; d >= 1; --d) {
    x[d] = (int)(r % (uint32_t)g.N[d]);
    r /= (uint32_t)g.N[d];
  }
  x[0] = 0;
}

struct PassArgs {
  int64_t inner;   // stride of the transformed axis
  int64_t ncols;   // number of lines = outer * inner
};

// One axis pass over a plane, in place, on tiles of CW lines. SRC and DST
// other than kSrcPlane / kDstPlane occur on the time axis only (first forward
// / last inverse pass). KIND = kFwdScaleInv (last axis only) applies forward,
// 1/Lambda, inverse.
template <typename T, int D, int KIND, int SRC, int DST, int CW>
__device__ __forceinline__ void axis_pass_body(const Geo& g, const PassArgs& pa, const AxisTab<T>& a,
                                               T* __restrict__ plane, double* __restrict__ phi,
                                               const T* __restrict__ lam_other, const T* __restrict__ lam_last,
                                               int64_t blk) {
  extern __shared__ unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  const int L = a.L;
  const int64_t c0 = blk * CW;
  const uint32_t inner = (uint32_t)pa.inner;
  const int64_t ncols = pa.ncols;
  gp<T> pl = glob(plane);
  gp<double> ph = glob(phi);
  const int tot = L * CW;
  if (KIND == kFwdScaleInv) {
    // stage the eigenvalue tables of this tile behind it in LDS (read after
    // the forward transform, so their latency hides behind the tile load)
    T* lam_r = tile + L * (CW + 1);
    T* lam_c = lam_r + L;
    for (int e = threadIdx.x; e < L + CW; e += blockDim.x) {
      if (e < L)
        lam_r[e] = glob(lam_last)[e];
      else
        lam_c[e - L] = c0 + (e - L) < ncols ? glob(lam_other)[c0 + (e - L)] : T(0);
    }
  }
  // Loads and stores use 32-bit index math (planes hold at most 2^28
  // elements). Lines along the last axis (inner == 1) are contiguous and are
  // walked line by line; strided lines (column c = o * inner + ii) give each
  // thread one fixed tile column (blockDim is a multiple of CW) and a row
  // stride, so CW consecutive columns of a row are consecutive in memory.
  const int nthr = blockDim.x;
  const int my_cl = threadIdx.x % CW, row0 = threadIdx.x / CW, rstep = nthr / CW;
  uint32_t cbase = 0;
  bool cok = false;
  if (inner != 1) {
    const int64_t c = c0 + my_cl;
    cok = c < ncols;
    const uint32_t cu = (uint32_t)c;
    const uint32_t o = cu / inner, ii = cu - o * inner;
    cbase = o * (uint32_t)L * inner + ii;
  }
  const uint32_t lbase = (uint32_t)c0 * (uint32_t)L;
  const uint32_t llim = (uint32_t)ncols * (uint32_t)L;
  // load: each thread issues kLoadBatch independent loads before writing
  // them to the tile, so the memory latency is paid once per batch
  if (inner == 1) {
    for (int e0 = threadIdx.x; e0 < tot; e0 += kLoadBatch * nthr) {
      T v[kLoadBatch];
#pragma unroll
      for (int r = 0; r < kLoadBatch; ++r) {
        const int e = e0 + r * nthr;
        v[r] = (e < tot && lbase + e < llim) ? (SRC == kSrcPlaneF64 ? (T)ph[lbase + e] : pl[lbase + e]) : T(0);
      }
#pragma unroll
      for (int r = 0; r < kLoadBatch; ++r) {
        const int e = e0 + r * nthr;
        if (e < tot) {
          const int cl = e / L, j = e - cl * L;
          tile[j * (CW + 1) + cl] = v[r];
        }
      }
    }
  } else {
    for (int j0 = row0; j0 < L; j0 += kLoadBatch * rstep) {
      T v[kLoadBatch];
#pragma unroll
      for (int r = 0; r < kLoadBatch; ++r) {
        const int j = j0 + r * rstep;
        const uint32_t o = cbase + (uint32_t)j * inner;
        v[r] = (cok && j < L) ? (SRC == kSrcPlaneF64 ? (T)ph[o] : pl[o]) : T(0);
      }
#pragma unroll
      for (int r = 0; r < kLoadBatch; ++r) {
        const int j = j0 + r * rstep;
        if (j < L) tile[j * (CW + 1) + my_cl] = v[r];
      }
    }
  }
  __syncthreads();

  if (KIND == kFwd || KIND == kFwdScaleInv) tile_forward<T, CW>(tile, a);
  if (KIND == kFwdScaleInv) {
    // eigenvalue sums Lambda = lam_other[column] + lam_last[row] from the
    // copies staged in LDS at entry
    const T* lam_r = tile + L * (CW + 1);
    const T* lam_c = lam_r + L;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
      const int k = e / CW, cl = e % CW;
      const int64_t c = c0 + cl;
      T s = T(0);
      if (c < ncols) {
        const T lam = lam_c[cl] + lam_r[k];
        s = lam > T(0) ? T(1) / lam : T(0);  // mode (0,...,0): phi in rge A^*
      }
      tile[k * (CW + 1) + cl] *= s;
    }
    __syncthreads();
  }
  if (KIND == kInv || KIND == kFwdScaleInv) tile_inverse<T, CW>(tile, a);

  // store (phi += result in batches: loads first, then the stores)
  auto put = [&](uint32_t o, T v, double old) {
    if (DST == kDstPhiAdd)
      ph[o] = old + (double)v;
    else if (DST == kDstPhiSet)
      ph[o] = (double)v;
    else
      pl[o] = v;
  };
  if (inner == 1) {
    for (int e0 = threadIdx.x; e0 < tot; e0 += kLoadBatch * nthr) {
      double old[kLoadBatch];
#pragma unroll
      for (int r = 0; r < kLoadBatch; ++r) {
        const int e = e0 + r * nthr;
        old[r] = (DST == kDstPhiAdd && e < tot && lbase + e < llim) ? ph[lbase + e] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < kLoadBatch; ++r) {
        const int e = e0 + r * nthr;
        if (e < tot && lbase + e < llim) {
          const int cl = e / L, j = e - cl * L;
          put(lbase + e, tile[j * (CW + 1) + cl], old[r]);
        }
      }
    }
  } else if (cok) {
    for (int j0 = row0; j0 < L; j0 += kLoadBatch * rstep) {
      double old[kLoadBatch];
#pragma unroll
      for (int r = 0; r < kLoadBatch; ++r) {
        const int j = j0 + r * rstep;
        old[r] = (DST == kDstPhiAdd && j < L) ? ph[cbase + (uint32_t)j * inner] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < kLoadBatch; ++r) {
        const int j = j0 + r * rstep;
        if (j < L) put(cbase + (uint32_t)j * inner, tile[j * (CW + 1) + my_cl], old[r]);
      }
    }
  }
}

// Last-axis solve by tridiagonal elimination instead of forward transform,
// 1/Lambda and inverse transform. After the transforms of the other axes the
// system decouples into one tridiagonal system per line of the last axis:
//   lambda x_i + n^2 (deg_i x_i - x_{i-1} - x_{i+1}) = b_i,
// deg_i = 1 at the two ends and 2 inside (the path-graph Laplacian / h^2 that
// the DCT-II diagonalises), lambda = the line's eigenvalue sum over the other
// axes. lambda > 0: Thomas elimination in FP64 (diagonally dominant, no
// pivoting; the pivot reciprocal is the hardware reciprocal refined by one
// Newton step). lambda = 0 (the line of mode 0 on every other axis): the
// singular Neumann system is solved through its fluxes
// f_i = n^2 (x_{i+1} - x_i), f_0 = -b_0, f_i = f_{i-1} - b_i, and the line
// mean is removed (the constant mode of phi is zero). A workgroup takes CW
// consecutive lines (contiguous, stride 1 along the line) and walks them in
// chunks of kTriChunk points: the next chunk is loaded coalesced (all
// threads) while the current one is eliminated, one thread per line running
// the recurrence on its chunk in registers; chunks pass through LDS. The
// forward sweep stores d' in place and one c' checkpoint per chunk in `cpl`;
// the backward sweep recomputes c' from the checkpoints and stores x.
constexpr int kTriChunk = 32;
constexpr int kTriThreads = 256;

template <typename T, int CW>
struct TriTile {
  T a[2][CW][kTriChunk + 1];  // b, then d', then x (double buffered)
};

// Coalesced copy of one chunk (CW lines x kTriChunk points; element e is
// line e / kTriChunk, point e % kTriChunk) from a plane into registers, and
// from there into one buffer of the tile.
template <typename T, int CW>
struct TriChunk {
  static constexpr int kPer = (CW * kTriChunk + kTriThreads - 1) / kTriThreads;
  T v[kPer];
  __device__ __forceinline__ void load(gp<const T> src, uint32_t base, int L, int nl, int i0, int m) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int e = threadIdx.x + r * kTriThreads;
      const int l = e / kTriChunk, j = e - l * kTriChunk;
      v[r] = (l < nl && j < m) ? src[base + (uint32_t)l * L + i0 + j] : T(0);
    }
  }
  __device__ __forceinline__ void put(T (&buf)[CW][kTriChunk + 1]) const {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int e = threadIdx.x + r * kTriThreads;
      const int l = e / kTriChunk, j = e - l * kTriChunk;
      if (l < CW) buf[l][j] = v[r];
    }
  }
};

template <typename T, int CW>
__device__ __forceinline__ void tri_store(gp<T> dst, const T (&buf)[CW][kTriChunk + 1], uint32_t base, int L, int nl,
                                          int i0, int m) {
  for (int e = threadIdx.x; e < CW * kTriChunk; e += kTriThreads) {
    const int l = e / kTriChunk, j = e - l * kTriChunk;
    if (l < nl && j < m) dst[base + (uint32_t)l * L + i0 + j] = buf[l][j];
  }
}

__device__ __forceinline__ double tri_recip(double b) {
  const double r = __builtin_amdgcn_rcp(b);
  return r * fma(-b, r, 2.0);
}

// One step of the elimination coefficients of a line of the tridiagonal
// system (lam + n^2 L_path) x = b: pivot reciprocal r_i of node i given
// c'_{i-1} (0 before the first node) and the new c'_i = -n^2 r_i. The forward
// and the backward sweep both call it, so the c' that the backward sweep
// recomputes are those the forward sweep used, bit for bit.
__device__ __forceinline__ double tri_cstep(double lam, double s2, int i, int L, double cp, double* r) {
  const double diag = lam + s2 * ((i == 0 || i == L - 1) ? 1.0 : 2.0);
  *r = tri_recip(diag + s2 * cp);
  return -s2 * *r;
}

// Tridiagonal solve along the last axis for one tile of CW lines (one owner
// thread per line runs the recurrences; all threads stage chunks of
// kTriChunk points through LDS). The forward sweep overwrites b with d' and
// keeps, per line and chunk, only the c' carried into the chunk (FP64, in
// `cpl` reused as an array [chunk][line]); the backward sweep re-runs the c'
// recurrence of each chunk from that checkpoint, so c' never goes through HBM
// (per point 4 plane accesses instead of 6).
template <typename T, int CW>
__device__ __forceinline__ void tri_pass_body(const Geo& g, T* __restrict__ plane, T* __restrict__ cpl,
                                              const T* __restrict__ lam_other, int64_t blk) {
  const int D = g.D;
  const int L = g.N[D];
  const double s2 = (double)g.n[D] * (double)g.n[D];
  // the zero line's flux steps multiply by 1 / n^2 (exact for n_D a power of
  // two) rather than divide: an FP64 division per step made its workgroup the
  // last to finish
  const double inv_s2 = 1.0 / s2;
  const int64_t ncols = g.nb / L;
  const int64_t c0 = blk * CW;
  const int nl = (int)((ncols - c0) < CW ? (ncols - c0) : CW);  // lines of this tile
  __shared__ TriTile<T, CW> tt;
  gp<T> pl = glob(plane);
  // checkpoints: nch * ncols doubles, within the plane's nb * sizeof(T) bytes
  // for every L >= 2 (nch = ceil(L / 32) <= L / 2)
  gp<double> ck = glob(reinterpret_cast<double*>(cpl));
  const uint32_t base = (uint32_t)c0 * (uint32_t)L;
  const int me = threadIdx.x;
  const bool owner = me < nl;
  const double lam = owner ? (double)glob(lam_other)[c0 + me] : 1.0;
  const bool zero = lam == 0.0;
  const int nch = (L + kTriChunk - 1) / kTriChunk;
  auto len = [&](int k) { return L - k * kTriChunk < kTriChunk ? L - k * kTriChunk : kTriChunk; };
  auto ck_at = [&](int k) { return (size_t)k * (size_t)ncols + (size_t)(c0 + me); };
  double cp = 0.0, dp = 0.0, sum = 0.0;
  TriChunk<T, CW> nx;
  // forward sweep
  nx.load(pl, base, L, nl, 0, len(0));
  nx.put(tt.a[0]);
  __syncthreads();
  for (int k = 0; k < nch; ++k) {
    const int i0 = k * kTriChunk, m = len(k);
    const int b = k & 1;
    if (k + 1 < nch) nx.load(pl, base, L, nl, i0 + kTriChunk, len(k + 1));
    if (owner) {
      if (!zero) ck[ck_at(k)] = cp;
      T rv[kTriChunk];
#pragma unroll
      for (int j = 0; j < kTriChunk; ++j) rv[j] = tt.a[b][me][j];
#pragma unroll
      for (int j = 0; j < kTriChunk; ++j) {
        if (j < m) {
          const int i = i0 + j;
          const double bj = (double)rv[j];
          if (zero) {
            // x_0 = 0, x_{i+1} = x_i + f_i / n^2 with f_i = f_{i-1} - b_i
            rv[j] = (T)dp;
            sum += dp;
            cp -= bj;
            dp += cp * inv_s2;
          } else {
            double r;
            cp = tri_cstep(lam, s2, i, L, cp, &r);
            dp = (bj + s2 * dp) * r;
            rv[j] = (T)dp;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kTriChunk; ++j) tt.a[b][me][j] = rv[j];
    }
    __syncthreads();
    tri_store<T, CW>(pl, tt.a[b], base, L, nl, i0, m);
    if (k + 1 < nch) nx.put(tt.a[b ^ 1]);
    __syncthreads();
  }
  // backward sweep: x_{L-1} = d'_{L-1}, x_i = d'_i - c'_i x_{i+1} (c' = 0 on
  // the zero line, whose d' already is x), minus the line mean on the zero line
  const double mean = zero ? sum / (double)L : 0.0;
  double x = 0.0;
  double cnext = (owner && !zero) ? ck[ck_at(nch - 1)] : 0.0;
  nx.load(pl, base, L, nl, (nch - 1) * kTriChunk, len(nch - 1));
  nx.put(tt.a[0]);
  __syncthreads();
  for (int k = nch - 1, u = 0; k >= 0; --k, ++u) {
    const int i0 = k * kTriChunk, m = len(k);
    const int b = u & 1;
    const double cstart = cnext;
    if (k > 0) {
      nx.load(pl, base, L, nl, i0 - kTriChunk, kTriChunk);
      if (owner && !zero) cnext = ck[ck_at(k - 1)];
    }
    if (owner) {
      T dv[kTriChunk], cv[kTriChunk];
      double c = cstart;
#pragma unroll
      for (int j = 0; j < kTriChunk; ++j) {
        cv[j] = T(0);
        if (j < m && !zero) {
          double r;
          c = tri_cstep(lam, s2, i0 + j, L, c, &r);
          cv[j] = (T)c;
        }
      }
#pragma unroll
      for (int j = 0; j < kTriChunk; ++j) dv[j] = tt.a[b][me][j];
#pragma unroll
      for (int j = kTriChunk - 1; j >= 0; --j) {
        if (j < m) {
          x = (double)dv[j] - (double)cv[j] * x;
          dv[j] = (T)(x - mean);
        }
      }
#pragma unroll
      for (int j = 0; j < kTriChunk; ++j) tt.a[b][me][j] = dv[j];
    }
    __syncthreads();
    tri_store<T, CW>(pl, tt.a[b], base, L, nl, i0, m);
    if (k > 0) nx.put(tt.a[b ^ 1]);
    __syncthreads();
  }
}

// ---- partitioned elimination of the last-axis line systems -------------------
// The same line systems as tri_pass_body, (lam + n^2 L_path) x = b along each
// line of the last axis, solved with P lanes per line instead of one. Lane k
// of a line's group owns the consecutive rows [lo, hi) (segment sizes differ
// by at most one); u = x_{lo-1} and z = x_{hi-1} denote the row before its
// segment and its own last row.
//   1. Forward elimination of the segment with u kept as an unknown gives its
//      last row as z = d + g u - c x_{hi} (c = -n^2 r, r the pivot reciprocals,
//      which are kept).
//   2. Elimination of rows hi-2 .. lo from the bottom, with z kept as an
//      unknown, gives its first row as x_lo = al + be u + ga z.
//   3. Putting the next segment's first-row relation into the first gives one
//      equation per segment in the last rows z_k:
//        -g z_{k-1} + (1 + c be') z_k + c ga' z_{k+1} = d - c al',
//      a tridiagonal system of order P (the primes: the next segment's
//      values), solved by the P lanes together by parallel cyclic reduction
//      through cross-lane shuffles (log2 P steps; the reduced system of a
//      diagonally dominant one is diagonally dominant).
//   4. With u = z_{k-1} known, the segment's rows follow from a forward pass
//      with the kept pivots and a backward pass from z_k.
// All arithmetic is FP64 (the plane's type only for load and store). The lines
// of a round are staged in LDS as FP64 (padded by one element per 16, so that
// lanes reading rows about 16 apart fall on different banks), so the plane is
// read once and written once, coalesced, and the passes read their rows from
// LDS. The line with lam = 0 (mode 0 on every other axis) is the singular
// Neumann problem: its fluxes f_i = -(b_0 + ... + b_i) and values x_i =
// (f_0 + ... + f_{i-1}) / n^2 are prefix sums, taken per segment and across
// the lanes by shuffle scans, and the line mean is removed (the constant mode
// of phi is zero), as in the one-lane solve.
// The rows per lane are bounded by kTriSeg, a compile-time constant (the size
// of the register arrays); lines of up to 64 kTriSeg nodes take this solve,
// longer ones the one-lane-per-line solve (measured at 1025 nodes: with 17
// rows per lane the arrays no longer fit the registers of two waves per SIMD,
// and the partitioned solve was slower than the one-lane solve, 230-260 us
// against 208 us per pass at 2D 32x1024^2 mixed).
constexpr int kTriSeg = 9;
constexpr int kTriPartMaxNodes = 64 * kTriSeg;  // longest line (64 lanes of 9 rows)

// Lanes per line: 16, 32 or 64, the fewest that keep segments within kTriSeg rows.
__device__ __host__ __forceinline__ int tri_lanes(int L) {
  return L <= 16 * kTriSeg ? 16 : (L <= 32 * kTriSeg ? 32 : 64);
}

__device__ __forceinline__ int tri_pad(int i) { return i + (i >> 4); }

// Inclusive prefix sum of v over the P lanes of a group (Hillis-Steele).
__device__ __forceinline__ double group_scan(double v, int k, int P) {
  for (int s = 1; s < P; s <<= 1) {
    const double o = __shfl_up(v, s, P);
    if (k >= s) v += o;
  }
  return v;
}

__device__ __forceinline__ double group_sum(double v, int P) {
  for (int s = P >> 1; s >= 1; s >>= 1) v += __shfl_xor(v, s, P);
  return v;
}

template <typename T>
__device__ __forceinline__ void tri_part_body(const Geo& g, T* __restrict__ plane, const T* __restrict__ lam_other,
                                              int64_t tile, int cw) {
  constexpr int kTriSegMax = kTriSeg;
  constexpr int kTriLoadPer = kTriSeg;  // elements per thread of one round's copy (lpr L <= 16 kTriSeg * 16)
  constexpr int kTriPartElems = 16 * (16 * kTriSeg + kTriSeg + 1);  // LDS doubles of one round (padded lines)
  __shared__ double buf[kTriPartElems];
  const int D = g.D;
  const int L = g.N[D];
  const double s2 = (double)g.n[D] * (double)g.n[D];
  const double inv_s2 = 1.0 / s2;
  const int P = tri_lanes(L);
  const int lpr = kTriThreads / P;  // lines per round
  const int64_t ncols = g.nb / L;
  const int64_t ct = tile * cw;
  const int nlt = (int)((ncols - ct) < cw ? (ncols - ct) : cw);
  const int k = threadIdx.x & (P - 1);  // segment of this lane
  const int grp = threadIdx.x / P;      // line of this lane within the round
  const int lo = (k * L) / P, hi = ((k + 1) * L) / P, len = hi - lo;
  const int Lp = tri_pad(L) + 1;  // padded line length in LDS
  gp<T> pl = glob(plane);
  auto diag_at = [&](double lam, int i) { return lam + s2 * ((i == 0 || i == L - 1) ? 1.0 : 2.0); };
  for (int r0 = 0; r0 < nlt; r0 += lpr) {
    const int nl = nlt - r0 < lpr ? nlt - r0 : lpr;
    const uint32_t base = (uint32_t)(ct + r0) * (uint32_t)L;
    const int tot = nl * L;
    {
      // coalesced copy of the round's lines into LDS; every thread issues its
      // loads before the first LDS write
      T v[kTriLoadPer];
      int i = threadIdx.x, ln = 0;  // line ln, node i of element threadIdx.x
      while (i >= L) {
        i -= L;
        ++ln;
      }
#pragma unroll
      for (int r = 0; r < kTriLoadPer; ++r) {
        const int e = threadIdx.x + r * kTriThreads;
        v[r] = e < tot ? pl[base + e] : T(0);
      }
#pragma unroll
      for (int r = 0; r < kTriLoadPer; ++r) {
        const int e = threadIdx.x + r * kTriThreads;
        if (e < tot) buf[ln * Lp + tri_pad(i)] = (double)v[r];
        i += kTriThreads;
        while (i >= L) {
          i -= L;
          ++ln;
        }
      }
    }
    __syncthreads();
    const bool active = grp < nl;
    const double lam = active ? (double)glob(lam_other)[ct + r0 + grp] : 1.0;
    double* row = buf + (active ? grp : 0) * Lp;  // this lane's line
    auto rd = [&](int j) { return active ? row[tri_pad(lo + j)] : 0.0; };
    if (lam == 0.0) {
      // singular line: prefix sums of b, then of the fluxes
      double sb = 0.0;
      for (int j = 0; j < len; ++j) sb += rd(j);
      const double pb = group_scan(sb, k, P) - sb;  // b_0 + ... + b_{lo-1}
      double cb = pb, sf = 0.0;
      for (int j = 0; j < len; ++j) {
        cb += rd(j);
        sf -= cb;  // f_{lo+j} = -(b_0 + ... + b_{lo+j})
      }
      double x = group_scan(sf, k, P) - sf;  // f_0 + ... + f_{lo-1}
      double sx = 0.0;
      cb = pb;
      for (int j = 0; j < len; ++j) {
        const double bj = rd(j);
        const double xj = x * inv_s2;
        if (active) row[tri_pad(lo + j)] = xj;
        sx += xj;
        cb += bj;
        x -= cb;
      }
      const double mean = group_sum(sx, P) / (double)L;
      if (active)
        for (int j = 0; j < len; ++j) row[tri_pad(lo + j)] -= mean;
    } else {
      // the segment's right-hand side in registers (rows past its end read
      // its last row; every loop below runs the full length and keeps the
      // values of valid rows only, without branches)
      double bv[kTriSegMax];
#pragma unroll
      for (int j = 0; j < kTriSegMax; ++j) bv[j] = row[tri_pad(lo + (j < len ? j : len - 1))];
      if (!active) {
#pragma unroll
        for (int j = 0; j < kTriSegMax; ++j) bv[j] = 0.0;
      }
      // 1: forward elimination with u unknown; pivots kept
      double rv[kTriSegMax];
      double cp = 0.0, dp = 0.0, gq = lo > 0 ? 1.0 : 0.0;
#pragma unroll
      for (int j = 0; j < kTriSegMax; ++j) {
        const int i = lo + j;
        const double r = tri_recip(diag_at(lam, i) + s2 * cp);
        const bool ok = j < len;
        rv[j] = r;
        dp = ok ? (bv[j] + s2 * dp) * r : dp;
        gq = ok ? s2 * gq * r : gq;
        cp = ok ? (i < L - 1 ? -s2 * r : 0.0) : cp;
      }
      // 2: first row in terms of u and z, by elimination from the bottom
      double al = 0.0, ga = 1.0, f = 0.0;
#pragma unroll
      for (int j = kTriSegMax - 2; j >= 0; --j) {
        const bool ok = j < len - 1;
        const double q = tri_recip(diag_at(lam, lo + j) + s2 * f);
        al = ok ? (bv[j] + s2 * al) * q : al;
        ga = ok ? s2 * ga * q : ga;
        f = ok ? -s2 * q : f;
      }
      const double be = lo > 0 ? -f : 0.0;
      // 3: reduced system of the segments' last rows, cyclic reduction across lanes
      const double al1 = __shfl_down(al, 1, P), be1 = __shfl_down(be, 1, P), ga1 = __shfl_down(ga, 1, P);
      const bool last = k == P - 1;
      double A = -gq;
      double Bq = last ? 1.0 : 1.0 + cp * be1;
      double C = last ? 0.0 : cp * ga1;
      double R = last ? dp : dp - cp * al1;
      for (int s = 1; s < P; s <<= 1) {
        const double Am = __shfl_up(A, s, P), Bm = __shfl_up(Bq, s, P), Cm = __shfl_up(C, s, P),
                     Rm = __shfl_up(R, s, P);
        const double Ap = __shfl_down(A, s, P), Bp = __shfl_down(Bq, s, P), Cp = __shfl_down(C, s, P),
                     Rp = __shfl_down(R, s, P);
        const bool hm = k >= s, hp = k + s < P;
        const double a = hm ? -A * tri_recip(Bm) : 0.0;
        const double c = hp ? -C * tri_recip(Bp) : 0.0;
        const double An = hm ? a * Am : 0.0;
        const double Cn = hp ? c * Cp : 0.0;
        Bq = Bq + (hm ? a * Cm : 0.0) + (hp ? c * Ap : 0.0);
        R = R + (hm ? a * Rm : 0.0) + (hp ? c * Rp : 0.0);
        A = An;
        C = Cn;
      }
      const double z = R * tri_recip(Bq);
      // every lane takes part in the shuffle: a lane outside the active set
      // of a cross-lane read supplies nothing
      const double zm = __shfl_up(z, 1, P);
      const double u = k > 0 ? zm : 0.0;
      // 4: the segment's rows from u and z (bv holds the forward values, then x)
      double d = u;
#pragma unroll
      for (int j = 0; j < kTriSegMax - 1; ++j) {
        bv[j] = (bv[j] + s2 * d) * rv[j];
        d = j < len - 1 ? bv[j] : d;
      }
      double x = z;
#pragma unroll
      for (int j = kTriSegMax - 2; j >= 0; --j) {
        x = j < len - 1 ? bv[j] + s2 * rv[j] * x : x;
        bv[j] = x;
      }
      if (active) {
        double* seg = row + tri_pad(lo);
#pragma unroll
        for (int j = 0; j < kTriSegMax; ++j) {
          if (j < len - 1) seg[tri_pad(lo + j) - tri_pad(lo)] = bv[j];
        }
        row[tri_pad(hi - 1)] = z;
      }
    }
    __syncthreads();
    {
      int i = threadIdx.x, ln = 0;
      while (i >= L) {
        i -= L;
        ++ln;
      }
#pragma unroll
      for (int r = 0; r < kTriLoadPer; ++r) {
        const int e = threadIdx.x + r * kTriThreads;
        if (e < tot) pl[base + e] = (T)buf[ln * Lp + tri_pad(i)];
        i += kTriThreads;
        while (i >= L) {
          i -= L;
          ++ln;
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace dot
