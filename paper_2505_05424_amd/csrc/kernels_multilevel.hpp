// Multilevel initialisation (the multilevel strategy of the implementation
// details of Sec. 5.3 and of the experiments of Sec. 5.4): an iterate on a
// grid with half the segments per axis is interpolated linearly to the finer
// grid and used as the initial point there.
//
// One lane per fine plane entry. Along each axis the entry sits at a node
// (x / n) or at a staggered point ((s + 1/2) / n); its position in coarse
// index units is u = x / 2 (nodes) or u = (s - 1/2) / 2 (staggered), clamped
// to the coarse index range (constant extension beyond the ends). The value
// is the tensor product of the per-axis linear weights over the 2^(D+1)
// surrounding coarse entries.
#pragma once
#include "geometry.hpp"

namespace dot {

template <typename T, int D>
__global__ void __launch_bounds__(256)
kb_prolong(const Geo gc, const Geo gf, const T* __restrict__ src, T* __restrict__ dst, int kind) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= gf.nb) return;
  const size_t plane = blockIdx.y;
  gp<const T> s = glob(src) + plane * (size_t)gc.nb;
  gp<T> o = glob(dst) + plane * (size_t)gf.nb;
  int lo[kMaxAxes], hi[kMaxAxes];
  double w[kMaxAxes];
  int64_t r = i;
  bool inside = true;
#pragma unroll
  for (int a = D; a >= 0; --a) {
    const int x = (int)(r % gf.N[a]);
    r /= gf.N[a];
    const bool stag = (kind >> a) & 1;
    const int last = stag ? gc.n[a] - 1 : gc.n[a];  // last coarse index on this axis
    if (stag && x >= gf.n[a]) inside = false;          // padding entry of a staggered axis
    const double u = stag ? 0.5 * ((double)x - 0.5) : 0.5 * (double)x;
    if (u <= 0.0) {
      lo[a] = hi[a] = 0;
      w[a] = 0.0;
    } else if (u >= (double)last) {
      lo[a] = hi[a] = last;
      w[a] = 0.0;
    } else {
      lo[a] = (int)u;
      hi[a] = lo[a] + 1;
      w[a] = u - (double)lo[a];
    }
  }
  if (!inside) {
    o[i] = T(0);
    return;
  }
  double v = 0.0;
#pragma unroll
  for (int corner = 0; corner < (1 << (D + 1)); ++corner) {
    double wt = 1.0;
    int64_t ci = 0;
#pragma unroll
    for (int a = 0; a <= D; ++a) {
      const bool up = (corner >> a) & 1;
      wt *= up ? w[a] : 1.0 - w[a];
      ci += (int64_t)(up ? hi[a] : lo[a]) * gc.stride[a];
    }
    if (wt != 0.0) v += wt * (double)s[ci];
  }
  o[i] = (T)v;
}

// FP32 planes of a mixed-precision state widened to FP64 (exact), for
// continuing a solve in FP64.
__global__ void __launch_bounds__(256) kb_widen(const float* __restrict__ src, double* __restrict__ dst, int64_t n) {
  gp<const float> s = glob(src);
  gp<double> o = glob(dst);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    o[i] = (double)s[i];
}

}  // namespace dot
