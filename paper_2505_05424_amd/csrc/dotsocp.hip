// Host driver and C ABI of the gfx950 inexact proximal ALM for dynamic OT
// (arXiv 2505.05424, Algorithm 2). See include/dotsocp.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/dotsocp.h"
#include "geometry.hpp"
#include "kernels_dct.hpp"
#include "kernels_update.hpp"

namespace dot {

template <typename T, int D>
__global__ void __launch_bounds__(256)
k_divergence(Geo g, const T* __restrict__ q, const T* __restrict__ al, const double* __restrict__ c_lo,
             const double* __restrict__ c_hi, double inv_sigma, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nb) return;
  const int t = (int)(i / g.stride[0]);
  const uint32_t xs = (uint32_t)(i % g.stride[0]);
  int x[kMaxAxes];
  spatial_coords<D>(g, xs, x);
  b[i] = divergence_at<T, D>(g, q, al, c_lo, c_hi, inv_sigma, t, xs, x);
}

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(DOT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

constexpr int kBlock = 256;
constexpr double kOmegaObstacle = 1e-6;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Device copy of the folded transform tables of one axis, in scalar type T.
template <typename T>
struct AxisDev {
  T* buf = nullptr;
  AxisTab<T> tab{};
};

}  // namespace
}  // namespace dot

using namespace dot;

struct dot_plan {
  Geo g{};
  int precision = DOT_FP64;
  int scalar_bytes = 8;
  int D = 0, K = 0;
  int n[4] = {0, 0, 0, 0};
  double tau = 1.9, sigma0 = 1.0, tol = 1e-6;
  int max_iter = 1000, cadence = 5, adapt = 1, gap0 = 10;
  double growth = 1.2;
  double vol = 1.0, c_norm2 = 0.0, d_norm2 = 0.0;
  int64_t nblocks = 0;  // blocks of kBlock over one plane
  // device constant tables
  double* sw_sp = nullptr;  // sqrt(omega/2) on spatial nodes
  double* om_sp = nullptr;  // omega on spatial nodes
  double* c_lo = nullptr;   // c~ at t = 0
  double* c_hi = nullptr;   // c~ at t = n0
  void* lam_other = nullptr;
  void* lam_last = nullptr;
  void* axis_buf[4] = {nullptr, nullptr, nullptr, nullptr};
  AxisTab<double> tab64[4]{};
  AxisTab<float> tab32[4]{};
  // scratch for step-level calls
  Ctl* step_ctl = nullptr;
  double* step_partials = nullptr;
  void* step_scratch = nullptr;  // FP32 transform plane (mixed precision)
  Ctl* host_ctl = nullptr;       // pinned
  // state layout (byte offsets): phi (FP64) | transform scratch (mixed only) |
  // q | q_new | alpha | beta | W (bulk scalar type) | control block | partials
  int n_planes = 0;  // bulk-type planes
  size_t off_phi = 0, off_scr = 0, off_q = 0, off_qn = 0, off_alpha = 0, off_beta = 0, off_w = 0;
  size_t ctl_offset = 0, partials_offset = 0, state_bytes = 0;
  int device = 0;
  // measurement hook: events around launches of one kernel class
  int prof_class = -1;
  std::vector<hipEvent_t> prof_ev;  // pairs (start, stop)
  size_t prof_used = 0;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
};

namespace {

template <typename T>
int upload(T** dst, const std::vector<T>& v) {
  HIP_OK(hipMalloc((void**)dst, std::max<size_t>(1, v.size()) * sizeof(T)));
  if (!v.empty()) HIP_OK(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return DOT_OK;
}

// Orthonormal DCT-II matrix entry C[k][j] = s_k cos(pi k (2j+1) / (2L)); the
// angle is reduced exactly in integers before the cosine.
double dct_entry(int L, int k, int j) {
  const long long m = ((long long)k * (2LL * j + 1)) % (4LL * L);
  const double s = (k == 0) ? std::sqrt(1.0 / L) : std::sqrt(2.0 / L);
  return s * std::cos(M_PI * (double)m / (2.0 * L));
}

int ksteps(int n_in) { return ((n_in + 3) / 4 + kU - 1) / kU * kU; }

// Fragment-major copy of an n_out x n_in matrix H in chunks of kU k-steps
// (see AxisTab), with one trailing zero chunk per row block.
template <typename T, typename F>
void frag_major(std::vector<T>& out, int n_out, int n_in, F H) {
  const int rb = (n_out + 15) / 16, nch = ksteps(n_in) / kU + 1;
  const size_t base = out.size();
  out.resize(base + (size_t)rb * nch * 64 * kU, T(0));
  for (int m = 0; m < rb; ++m)
    for (int ch = 0; ch < nch; ++ch)
      for (int l = 0; l < 64; ++l)
        for (int u = 0; u < kU; ++u) {
          const int st = ch * kU + u;
          const int r = m * 16 + l % 16, c = st * 4 + l / 16;
          if (r < n_out && c < n_in)
            out[base + (((size_t)m * nch + ch) * 64 + l) * kU + u] = (T)H(r, c);
        }
}

template <typename T>
int build_axis(dot_plan* P, int a, void** buf, AxisTab<T>* tab) {
  const int L = P->g.N[a];
  const int M = L / 2, ne = L - M, no = M;
  std::vector<T> fe, fo, ie, io;
  frag_major(fe, ne, ne, [&](int k, int j) { return dct_entry(L, 2 * k, j); });
  frag_major(fo, no, no, [&](int k, int j) { return dct_entry(L, 2 * k + 1, j); });
  frag_major(ie, ne, ne, [&](int j, int k) { return dct_entry(L, 2 * k, j); });
  frag_major(io, no, no, [&](int j, int k) { return dct_entry(L, 2 * k + 1, j); });
  std::vector<T> all;
  all.insert(all.end(), fe.begin(), fe.end());
  all.insert(all.end(), fo.begin(), fo.end());
  all.insert(all.end(), ie.begin(), ie.end());
  all.insert(all.end(), io.begin(), io.end());
  T* d = nullptr;
  int rc = upload(&d, all);
  if (rc) return rc;
  *buf = d;
  tab->fe = d;
  tab->fo = d + fe.size();
  tab->ie = d + fe.size() + fo.size();
  tab->io = d + fe.size() + fo.size() + ie.size();
  tab->L = L;
  tab->M = M;
  tab->ne = ne;
  tab->no = no;
  tab->rb_e = (ne + 15) / 16;
  tab->rb_o = (no + 15) / 16;
  tab->ks_e = ksteps(ne);
  tab->ks_o = ksteps(no);
  return DOT_OK;
}

// Waves per workgroup of a transform pass: enough for every work item of the
// axis to fit in MfmaOps<T>::kItems rounds.
template <typename T>
int pass_waves(int L) {
  const int M = L / 2, ne = L - M, no = M;
  const int items = 2 * ((ne + 15) / 16 + (no + 15) / 16);
  const int w = (items + MfmaOps<T>::kItems - 1) / MfmaOps<T>::kItems;
  return std::max(1, std::min(kMaxWaves, std::max(w, 4)));
}

template <typename T>
bool axis_fits(int L) {
  const int M = L / 2, ne = L - M, no = M;
  const int items = 2 * ((ne + 15) / 16 + (no + 15) / 16);
  return items <= MfmaOps<T>::kItems * kMaxWaves;
}

double axis_eig(int N, int nseg, int k) {
  const double s = std::sin(M_PI * k / (2.0 * N));
  return 4.0 * (double)nseg * (double)nseg * s * s;
}

template <typename T>
int build_eigs(dot_plan* P) {
  const Geo& g = P->g;
  const int D = P->D;
  const int64_t lines = g.nb / g.N[D];
  std::vector<T> other((size_t)lines), last((size_t)g.N[D]);
  for (int64_t c = 0; c < lines; ++c) {
    int64_t r = c;
    double s = 0.0;
    for (int a = D - 1; a >= 0; --a) {
      const int k = (int)(r % g.N[a]);
      r /= g.N[a];
      s += axis_eig(g.N[a], g.n[a], k);
    }
    other[(size_t)c] = (T)s;
  }
  for (int k = 0; k < g.N[D]; ++k) last[k] = (T)axis_eig(g.N[D], g.n[D], k);
  T* a = nullptr;
  T* b = nullptr;
  int rc = upload(&a, other);
  if (rc) return rc;
  rc = upload(&b, last);
  if (rc) return rc;
  P->lam_other = a;
  P->lam_last = b;
  return DOT_OK;
}

template <typename T>
T* at(void* state, size_t byte_off) {
  return reinterpret_cast<T*>(static_cast<char*>(state) + byte_off);
}

Ctl* state_ctl(void* state, const dot_plan* P) {
  return reinterpret_cast<Ctl*>(static_cast<char*>(state) + P->ctl_offset);
}

double* state_partials(void* state, const dot_plan* P) {
  return reinterpret_cast<double*>(static_cast<char*>(state) + P->partials_offset);
}

// Event bracket for the measurement hook; a no-op unless `cls` is selected.
struct ProfScope {
  dot_plan* P;
  hipStream_t st;
  bool on;
  hipEvent_t stop = nullptr;
  ProfScope(const dot_plan* Pc, int cls, hipStream_t s) : P(const_cast<dot_plan*>(Pc)), st(s), on(Pc->prof_class == cls) {
    if (!on) return;
    if (P->prof_used + 2 > P->prof_ev.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
          on = false;
          return;
        }
        P->prof_ev.push_back(e);
      }
    }
    hipEvent_t start = P->prof_ev[P->prof_used];
    stop = P->prof_ev[P->prof_used + 1];
    P->prof_used += 2;
    (void)hipEventRecord(start, st);
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord(stop, st);
  }
};

// Sum the recorded event pairs (the stream must be synchronised).
void prof_collect(dot_plan* P) {
  for (size_t k = 0; k + 1 < P->prof_used; k += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P->prof_ev[k], P->prof_ev[k + 1]) == hipSuccess) {
      P->prof_ms += ms;
      P->prof_launches += 1;
    }
  }
  P->prof_used = 0;
}

template <typename T>
const AxisTab<T>& tab_of(const dot_plan* P, int a);
template <>
const AxisTab<double>& tab_of<double>(const dot_plan* P, int a) { return P->tab64[a]; }
template <>
const AxisTab<float>& tab_of<float>(const dot_plan* P, int a) { return P->tab32[a]; }

template <typename T, int D, int KIND, int SRC, int DST>
int launch_pass(const dot_plan* P, int a, T* work, const T* q, const T* al, double* phi, const Ctl* ctl,
                double sigma, hipStream_t st) {
  const Geo& g = P->g;
  PassArgs pa;
  pa.inner = g.stride[a];
  pa.ncols = g.nb / g.N[a];
  const size_t smem = (size_t)g.N[a] * (kCW + 1) * sizeof(T);
  auto fn = k_axis_pass<T, D, KIND, SRC, DST>;
  // the LDS opt-in is per kernel and process; set it once to the device maximum
  static int smem_set = 0;
  if (!smem_set) {
    int max_smem = 0;
    HIP_OK(hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device));
    HIP_OK(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_smem));
    smem_set = 1;
  }
  const unsigned grid = (unsigned)((pa.ncols + kCW - 1) / kCW);
  const int cls = SRC != kSrcPlane ? DOT_K_DCT_FIRST
                  : KIND == kFwdScaleInv ? DOT_K_DCT_LAST
                  : KIND == kInv         ? DOT_K_DCT_INV
                                         : (a == 0 ? DOT_K_DCT_FIRST : DOT_K_DCT_MID);
  ProfScope ps(P, cls, st);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(pass_waves<T>(g.N[a]) * 64), smem, st, g, pa, tab_of<T>(P, a), work, q,
                     al, phi, P->c_lo, P->c_hi, (const T*)P->lam_other, (const T*)P->lam_last, ctl, sigma);
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

// The 2D+1 transform passes of one Poisson solve (a3 + a4): first pass on the
// time axis loads according to SRC, forward passes on the middle axes, the
// fused forward/scale/inverse pass on the last axis, inverse passes back to
// the time axis, which stores according to DST.
template <typename T, int D, int SRC, int DST>
int run_passes(const dot_plan* P, T* work, const T* q, const T* al, double* phi, const Ctl* ctl, double sigma,
               hipStream_t st) {
  int rc;
  if ((rc = launch_pass<T, D, kFwd, SRC, kDstPlane>(P, 0, work, q, al, phi, ctl, sigma, st))) return rc;
  for (int a = 1; a < D; ++a)
    if ((rc = launch_pass<T, D, kFwd, kSrcPlane, kDstPlane>(P, a, work, q, al, phi, ctl, sigma, st))) return rc;
  if ((rc = launch_pass<T, D, kFwdScaleInv, kSrcPlane, kDstPlane>(P, D, work, q, al, phi, ctl, sigma, st))) return rc;
  for (int a = D - 1; a >= 1; --a)
    if ((rc = launch_pass<T, D, kInv, kSrcPlane, kDstPlane>(P, a, work, q, al, phi, ctl, sigma, st))) return rc;
  return launch_pass<T, D, kInv, kSrcPlane, DST>(P, 0, work, q, al, phi, ctl, sigma, st);
}

// Poisson solve inside an iteration. FP64: the transforms run in place on
// phi. Mixed: the FP32 transforms solve A^*A dphi = b - A^*A phi on the
// scratch plane and the last pass adds dphi to the FP64 phi.
template <typename T, int D>
int poisson_iter(const dot_plan* P, double* phi, T* scratch, const T* q, const T* al, const Ctl* ctl, hipStream_t st) {
  if constexpr (std::is_same<T, double>::value)
    return run_passes<double, D, kSrcDivergence, kDstPlane>(P, phi, q, al, phi, ctl, 0.0, st);
  else
    return run_passes<T, D, kSrcDefect, kDstPhiAdd>(P, scratch, q, al, phi, ctl, 0.0, st);
}

// Poisson solve of the step-level calls: from (q, alpha, sigma) if q is given,
// else from the right-hand side already in phi; result in phi.
template <typename T, int D>
int poisson_step(const dot_plan* P, double* phi, const T* q, const T* al, double sigma, hipStream_t st) {
  if constexpr (std::is_same<T, double>::value) {
    if (q) return run_passes<double, D, kSrcDivergence, kDstPlane>(P, phi, q, al, phi, nullptr, sigma, st);
    return run_passes<double, D, kSrcPlane, kDstPlane>(P, phi, q, al, phi, nullptr, sigma, st);
  } else {
    T* scr = (T*)P->step_scratch;
    if (q) return run_passes<T, D, kSrcDivergence, kDstPhiSet>(P, scr, q, al, phi, nullptr, sigma, st);
    return run_passes<T, D, kSrcPlaneF64, kDstPhiSet>(P, scr, q, al, phi, nullptr, sigma, st);
  }
}

unsigned grid_nb(const dot_plan* P) { return (unsigned)P->nblocks; }

template <typename T, int D>
int run_update(const dot_plan* P, const double* phi, const T* q, T* alpha, T* beta, T* qn, T* W, Ctl* ctl,
               double* partials, int check, hipStream_t st) {
  const Geo& g = P->g;
  {
    ProfScope ps(P, DOT_K_CONE, st);
    hipLaunchKernelGGL((k_cone_q0<T, D>), dim3(grid_nb(P)), dim3(kBlock), 0, st, g, phi, q, alpha, beta,
                       P->sw_sp, qn, W, ctl);
  }
  HIP_OK(hipGetLastError());
  {
    ProfScope ps(P, DOT_K_QD, st);
    hipLaunchKernelGGL((k_qd<T, D>), dim3(grid_nb(P)), dim3(kBlock), 0, st, g, phi, alpha, P->om_sp, qn, W, ctl);
  }
  HIP_OK(hipGetLastError());
  {
    ProfScope ps(P, DOT_K_BETA, st);
    hipLaunchKernelGGL((k_beta<T, D>), dim3(grid_nb(P)), dim3(kBlock), 0, st, g, q, qn, beta, P->sw_sp, ctl,
                       partials, check);
  }
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

FinArgs fin_args(const dot_plan* P) {
  FinArgs fa;
  fa.vol = P->vol;
  fa.c_norm2 = P->c_norm2;
  fa.d_norm2 = P->d_norm2;
  fa.nblocks = P->nblocks;
  return fa;
}

template <typename T, int D>
int run_check(const dot_plan* P, const double* phi, const T* q, const T* alpha, const T* beta, Ctl* ctl,
              double* partials, int update_ctl, hipStream_t st) {
  const Geo& g = P->g;
  {
    ProfScope ps(P, DOT_K_RESID, st);
    hipLaunchKernelGGL((k_resid<T, D>), dim3(grid_nb(P)), dim3(kBlock), 0, st, g, phi, q, alpha, beta, P->om_sp,
                       P->sw_sp, P->c_lo, P->c_hi, update_ctl ? ctl : nullptr, partials);
  }
  HIP_OK(hipGetLastError());
  {
    ProfScope ps(P, DOT_K_FINAL, st);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, fin_args(P), partials, ctl, update_ctl);
  }
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

template <typename T, int D>
int run_iters(dot_plan* P, void* state, int max_iters, hipStream_t st, dot_result* res) {
  Ctl* ctl = state_ctl(state, P);
  double* partials = state_partials(state, P);
  HIP_OK(hipMemcpyAsync(P->host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  const int iter0 = P->host_ctl->iter;
  int stopped = P->host_ctl->stop;
  double* phi = at<double>(state, P->off_phi);
  T* scr = at<T>(state, P->off_scr);
  T* qa = at<T>(state, P->off_q);
  T* qb = at<T>(state, P->off_qn);
  T* alpha = at<T>(state, P->off_alpha);
  T* beta = at<T>(state, P->off_beta);
  T* W = at<T>(state, P->off_w);
  const int poll = 40;
  int rc;
  for (int j = 0; j < max_iters && !stopped; ++j) {
    const int it = iter0 + j;
    T* cur = (it % 2 == 0) ? qa : qb;
    T* nxt = (it % 2 == 0) ? qb : qa;
    if ((rc = poisson_iter<T, D>(P, phi, scr, cur, alpha, ctl, st))) return rc;
    const int check = ((it + 1) % P->cadence) == 0;
    if ((rc = run_update<T, D>(P, phi, cur, alpha, beta, nxt, W, ctl, partials, check, st))) return rc;
    if (check && (rc = run_check<T, D>(P, phi, nxt, alpha, beta, ctl, partials, 1, st))) return rc;
    if ((j + 1) % poll == 0 || j + 1 == max_iters) {
      HIP_OK(hipMemcpyAsync(P->host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      prof_collect(P);
      stopped = P->host_ctl->stop;
    }
  }
  HIP_OK(hipMemcpyAsync(P->host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  prof_collect(P);
  if (res) {
    const Ctl& c = *P->host_ctl;
    res->objective = c.objective;
    res->dual_objective = c.dual_objective;
    res->eta_dot = c.eta[0];
    res->eta_p = c.eta[1];
    res->eta_d = c.eta[2];
    res->eta_c = c.eta[3];
    res->eta_p_soc = c.eta[4];
    res->eta_d_soc = c.eta[5];
    res->sigma = c.sigma;
    res->iters = c.iter;
    res->checks = c.checks;
    res->sigma_changes = c.sigma_changes;
    res->term = c.stop == 1 ? DOT_CONVERGED : (c.stop == 3 ? DOT_DIVERGED : DOT_MAXITER);
  }
  return DOT_OK;
}

// Dispatch on (scalar type, D).
template <template <typename, int> class F, typename... A>
int dispatch(const dot_plan* P, A&&... args) {
  if (P->precision == DOT_FP64) {
    switch (P->D) {
      case 1: return F<double, 1>::run(std::forward<A>(args)...);
      case 2: return F<double, 2>::run(std::forward<A>(args)...);
      case 3: return F<double, 3>::run(std::forward<A>(args)...);
    }
  } else {
    switch (P->D) {
      case 1: return F<float, 1>::run(std::forward<A>(args)...);
      case 2: return F<float, 2>::run(std::forward<A>(args)...);
      case 3: return F<float, 3>::run(std::forward<A>(args)...);
    }
  }
  return fail(DOT_EINVAL, "unsupported D");
}

template <typename T, int D>
struct RunF {
  static int run(dot_plan* P, void* state, int max_iters, hipStream_t st, dot_result* res) {
    return run_iters<T, D>(P, state, max_iters, st, res);
  }
};

template <typename T, int D>
struct DivF {
  static int run(dot_plan* P, const void* q, const void* al, double sigma, void* b, hipStream_t st) {
    hipLaunchKernelGGL((k_divergence<T, D>), dim3(grid_nb(P)), dim3(kBlock), 0, st, P->g, (const T*)q,
                       (const T*)al, P->c_lo, P->c_hi, 1.0 / sigma, (double*)b);
    HIP_OK(hipGetLastError());
    return DOT_OK;
  }
};

template <typename T, int D>
struct PoissonF {
  static int run(dot_plan* P, void* b, const void* q, const void* al, double sigma, hipStream_t st) {
    return poisson_step<T, D>(P, (double*)b, (const T*)q, (const T*)al, sigma, st);
  }
};

template <typename T, int D>
struct ConeF {
  static int run(dot_plan* P, const void* q, const void* beta, double sigma, void* z, hipStream_t st) {
    hipLaunchKernelGGL((k_cone_out<T, D>), dim3(grid_nb(P)), dim3(kBlock), 0, st, P->g, (const T*)q,
                       (const T*)beta, P->sw_sp, 1.0 / sigma, (T*)z);
    HIP_OK(hipGetLastError());
    return DOT_OK;
  }
};

template <typename T, int D>
struct UpdateF {
  static int run(dot_plan* P, const void* phi, const void* q, void* alpha, void* beta, double sigma,
                 double tau, void* qn, void* W, hipStream_t st) {
    Ctl h{};
    h.sigma = sigma;
    h.tau = tau;
    h.stop = 0;
    HIP_OK(hipMemcpyAsync(P->step_ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, st));
    int rc = run_update<T, D>(P, (const double*)phi, (const T*)q, (T*)alpha, (T*)beta, (T*)qn, (T*)W, P->step_ctl,
                              P->step_partials, 0, st);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(st));
    return DOT_OK;
  }
};

template <typename T, int D>
struct ResidF {
  static int run(dot_plan* P, const void* phi, const void* z, const void* q, const void* alpha,
                 const void* beta, hipStream_t st) {
    hipLaunchKernelGGL((k_zres<T, D>), dim3(grid_nb(P)), dim3(kBlock), 0, st, P->g, (const T*)z, (const T*)q,
                       P->sw_sp, P->step_partials);
    HIP_OK(hipGetLastError());
    return run_check<T, D>(P, (const double*)phi, (const T*)q, (const T*)alpha, (const T*)beta, P->step_ctl,
                           P->step_partials, 0, st);
  }
};

int validate(const dot_problem* p) {
  if (!p) return fail(DOT_EINVAL, "null problem");
  if (p->D < 1 || p->D > 3) return fail(DOT_EINVAL, "D must be 1, 2 or 3");
  for (int d = 0; d <= p->D; ++d)
    if (p->n[d] < 1 || p->n[d] > 4096) return fail(DOT_EINVAL, "segment counts must be in [1, 4096]");
  if (!p->rho0 || !p->rho1) return fail(DOT_EINVAL, "rho0 and rho1 are required");
  if (p->precision != DOT_FP64 && p->precision != DOT_MIXED) return fail(DOT_EINVAL, "unknown precision");
  if (p->max_iter < 0) return fail(DOT_EINVAL, "max_iter must be >= 0");
  if (p->tau < 0 || p->tau >= 2) return fail(DOT_EINVAL, "tau must be in (0, 2) (0 selects 1.9)");
  if (p->sigma0 < 0 || !std::isfinite(p->sigma0)) return fail(DOT_EINVAL, "sigma0 must be > 0 (0 selects 1)");
  if (p->check_every < 0) return fail(DOT_EINVAL, "check_every must be >= 0");
  if (p->sigma_gap0 < 0 || p->sigma_growth < 0) return fail(DOT_EINVAL, "sigma schedule must be >= 0");
  int64_t nx = 1;
  for (int d = 1; d <= p->D; ++d) nx *= (int64_t)p->n[d] + 1;
  double m0 = 0.0, m1 = 0.0;
  for (int64_t i = 0; i < nx; ++i) {
    const double a = p->rho0[i], b = p->rho1[i];
    if (!std::isfinite(a) || !std::isfinite(b)) return fail(DOT_EINVAL, "rho0/rho1 must be finite");
    if (a < 0 || b < 0) return fail(DOT_EINVAL, "rho0/rho1 must be non-negative");
    m0 += a;
    m1 += b;
  }
  if (!(m0 > 0)) return fail(DOT_EINVAL, "rho0 must have positive total mass");
  if (std::fabs(m0 - m1) > 1e-12 * m0) return fail(DOT_EINVAL, "rho0 and rho1 must have equal total mass");
  return DOT_OK;
}

}  // namespace

extern "C" {

const char* dot_last_error(void) { return g_err.c_str(); }

void dot_plan_destroy(dot_plan* P) {
  if (!P) return;
  for (auto e : P->prof_ev) (void)hipEventDestroy(e);
  (void)hipFree(P->sw_sp);
  (void)hipFree(P->om_sp);
  (void)hipFree(P->c_lo);
  (void)hipFree(P->c_hi);
  (void)hipFree(P->lam_other);
  (void)hipFree(P->lam_last);
  for (auto* b : P->axis_buf) (void)hipFree(b);
  (void)hipFree(P->step_ctl);
  (void)hipFree(P->step_partials);
  (void)hipFree(P->step_scratch);
  (void)hipHostFree(P->host_ctl);
  delete P;
}

int dot_plan_create(const dot_problem* p, dot_plan** out) {
  if (!out) return fail(DOT_EINVAL, "null output pointer");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  std::unique_ptr<dot_plan, void (*)(dot_plan*)> P(new (std::nothrow) dot_plan(), dot_plan_destroy);
  if (!P) return fail(DOT_ENOMEM, "host allocation failed");
  const int D = p->D;
  P->D = D;
  P->K = 4 * D + 2;
  P->precision = p->precision;
  P->scalar_bytes = p->precision == DOT_FP64 ? 8 : 4;
  P->tau = p->tau > 0 ? p->tau : 1.9;
  P->sigma0 = p->sigma0 > 0 ? p->sigma0 : 1.0;
  P->tol = p->tol;
  P->max_iter = p->max_iter;
  P->cadence = p->check_every > 0 ? p->check_every : 5;
  P->adapt = p->adapt_sigma;
  P->gap0 = p->sigma_gap0 > 0 ? p->sigma_gap0 : 10;
  P->growth = p->sigma_growth > 0 ? p->sigma_growth : 1.2;
  HIP_OK(hipGetDevice(&P->device));
  Geo& g = P->g;
  g.D = D;
  g.K = P->K;
  for (int a = 0; a < kMaxAxes; ++a) {
    g.n[a] = a <= D ? p->n[a] : 0;
    g.N[a] = a <= D ? p->n[a] + 1 : 1;
    g.inv_h[a] = a <= D ? (double)p->n[a] : 0.0;
    P->n[a] = g.n[a];
  }
  int64_t s = 1;
  for (int a = kMaxAxes - 1; a >= 0; --a) {
    g.stride[a] = (a <= D) ? s : 0;
    if (a <= D) s *= g.N[a];
  }
  g.nb = s;
  g.nx = g.nb / g.N[0];
  // kernels index planes with 32-bit offsets up to a few planes apart
  if (g.nb > ((int64_t)1 << 28)) return fail(DOT_EINVAL, "a plane must hold at most 2^28 nodes");
  // LDS capacity of one transform tile
  int max_smem = 0;
  HIP_OK(hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device));
  for (int a = 0; a <= D; ++a) {
    const size_t need = (size_t)g.N[a] * (kCW + 1) * P->scalar_bytes;
    const bool fits = P->precision == DOT_FP64 ? axis_fits<double>(g.N[a]) : axis_fits<float>(g.N[a]);
    if ((int64_t)need > max_smem || !fits)
      return fail(DOT_EINVAL, "axis of " + std::to_string(g.N[a]) + " nodes exceeds the transform tile capacity");
  }
  // problem data
  const int64_t nx = g.nx;
  double vol = 1.0;
  for (int a = 0; a <= D; ++a) vol /= (double)g.n[a];
  P->vol = vol;
  std::vector<double> clo(nx), chi(nx), om(nx), sw(nx);
  double c2 = 0.0;
  for (int64_t i = 0; i < nx; ++i) {
    clo[i] = p->rho0[i] / vol;
    chi[i] = -p->rho1[i] / vol;
    c2 += clo[i] * clo[i] + chi[i] * chi[i];
    om[i] = (p->mask && p->mask[i]) ? kOmegaObstacle : 1.0;
    sw[i] = std::sqrt(om[i] / 2.0);
  }
  P->c_norm2 = c2;
  P->d_norm2 = 2.0 * (double)g.n[0] * (double)nx;
  if ((rc = upload(&P->c_lo, clo)) || (rc = upload(&P->c_hi, chi)) || (rc = upload(&P->om_sp, om)) ||
      (rc = upload(&P->sw_sp, sw)))
    return rc;
  for (int a = 0; a <= D; ++a) {
    rc = P->precision == DOT_FP64 ? build_axis<double>(P.get(), a, &P->axis_buf[a], &P->tab64[a])
                                  : build_axis<float>(P.get(), a, &P->axis_buf[a], &P->tab32[a]);
    if (rc) return rc;
  }
  rc = P->precision == DOT_FP64 ? build_eigs<double>(P.get()) : build_eigs<float>(P.get());
  if (rc) return rc;
  // state layout: phi (FP64) | scratch (mixed) | q (D+1) | q_new (D+1) | alpha (D+1) | beta (K) | W (4D) |
  // control block | partials
  const size_t pb = (size_t)g.nb * P->scalar_bytes;
  P->off_phi = 0;
  P->off_scr = align256((size_t)g.nb * sizeof(double));
  P->off_q = P->off_scr + (P->precision == DOT_MIXED ? align256(pb) : 0);
  P->off_qn = P->off_q + (size_t)(D + 1) * pb;
  P->off_alpha = P->off_qn + (size_t)(D + 1) * pb;
  P->off_beta = P->off_alpha + (size_t)(D + 1) * pb;
  P->off_w = P->off_beta + (size_t)P->K * pb;
  P->n_planes = 3 * (D + 1) + P->K + 4 * D;
  P->nblocks = (g.nb + kBlock - 1) / kBlock;
  P->ctl_offset = align256(P->off_w + (size_t)(4 * D) * pb);
  P->partials_offset = P->ctl_offset + align256(sizeof(Ctl));
  P->state_bytes = P->partials_offset + align256((size_t)P->nblocks * kNumSums * sizeof(double));
  if (P->precision == DOT_MIXED) HIP_OK(hipMalloc(&P->step_scratch, pb));
  HIP_OK(hipMalloc((void**)&P->step_ctl, sizeof(Ctl)));
  HIP_OK(hipMalloc((void**)&P->step_partials, (size_t)P->nblocks * kNumSums * sizeof(double)));
  HIP_OK(hipMemset(P->step_partials, 0, (size_t)P->nblocks * kNumSums * sizeof(double)));
  HIP_OK(hipHostMalloc((void**)&P->host_ctl, sizeof(Ctl), hipHostMallocDefault));
  *out = P.release();
  return DOT_OK;
}

int dot_plan_get_info(const dot_plan* P, dot_plan_info* o) {
  if (!P || !o) return fail(DOT_EINVAL, "null argument");
  o->D = P->D;
  o->K = P->K;
  for (int a = 0; a < 4; ++a) o->n[a] = P->n[a];
  o->nb = P->g.nb;
  o->scalar_bytes = P->scalar_bytes;
  o->n_planes = P->n_planes;
  o->state_bytes = P->state_bytes;
  o->off_phi = P->off_phi;
  o->off_scratch = P->off_scr;
  o->off_q = P->off_q;
  o->off_qn = P->off_qn;
  o->off_alpha = P->off_alpha;
  o->off_beta = P->off_beta;
  o->off_w = P->off_w;
  return DOT_OK;
}

int dot_state_reset(dot_plan* P, void* state, void* stream) {
  if (!P || !state) return fail(DOT_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIP_OK(hipMemsetAsync(state, 0, P->ctl_offset, st));
  Ctl h{};
  h.sigma = P->sigma0;
  h.tau = P->tau;
  h.tol = P->tol;
  h.iter = 0;
  h.stop = 0;
  h.next_update = P->gap0;
  h.gap = P->gap0;
  h.growth = P->growth;
  h.adapt = P->adapt;
  h.cadence = P->cadence;
  *P->host_ctl = h;
  HIP_OK(hipMemcpyAsync(state_ctl(state, P), P->host_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  return DOT_OK;
}

int dot_run(dot_plan* P, void* state, int32_t max_iters, void* stream, dot_result* res) {
  if (!P || !state || max_iters < 0) return fail(DOT_EINVAL, "bad argument");
  return dispatch<RunF>(P, P, state, (int)max_iters, (hipStream_t)stream, res);
}

int dot_extract(dot_plan* P, const void* state, double* rho_out, double* m_out, void* stream) {
  if (!P || !state) return fail(DOT_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const Geo& g = P->g;
  const size_t sb = P->scalar_bytes;
  std::vector<unsigned char> buf(g.nb * sb);
  auto get = [&](size_t i) -> double {
    return sb == 8 ? reinterpret_cast<const double*>(buf.data())[i] : reinterpret_cast<const float*>(buf.data())[i];
  };
  const char* base = static_cast<const char*>(state);
  if (rho_out) {
    HIP_OK(hipMemcpyAsync(buf.data(), base + P->off_alpha, g.nb * sb, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const int64_t ncell = (int64_t)g.n[0] * g.nx;
    for (int64_t i = 0; i < ncell; ++i) rho_out[i] = get(i);
  }
  if (m_out) {
    size_t o = 0;
    for (int d = 1; d <= P->D; ++d) {
      HIP_OK(hipMemcpyAsync(buf.data(), base + P->off_alpha + (size_t)d * g.nb * sb, g.nb * sb,
                            hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      for (int64_t i = 0; i < g.nb; ++i) {
        int64_t r = i / g.stride[d];
        const int xd = (int)(r % g.N[d]);
        if (xd < g.n[d]) m_out[o++] = get(i);
      }
    }
  }
  return DOT_OK;
}

int dot_step_divergence(dot_plan* P, const void* q, const void* alpha, double sigma, void* b, void* stream) {
  if (!P || !q || !alpha || !b || !(sigma > 0)) return fail(DOT_EINVAL, "bad argument");
  return dispatch<DivF>(P, P, q, alpha, sigma, b, (hipStream_t)stream);
}

int dot_step_poisson(dot_plan* P, void* b, void* stream) {
  if (!P || !b) return fail(DOT_EINVAL, "bad argument");
  return dispatch<PoissonF>(P, P, b, (const void*)nullptr, (const void*)nullptr, 1.0, (hipStream_t)stream);
}

int dot_step_rhs_poisson(dot_plan* P, const void* q, const void* alpha, double sigma, void* phi, void* stream) {
  if (!P || !q || !alpha || !phi || !(sigma > 0)) return fail(DOT_EINVAL, "bad argument");
  return dispatch<PoissonF>(P, P, phi, q, alpha, sigma, (hipStream_t)stream);
}

int dot_step_cone(dot_plan* P, const void* q, const void* beta, double sigma, void* z, void* stream) {
  if (!P || !q || !beta || !z || !(sigma > 0)) return fail(DOT_EINVAL, "bad argument");
  return dispatch<ConeF>(P, P, q, beta, sigma, z, (hipStream_t)stream);
}

int dot_step_update(dot_plan* P, const void* phi, const void* q, void* alpha, void* beta, double sigma, double tau,
                    void* q_out, void* w_scratch, void* stream) {
  if (!P || !phi || !q || !alpha || !beta || !q_out || !w_scratch || !(sigma > 0) || !(tau > 0))
    return fail(DOT_EINVAL, "bad argument");
  return dispatch<UpdateF>(P, P, phi, q, alpha, beta, sigma, tau, q_out, w_scratch, (hipStream_t)stream);
}

int dot_step_residuals(dot_plan* P, const void* phi, const void* z, const void* q, const void* alpha,
                       const void* beta, dot_result* res, void* stream) {
  if (!P || !phi || !z || !q || !alpha || !beta || !res) return fail(DOT_EINVAL, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = dispatch<ResidF>(P, P, phi, z, q, alpha, beta, st);
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(P->host_ctl, P->step_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  const Ctl& c = *P->host_ctl;
  std::memset(res, 0, sizeof(*res));
  res->objective = c.objective;
  res->dual_objective = c.dual_objective;
  res->eta_dot = c.eta[0];
  res->eta_p = c.eta[1];
  res->eta_d = c.eta[2];
  res->eta_c = c.eta[3];
  res->eta_p_soc = c.eta[4];
  res->eta_d_soc = c.eta[5];
  return DOT_OK;
}

int dot_profile_select(dot_plan* P, int32_t kernel_class) {
  if (!P || kernel_class < -1 || kernel_class > DOT_K_FINAL) return fail(DOT_EINVAL, "bad kernel class");
  P->prof_class = kernel_class;
  P->prof_used = 0;
  P->prof_ms = 0.0;
  P->prof_launches = 0;
  return DOT_OK;
}

int dot_profile_read(dot_plan* P, double* total_ms, int64_t* launches) {
  if (!P) return fail(DOT_EINVAL, "null plan");
  if (total_ms) *total_ms = P->prof_ms;
  if (launches) *launches = P->prof_launches;
  P->prof_ms = 0.0;
  P->prof_launches = 0;
  return DOT_OK;
}

int dot_solve(const dot_problem* p, double* rho_out, double* m_out, dot_result* res) {
  dot_plan* P = nullptr;
  int rc = dot_plan_create(p, &P);
  if (rc) return rc;
  void* state = nullptr;
  hipError_t e = hipMalloc(&state, P->state_bytes);
  if (e != hipSuccess) {
    dot_plan_destroy(P);
    return fail(DOT_ENOMEM, "state allocation failed");
  }
  rc = dot_state_reset(P, state, nullptr);
  if (!rc) rc = dot_run(P, state, p->max_iter, nullptr, res);
  if (!rc) rc = dot_extract(P, state, rho_out, m_out, nullptr);
  (void)hipFree(state);
  dot_plan_destroy(P);
  return rc;
}

}  // extern "C"
