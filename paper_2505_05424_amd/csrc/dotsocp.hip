// Host driver and C ABI of the gfx950 inexact proximal ALM for dynamic OT
// (arXiv 2505.05424, Algorithm 2). See include/dotsocp.h for the contract.
//
// Every iteration is a fixed sequence of launches: the right-hand side sweep
// (or nothing, when the previous iteration's beta launch computed it), 2D+1
// cosine-transform passes (the last-axis one a tridiagonal solve for long last
// axes), three update sweeps, and at residual checks two reduction kernels.
// Each launch covers all instances of an executor: one plan (dot_run, a batch
// of one) or a batch (dot_batch_run), through the descriptor arrays of
// batch.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/dotsocp.h"
#include "batch.hpp"
#include "geometry.hpp"
#include "kernels_dct.hpp"
#include "kernels_multilevel.hpp"
#include "kernels_update.hpp"

using namespace dot;

namespace {

thread_local std::string g_err;

// Graph captures and the calls that allocate, free or otherwise synchronise
// the whole device are serialised across host threads: such a call from one
// thread while another thread captures can invalidate that capture (the
// serving driver steps one context per host thread). Recursive, since entry
// points that hold it call others that take it.
std::recursive_mutex g_dev_mu;
using DevLock = std::lock_guard<std::recursive_mutex>;

// Captures still to fail on purpose (dot_test_fail_captures).
std::atomic<int> g_fail_captures{0};

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

constexpr double kOmegaObstacle = 1e-6;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Events around launches of one kernel class (the measurement hook).
struct Prof {
  int cls = -1;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  size_t used = 0;
  double ms = 0.0;
  int64_t launches = 0;
  ~Prof() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  void collect() {
    for (size_t k = 0; k + 1 < used; k += 2) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) == hipSuccess) {
        ms += t;
        launches += 1;
      }
    }
    used = 0;
  }
};

struct ProfScope {
  Prof* pr;
  hipStream_t st;
  bool on;
  hipEvent_t stop = nullptr;
  ProfScope(Prof* p, int cls, hipStream_t s) : pr(p), st(s), on(p && p->cls == cls) {
    if (!on) return;
    if (pr->used + 2 > pr->ev.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        // timing-only events: no system-scope fence (cache writeback and
        // invalidate) when they complete, which would add to each bracket
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
          on = false;
          return;
        }
        pr->ev.push_back(e);
      }
    }
    hipEvent_t start = pr->ev[pr->used];
    stop = pr->ev[pr->used + 1];
    pr->used += 2;
    (void)hipEventRecord(start, st);
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord(stop, st);
  }
};

// A captured block of kGraphIters iterations starting at a multiple of 10
// (the parity of q and the positions of the residual checks repeat with
// period 10, so one graph serves every such block), and one of the iterations
// between two polls of the control blocks (four such blocks; one graph launch
// per poll instead of four: 2D 32x64^2 FP64 51.3 -> 50.9 us per iteration).
// Capture happens only after plain launches have run once (one-time kernel
// attribute calls stay outside any capture).
constexpr int kGraphIters = 10;
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipGraphExec_t exec_poll = nullptr;  // the iterations between two polls
  hipStream_t cap = nullptr;       // private capture stream (default priority)
  hipStream_t cap_side = nullptr;  // second branch of the captured iterations
  hipStream_t side = nullptr;      // second branch of plain launches
  hipEvent_t fork = nullptr, join = nullptr;  // branch points (no timing)
  bool enabled = true;
  bool warm = false;
  ~GraphCache() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (exec_poll) (void)hipGraphExecDestroy(exec_poll);
    if (cap) (void)hipStreamDestroy(cap);
    if (cap_side) (void)hipStreamDestroy(cap_side);
    if (side) (void)hipStreamDestroy(side);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
  }
};

// Drops the captured iterations (the next run captures them anew, e.g. after
// the launch layout changed).
void drop_graph(GraphCache& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
  if (g.exec_poll) (void)hipGraphExecDestroy(g.exec_poll);
  g.exec_poll = nullptr;
}

// Transform schedule of an executor: tile width (lines per workgroup) and
// waves per workgroup of the passes over each axis; 0 takes the launch-size
// rule. Neither changes a computed value (each line's products run in one
// wave in a fixed order whatever the tile and wave count).
struct Sched {
  int cw[kMaxAxes] = {0, 0, 0, 0};
  int waves[kMaxAxes] = {0, 0, 0, 0};
  bool tuned = false;   // set by the autotuner (measured), not by the rule or the caller
  int candidates = 0;   // schedules the autotuner timed
  double us = 0.0;      // one transform sequence with this schedule (autotuner), us
  double us_rule = 0.0; // the same with the rule's schedule
};

}  // namespace

struct dot_plan {
  Geo g{};
  int precision = DOT_FP64;
  int scalar_bytes = 8;
  int D = 0, K = 0;
  int n[4] = {0, 0, 0, 0};
  double tau = 1.9, sigma0 = 30.0, tol = 1e-6;
  int max_iter = 1000, cadence = 5, adapt = 1, gap0 = 10;
  double growth = 1.2;
  double time_limit = 0.0;  // seconds per run call (0: none)
  double vol = 1.0, c_norm2 = 0.0, d_norm2 = 0.0;
  int64_t nblocks = 0;       // workgroups of one node sweep (g.nsweep)
  int64_t partial_rows = 0;  // capacity of the partial-sum rows (nsweep at one slice per workgroup)
  int64_t lines[kMaxAxes] = {0, 0, 0, 0};  // lines per axis (nb / N[a])
  bool wide_ok[kMaxAxes] = {true, true, true, true};  // the axis fits a tile of kCW lines
  bool mid_ok[kMaxAxes] = {true, true, true, true};   // a tile of kCWMid lines fits in kMidLds
  bool tri = false;      // the last axis is solved by tridiagonal elimination
  void* step_cbuf = nullptr;  // c' plane of the tridiagonal solve for step-level calls
  Sched sched;                // transform schedule of this plan's own launches
  // device constant tables
  double* sw_sp = nullptr;  // sqrt(omega/2) on spatial nodes
  double* om_sp = nullptr;  // omega on spatial nodes
  double* c_lo = nullptr;   // c~ at t = 0
  double* c_hi = nullptr;   // c~ at t = n0
  void* lam_other = nullptr;
  void* lam_last = nullptr;
  void* axis_buf[kMaxAxes] = {nullptr, nullptr, nullptr, nullptr};
  AxisTab<double> tab64[kMaxAxes]{};
  AxisTab<float> tab32[kMaxAxes]{};
  // single-instance executor resources
  void* d_inst = nullptr;  // two descriptor slots: [0] dot_run, [1] step calls
  Ctl* step_ctl = nullptr;
  double* step_partials = nullptr;
  void* step_scratch = nullptr;  // FP32 transform plane (mixed precision)
  Ctl* host_ctl = nullptr;       // pinned
  // state layout (byte offsets): phi (FP64) | transform scratch (mixed only) |
  // q | q_new | alpha | beta | W (bulk scalar type) | control block | partials
  int n_planes = 0;  // bulk-type planes
  size_t off_phi = 0, off_scr = 0, off_q = 0, off_qn = 0, off_alpha = 0, off_beta = 0, off_w = 0, off_dw = 0;
  size_t ctl_offset = 0, partials_offset = 0, state_bytes = 0;
  int device = 0;
  Prof prof;
  GraphCache graphs;
};

namespace {

// State layout of one instance (byte offsets): phi (FP64) | transform scratch
// (mixed only) | q (D+1) | q_new (D+1) | alpha (D+1, FP64) | beta (K) | W (4D)
// | dw (FP64) | control block | partials; bulk planes in the precision's
// scalar type (the same arithmetic as dot_footprint_bytes).
struct StateLayout {
  size_t off_phi, off_scr, off_q, off_qn, off_alpha, off_beta, off_w, off_dw, ctl_offset;
};
StateLayout state_layout(int D, int64_t nb, int precision) {
  const size_t pb = (size_t)nb * (precision == DOT_MIXED ? sizeof(float) : sizeof(double));
  const int K = 4 * D + 2;
  StateLayout l;
  l.off_phi = 0;
  l.off_scr = align256((size_t)nb * sizeof(double));
  l.off_q = l.off_scr + (precision == DOT_MIXED ? align256(pb) : 0);
  l.off_qn = l.off_q + (size_t)(D + 1) * pb;
  l.off_alpha = align256(l.off_qn + (size_t)(D + 1) * pb);
  l.off_beta = l.off_alpha + (size_t)(D + 1) * nb * sizeof(double);
  l.off_w = l.off_beta + (size_t)K * pb;
  l.off_dw = align256(l.off_w + (size_t)(4 * D) * pb);
  l.ctl_offset = align256(l.off_dw + (size_t)nb * sizeof(double));
  return l;
}

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
          if (r < n_out && c < n_in) out[base + (((size_t)m * nch + ch) * 64 + l) * kU + u] = (T)H(r, c);
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

// Waves per workgroup of a transform pass over an axis of L points. A launch
// with few tiles (fewer than kManyTiles workgroups) gives each work item its
// own wave, so the coefficient streams of all items run concurrently; with
// many tiles each wave takes up to items_per_wave items and more workgroups
// share a CU.
constexpr int64_t kManyTiles = 1024;

int pass_items(int L, int cw) {
  const int M = L / 2, ne = L - M, no = M;
  const int groups = cw >= 32 ? cw / 32 : 1;  // work items per row block (see tile_mfma)
  return groups * ((ne + 15) / 16 + (no + 15) / 16);
}

template <typename T>
int wave_items(int cw) {
  return cw >= 32 ? items_per_wave<T, kCW>() : items_per_wave<T, kCWNarrow>();
}

template <typename T>
int pass_waves(int L, int64_t tiles, int cw) {
  const int items = pass_items(L, cw);
  const int rounds = (items + wave_items<T>(cw) - 1) / wave_items<T>(cw);
  // many tiles: small workgroups, several per CU; few tiles: spread the items
  const int w = (tiles >= kManyTiles || items > kMaxWaves) ? rounds : items;
  return std::max(4, std::min(kMaxWaves, w));
}

// Dynamic LDS of a transform pass over an axis of L points: the tile of
// cw columns (row stride cw + 1) and, behind it, the eigenvalue tables of the
// scale pass (L rows, cw columns).
size_t pass_smem(int L, int scalar_bytes, int cw) { return ((size_t)L * (cw + 1) + L + cw) * scalar_bytes; }

// Whether an axis of L points fits a tile of cw lines: its work items within
// one workgroup's waves and the tile within the LDS.
template <typename T>
bool axis_fits(int L, int cw, int max_smem) {
  return pass_items(L, cw) <= wave_items<T>(cw) * kMaxWaves &&
         (int64_t)pass_smem(L, sizeof(T), cw) <= (int64_t)max_smem;
}

// Tile width of a transform launch over `lines` lines in all: the wide tile
// when every axis of the launch fits it and it still gives many workgroups;
// else the middle width when its tile is small enough for several workgroups
// per CU (kMidLds) and the launch keeps kMidTiles tiles (half the
// coefficient traffic of the narrow tile; measured: 2D 64x128^2 mixed 167 ->
// 153 us per iteration, neutral where the LDS or the tile count rule it out);
// else the narrow one.
constexpr int64_t kMidTiles = 256;
constexpr size_t kMidLds = 40 << 10;
int choose_cw(int64_t lines, bool wide_ok, bool mid_ok) {
  if (wide_ok && (lines + kCW - 1) / kCW >= kManyTiles) return kCW;
  if (mid_ok && (lines + kCWMid - 1) / kCWMid >= kMidTiles) return kCWMid;
  return kCWNarrow;
}

// Lines per workgroup on a last axis that every instance solves by
// elimination: one round of the partitioned solve (256 / lanes per line: 8
// for lines of up to 288 nodes, 4 up to 576), so that each workgroup loads,
// solves and stores once; 64 when some line is longer (the one-lane-per-line
// solve takes tiles of 16, 32 or 64 lines).
int tri_default_cw(dot_plan* const* plans, int count) {
  int L = 0;
  for (int i = 0; i < count; ++i) L = std::max(L, plans[i]->g.N[plans[i]->D]);
  if (L > kTriPartMaxNodes) return kCW;
  return kTriThreads / tri_lanes(L);
}

// Tile widths a last axis solved by elimination in every instance may take.
bool tri_cw_ok(dot_plan* const* plans, int count, int cw) {
  if (cw == kCW || cw == kCWMid || cw == kCWNarrow) return true;
  if (cw != 4 && cw != 8) return false;
  for (int i = 0; i < count; ++i)
    if (plans[i]->g.N[plans[i]->D] > kTriPartMaxNodes) return false;
  return true;
}
int64_t tiles_for(int64_t lines, int cw) { return (lines + cw - 1) / cw; }

// Launch geometry of the passes over axis a of one launch covering the
// instances plans[0..count): tile width and waves from s where it sets them,
// else from the rules above (a last axis that every instance solves by
// elimination takes one round of the partitioned solve: 8 lines of up to 288
// nodes, 4 of up to 576 per 256 lanes; 64 for longer lines), and the LDS bytes.
struct AxisGeom {
  int cw = kCW, waves = 4;
  int64_t tiles = 0;
  size_t smem = 0;
};
template <typename T>
AxisGeom axis_geom(dot_plan* const* plans, int count, int a, const Sched& s) {
  int64_t all_lines = 0;
  bool wide_ok = true, mid_ok = true, all_tri = true;
  for (int i = 0; i < count; ++i) {
    all_lines += plans[i]->lines[a];
    wide_ok = wide_ok && plans[i]->wide_ok[a];
    mid_ok = mid_ok && plans[i]->mid_ok[a];
    all_tri = all_tri && plans[i]->tri;
  }
  AxisGeom ag;
  ag.cw = s.cw[a] ? s.cw[a]
                  : ((a == plans[0]->D && all_tri) ? tri_default_cw(plans, count) : choose_cw(all_lines, wide_ok, mid_ok));
  for (int i = 0; i < count; ++i) ag.tiles += tiles_for(plans[i]->lines[a], ag.cw);
  int waves = 1;
  for (int i = 0; i < count; ++i) {
    if (a == plans[i]->D && plans[i]->tri) continue;  // takes the tridiagonal solve on this axis
    ag.smem = std::max(ag.smem, pass_smem(plans[i]->g.N[a], (int)sizeof(T), ag.cw));
    waves = std::max(waves, pass_waves<T>(plans[i]->g.N[a], ag.tiles, ag.cw));
  }
  ag.waves = s.waves[a] ? s.waves[a] : waves;
  return ag;
}

// Schedules of axis a that every instance of a launch can take: the tile
// widths its LDS and waves hold (the wide one only where the rule may pick
// it; the tridiagonal-only last axis keeps its tile) and, per width, the wave
// counts from the fewest that hold every work item up to kMaxWaves (that
// fewest, 4, 8, 16, one wave per item, the rule's).
template <typename T>
std::vector<std::pair<int, int>> axis_candidates(dot_plan* const* plans, int count, int a, int max_smem) {
  std::vector<std::pair<int, int>> out;
  bool all_tri = true, wide_ok = true, mid_fits = true;
  for (int i = 0; i < count; ++i) {
    all_tri = all_tri && plans[i]->tri;
    if (a == plans[i]->D && plans[i]->tri) continue;  // no transform pass for this one
    wide_ok = wide_ok && plans[i]->wide_ok[a];
    mid_fits = mid_fits && axis_fits<T>(plans[i]->g.N[a], kCWMid, max_smem);
  }
  if (a == plans[0]->D && all_tri) {
    // only the tridiagonal solve runs on this axis: 256 threads whatever the
    // waves; the width sets the lines per workgroup (and its LDS)
    std::vector<int> cws = {tri_default_cw(plans, count), kCWNarrow, kCWMid, kCW};
    std::sort(cws.begin(), cws.end());
    cws.erase(std::unique(cws.begin(), cws.end()), cws.end());
    for (int cw : cws) {
      Sched s;
      s.cw[a] = cw;
      out.push_back({cw, axis_geom<T>(plans, count, a, s).waves});
    }
    return out;
  }
  for (int cw : {kCWNarrow, kCWMid, kCW}) {
    if ((cw == kCW && !wide_ok) || (cw == kCWMid && !mid_fits)) continue;
    int lo = 1, items = 1;
    for (int i = 0; i < count; ++i) {
      if (a == plans[i]->D && plans[i]->tri) continue;
      const int it = pass_items(plans[i]->g.N[a], cw);
      items = std::max(items, it);
      lo = std::max(lo, (it + wave_items<T>(cw) - 1) / wave_items<T>(cw));
    }
    if (lo > kMaxWaves) continue;
    Sched s;
    s.cw[a] = cw;
    const int rule = axis_geom<T>(plans, count, a, s).waves;
    std::vector<int> ws = {lo, 4, 8, 16, std::min(items, kMaxWaves), rule};
    std::sort(ws.begin(), ws.end());
    ws.erase(std::unique(ws.begin(), ws.end()), ws.end());
    for (int w : ws)
      if (w >= lo && w <= kMaxWaves) out.push_back({cw, w});
  }
  return out;
}

// Last axes of at least this many nodes are solved by tridiagonal elimination
// (its cost per point does not grow with the axis length; measured per
// iteration: 2D 32x1024^2 mixed 6.15 -> 5.13 ms, 2D 64x256^2 FP64 844 -> 823 us,
// mixed 534 -> 531 us). With the partitioned elimination also taking the
// shorter last axes (threshold 33 instead of 257), per iteration: 2D 32x64^2
// FP64 55.6 us either way, 2D 64x128^2 mixed 145.6 -> 133.7 us, but 3D 32x64^3
// mixed 1227 -> 1291 us and the 64-instance 2D batch 1181 -> 1264 us; the
// transform keeps the short axes.
constexpr int kTriMinNodes = 257;

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
T* at(void* base, size_t byte_off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + byte_off);
}

template <typename T>
const AxisTab<T>& tab_of(const dot_plan* P, int a);
template <>
const AxisTab<double>& tab_of<double>(const dot_plan* P, int a) { return P->tab64[a]; }
template <>
const AxisTab<float>& tab_of<float>(const dot_plan* P, int a) { return P->tab32[a]; }

// Time slices per workgroup of the node sweeps: about 8192 workgroups per
// instance when the grid allows (32 per CU; measured against 1024..65536:
// 2D 64x256^2 mixed 546 -> 533 us and 3D 32x64^3 mixed 1386 -> 1319 us per
// iteration going from 4096 to 8192), at most 4 slices each (2D 32x1024^2
// mixed: 5.15 ms per iteration at 16 slices, 4.83 at 8, 4.70 at 4, 4.72 at 2).
int default_tc(int64_t nx, int N0) {
  const int64_t nxb = (nx + kBlock - 1) / kBlock;
  const int64_t tc = (int64_t)N0 * nxb / 8192;
  return (int)std::max<int64_t>(1, std::min<int64_t>(4, tc));
}

void set_sweep(Geo& g, int tc) {
  g.tc = tc;
  g.nxb = (uint32_t)((g.nx + kBlock - 1) / kBlock);
  g.nsweep = g.nxb * (uint32_t)((g.N[0] + tc - 1) / tc);
}

// Workgroups of a flat sweep (one lane per plane entry).
unsigned flat_grid(const dot_plan* P) { return (unsigned)((P->g.nb + kBlock - 1) / kBlock); }

FinArgs fin_args(const dot_plan* P) {
  FinArgs fa;
  fa.vol = P->vol;
  fa.c_norm2 = P->c_norm2;
  fa.d_norm2 = P->d_norm2;
  fa.nblocks = P->nblocks;
  fa.staged = P->nblocks >= kFinStageMinRows ? 1 : 0;
  return fa;
}

// Descriptor of one instance with caller planes: phi / b and alpha (FP64), q,
// q_new, beta, W (bulk type), transform work plane, control block, partials.
template <typename T>
Inst<T> inst_of(const dot_plan* P, double* phi, T* scr, T* q, T* qn, double* alpha, T* beta, T* W, double* dw,
                Ctl* ctl, double* partials) {
  Inst<T> s{};
  s.g = P->g;
  s.phi = phi;
  s.work = std::is_same<T, double>::value ? reinterpret_cast<T*>(phi) : scr;
  s.q[0] = q;
  s.q[1] = qn;
  s.alpha = alpha;
  s.beta = beta;
  s.W = W;
  s.dw = dw;
  s.ctl = ctl;
  s.partials = partials;
  s.sw = P->sw_sp;
  s.om = P->om_sp;
  s.c_lo = P->c_lo;
  s.c_hi = P->c_hi;
  s.lam_other = (const T*)P->lam_other;
  s.lam_last = (const T*)P->lam_last;
  for (int a = 0; a < kMaxAxes; ++a) s.tab[a] = tab_of<T>(P, a);
  s.fa = fin_args(P);
  s.tri = P->tri;
  return s;
}

// Descriptor of an instance whose state buffer (plan layout) is at `state`
// and whose control block is at `ctl`.
template <typename T>
Inst<T> state_inst(const dot_plan* P, void* state, Ctl* ctl) {
  return inst_of<T>(P, at<double>(state, P->off_phi), at<T>(state, P->off_scr), at<T>(state, P->off_q),
                    at<T>(state, P->off_qn), at<double>(state, P->off_alpha), at<T>(state, P->off_beta),
                    at<T>(state, P->off_w), at<double>(state, P->off_dw), ctl, at<double>(state, P->partials_offset));
}

Ctl initial_ctl(const dot_plan* P) {
  Ctl h{};
  h.sigma = P->sigma0;
  h.tau = P->tau;
  h.tol = P->tol;
  h.next_update = P->gap0;
  h.gap = P->gap0;
  h.growth = P->growth;
  h.adapt = P->adapt;
  h.cadence = P->cadence;
  h.iter_limit = INT32_MAX;
  return h;
}

// Launch geometry of one executor: the descriptor array, block maps and,
// per phase, grid size, LDS bytes and waves.
struct Exec {
  int D = 0, precision = 0, ninst = 0, cadence = 5;
  int nact = 0;  // instances with workgroups in the launch grids (a compacted batch leaves out stopped ones)
  int nstaged = 0;  // of those, instances whose residual partials take the two-stage reduction
  void* d_inst = nullptr;
  const uint16_t* map_nodes = nullptr;
  const uint16_t* map_axis[kMaxAxes] = {nullptr, nullptr, nullptr, nullptr};
  unsigned grid_nodes = 0;
  unsigned grid_axis[kMaxAxes] = {0, 0, 0, 0};
  size_t smem_axis[kMaxAxes] = {0, 0, 0, 0};
  int waves_axis[kMaxAxes] = {0, 0, 0, 0};
  int cw_axis[kMaxAxes] = {kCW, kCW, kCW, kCW};  // transform tile width per axis
  int ntri = 0;       // instances whose last axis takes the tridiagonal solve
  int ntri_long = 0;  // of those, lines longer than the partitioned solve takes
  int64_t nodes = 0;  // grid nodes over all instances
  Prof* prof = nullptr;
  int device = 0;
  struct GraphCache* graphs = nullptr;  // captured 10-iteration blocks (nullptr: plain launches)
};

// Raise a kernel's dynamic LDS limit to the device maximum.
int set_max_lds(const void* fn, int device) {
  int max_smem = 0;
  HIP_OK(hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
  HIP_OK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_smem));
  return DOT_OK;
}

template <typename T, int D, int KIND, int SRC, int DST, int CW>
int launch_pass_cw(const Exec& E, int a, hipStream_t st) {
  auto fn = kb_axis_pass<T, D, KIND, SRC, DST, CW>;
  // the LDS opt-in is per kernel and process: set once (thread-safe static)
  static const int smem_rc = set_max_lds((const void*)fn, E.device);
  if (smem_rc) return smem_rc;
  const int cls = KIND == kFwdScaleInv ? DOT_K_DCT_LAST
                  : KIND == kInv         ? DOT_K_DCT_INV
                                         : (a == 0 ? DOT_K_DCT_FIRST : DOT_K_DCT_MID);
  ProfScope ps(E.prof, cls, st);
  hipLaunchKernelGGL(fn, dim3(E.grid_axis[a]), dim3(E.waves_axis[a] * 64), E.smem_axis[a], st,
                     (const Inst<T>*)E.d_inst, E.map_axis[a], a);
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

template <typename T, int D, int KIND, int SRC, int DST>
int launch_pass(const Exec& E, int a, int par, double sigma, hipStream_t st) {
  (void)par;
  (void)sigma;
  switch (E.cw_axis[a]) {
    case kCW: return launch_pass_cw<T, D, KIND, SRC, DST, kCW>(E, a, st);
    case kCWMid: return launch_pass_cw<T, D, KIND, SRC, DST, kCWMid>(E, a, st);
    default: return launch_pass_cw<T, D, KIND, SRC, DST, kCWNarrow>(E, a, st);
  }
}

// Tridiagonal last-axis solve over the last-axis tile grid (tiles of cw
// lines).
template <typename T, int D, int CW>
int launch_tri_cw(const Exec& E, hipStream_t st) {
  ProfScope ps(E.prof, DOT_K_DCT_LAST, st);
  hipLaunchKernelGGL((kb_tri_pass<T, D, CW>), dim3(E.grid_axis[D]), dim3(kTriThreads), 0, st, (const Inst<T>*)E.d_inst,
                     E.map_axis[D]);
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

// Last-axis elimination: the partitioned solve for lines of up to
// kTriPartMaxNodes nodes, the one-lane-per-line solve for longer ones.
template <typename T, int D>
int launch_tri(const Exec& E, hipStream_t st) {
  if (E.ntri > E.ntri_long) {
    ProfScope ps(E.prof, DOT_K_DCT_LAST, st);
    hipLaunchKernelGGL((kb_tri_part<T, D>), dim3(E.grid_axis[D]), dim3(kTriThreads), 0, st, (const Inst<T>*)E.d_inst,
                       E.map_axis[D], E.cw_axis[D]);
    HIP_OK(hipGetLastError());
  }
  if (E.ntri_long == 0) return DOT_OK;
  switch (E.cw_axis[D]) {
    case kCW: return launch_tri_cw<T, D, kCW>(E, st);
    case kCWMid: return launch_tri_cw<T, D, kCWMid>(E, st);
    default: return launch_tri_cw<T, D, kCWNarrow>(E, st);
  }
}

// The 2D+1 transform passes of one Poisson solve (a3 + a4): first pass on the
// time axis loads according to SRC, forward passes on the middle axes, the
// fused forward/scale/inverse pass on the last axis (or, for instances with
// a long last axis, the tridiagonal solve along it), inverse passes back to
// the time axis, which stores according to DST.
template <typename T, int D, int SRC, int DST>
int run_passes(const Exec& E, int par, double sigma, hipStream_t st) {
  int rc;
  if ((rc = launch_pass<T, D, kFwd, SRC, kDstPlane>(E, 0, par, sigma, st))) return rc;
  for (int a = 1; a < D; ++a)
    if ((rc = launch_pass<T, D, kFwd, kSrcPlane, kDstPlane>(E, a, par, sigma, st))) return rc;
  if (E.ntri < E.nact && (rc = launch_pass<T, D, kFwdScaleInv, kSrcPlane, kDstPlane>(E, D, par, sigma, st)))
    return rc;
  if (E.ntri > 0 && (rc = launch_tri<T, D>(E, st))) return rc;
  for (int a = D - 1; a >= 1; --a)
    if ((rc = launch_pass<T, D, kInv, kSrcPlane, kDstPlane>(E, a, par, sigma, st))) return rc;
  return launch_pass<T, D, kInv, kSrcPlane, DST>(E, 0, par, sigma, st);
}

// Poisson solve inside an iteration. FP64: the transforms run in place on
// phi. Mixed: the FP32 transforms solve A^*A dphi = b - A^*A phi on the
// scratch plane and the last pass adds dphi to the FP64 phi.
template <typename T, int D, bool DEFECT>
int launch_rhs(const Exec& E, int par, double sigma, hipStream_t st) {
  {
    ProfScope ps(E.prof, DOT_K_RHS, st);
    hipLaunchKernelGGL((kb_rhs<T, D, DEFECT>), dim3(E.grid_nodes), dim3(kBlock), 0, st, (const Inst<T>*)E.d_inst,
                       E.map_nodes, par, sigma);
  }
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

template <typename T, int D>
int poisson_iter(const Exec& E, int par, hipStream_t st, bool rhs_ready = false) {
  constexpr bool kMixed = !std::is_same<T, double>::value;
  int rc;
  if (!rhs_ready && (rc = launch_rhs<T, D, kMixed>(E, par, 0.0, st))) return rc;
  if constexpr (kMixed)
    return run_passes<T, D, kSrcPlane, kDstPhiAdd>(E, par, 0.0, st);
  else
    return run_passes<double, D, kSrcPlane, kDstPlane>(E, par, 0.0, st);
}

template <typename T, int D>
int launch_cone(const Exec& E, int par, hipStream_t st) {
  ProfScope ps(E.prof, DOT_K_CONE, st);
  hipLaunchKernelGGL((kb_cone<T, D>), dim3(E.grid_nodes), dim3(kBlock), 0, st, (const Inst<T>*)E.d_inst,
                     E.map_nodes, par);
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

// z-step and right-hand side of iteration par in one launch (runs only
// where the z-step may precede the phi-step: no one-lane elimination, whose
// checkpoints use W plane 0).
template <typename T, int D>
int launch_cone_rhs(const Exec& E, int par, hipStream_t st) {
  constexpr bool kMixed = !std::is_same<T, double>::value;
  ProfScope ps(E.prof, DOT_K_CONE, st);
  hipLaunchKernelGGL((kb_cone_rhs<T, D, kMixed>), dim3(E.grid_nodes), dim3(kBlock), 0, st, (const Inst<T>*)E.d_inst,
                     E.map_nodes, par);
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

template <typename T, int D>
int launch_q(const Exec& E, int par, hipStream_t st) {
  ProfScope ps(E.prof, DOT_K_QD, st);
  hipLaunchKernelGGL((kb_q<T, D>), dim3(E.grid_nodes), dim3(kBlock), 0, st, (const Inst<T>*)E.d_inst, E.map_nodes,
                     par);
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

// beta update of the iteration with parity par (q[par] the old q, q[par ^ 1]
// the new one); with cone_next also the z-step of the next iteration, with
// rhs_next also its right-hand side (both only after an iteration without a
// check).
template <typename T, int D>
int launch_beta(const Exec& E, int par, int check, hipStream_t st, bool rhs_next, bool cone_next = false) {
  const Inst<T>* I = (const Inst<T>*)E.d_inst;
  constexpr bool kMixed = !std::is_same<T, double>::value;
  ProfScope ps(E.prof, DOT_K_BETA, st);
  if (cone_next && rhs_next)
    hipLaunchKernelGGL((kb_beta_cone_rhs<T, D, kMixed>), dim3(E.grid_nodes), dim3(kBlock), 0, st, I, E.map_nodes,
                       par);
  else if (cone_next)
    hipLaunchKernelGGL((kb_beta_cone<T, D>), dim3(E.grid_nodes), dim3(kBlock), 0, st, I, E.map_nodes, par);
  else if (rhs_next)
    hipLaunchKernelGGL((kb_beta_rhs<T, D, kMixed>), dim3(E.grid_nodes), dim3(kBlock), 0, st, I, E.map_nodes, par);
  else
    hipLaunchKernelGGL((kb_beta<T, D>), dim3(E.grid_nodes), dim3(kBlock), 0, st, I, E.map_nodes, par, check);
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

// z-step, q-step and multiplier steps of one iteration, one after the other.
template <typename T, int D>
int update_iter(const Exec& E, int par, int check, hipStream_t st, bool rhs_next = false) {
  int rc;
  if ((rc = launch_cone<T, D>(E, par, st)) || (rc = launch_q<T, D>(E, par, st))) return rc;
  return launch_beta<T, D>(E, par, check, st, rhs_next);
}

// Residual partials at the iterate in q[qpar], the first stage of their
// reduction (kFinChunks blocks per instance; large instances only), then one
// finalize block per instance.
template <typename T, int D>
int check_iter(const Exec& E, int qpar, int update_ctl, hipStream_t st) {
  const Inst<T>* I = (const Inst<T>*)E.d_inst;
  {
    ProfScope ps(E.prof, DOT_K_RESID, st);
    hipLaunchKernelGGL((kb_resid<T, D>), dim3(E.grid_nodes), dim3(kBlock), 0, st, I, E.map_nodes, qpar);
  }
  HIP_OK(hipGetLastError());
  {
    ProfScope ps(E.prof, DOT_K_FINAL, st);
    if (E.nstaged > 0) {
      hipLaunchKernelGGL((kb_fin_stage<T>), dim3(E.ninst * kFinChunks), dim3(256), 0, st, I);
      HIP_OK(hipGetLastError());
    }
    hipLaunchKernelGGL((kb_finalize<T>), dim3(E.ninst), dim3(256), 0, st, I, update_ctl);
  }
  HIP_OK(hipGetLastError());
  return DOT_OK;
}

// What one iteration hands to the next inside a launch sequence: its
// right-hand side and its z-step already computed by the previous beta
// launch (sequential order), or the previous beta update still to run, fused
// with this iteration's z-step (overlapped order).
struct Carry {
  bool rhs_ready = false;
  bool cone_ready = false;
  bool beta_pending = false;
};

// Whether the executor runs the z-step beside the phi-step: needs the branch
// streams, no kernel class being timed, no instance whose last axis takes the
// one-lane elimination (it keeps its checkpoints in W plane 0, which the
// z-step writes), and at least kOverlapMinNodes grid nodes in all. The fork
// and the join cost about 10 us per iteration; below that size the kernels
// they would overlap are shorter. Measured per iteration, sequential ->
// overlapped (with the fused beta and z-step in both orders): 2D 64x128^2
// mixed (1.08M nodes) 132 -> 141 us; 2D 64x192^2 mixed (2.4M) 299 -> 291 us;
// 2D 64x256^2 mixed 465 -> 447 us, FP64 699 -> 685 us; 3D 32x64^3 mixed
// 1185 -> 1162 us; the 64-instance 2D batch 1154 -> 1086 us.
constexpr int64_t kOverlapMinNodes = int64_t(1) << 21;
bool overlapped(const Exec& E) {
  return E.graphs && !(E.prof && E.prof->cls >= 0) && E.ntri_long == 0 && E.nodes >= kOverlapMinNodes;
}

int branch_streams(GraphCache* g) {
  if (!g->side) HIP_OK(hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking));
  if (!g->cap_side) HIP_OK(hipStreamCreateWithFlags(&g->cap_side, hipStreamNonBlocking));
  if (!g->fork) HIP_OK(hipEventCreateWithFlags(&g->fork, hipEventDisableTiming));
  if (!g->join) HIP_OK(hipEventCreateWithFlags(&g->join, hipEventDisableTiming));
  return DOT_OK;
}

// One iteration of every instance of E: Poisson solve, cone and updates, and
// on check iterations the residual reductions and the control update.
//
// Sequential order (one stream): [rhs] passes [cone] q beta, where an
// iteration without a check followed by another in the same sequence (`more`)
// runs the next iteration's z-step and right-hand side in its beta launch
// (the z-step reads only the new q and beta; the right-hand side the new q,
// alpha and phi). An executor with an instance whose last axis takes the
// one-lane elimination keeps the z-step after the passes (those keep their
// checkpoints in W plane 0) and fuses only the right-hand side.
// Overlapped order: the z-step reads only q and beta, so it runs on a second
// stream (`side`, a parallel branch inside a captured graph) while the main
// stream computes the right-hand side and the transforms; the beta update of
// an iteration without a check is deferred to the side branch of the next
// iteration, fused with its z-step, beside the next right-hand side (the two
// read q and alpha and write disjoint planes):
//   main: rhs -> passes ---------------\
//   side: [beta of it-1 +] cone --------+-> q [-> beta -> resid -> finalize]
// An iteration with a check, or the last one of a sequence (`more` false),
// runs its beta update alone, so that every sequence ends with a complete
// iterate. All orders compute the same values.
template <typename T, int D>
int one_iter(const Exec& E, int it, hipStream_t st, hipStream_t side, bool more, Carry* cy) {
  const int par = it & 1;
  const int check = ((it + 1) % E.cadence) == 0;
  int rc;
  if (side) {
    GraphCache* g = E.graphs;
    HIP_OK(hipEventRecord(g->fork, st));
    HIP_OK(hipStreamWaitEvent(side, g->fork, 0));
    if (cy->beta_pending)
      rc = launch_beta<T, D>(E, par ^ 1, 0, side, false, true);
    else
      rc = launch_cone<T, D>(E, par, side);
    if (rc) return rc;
    HIP_OK(hipEventRecord(g->join, side));
    if ((rc = poisson_iter<T, D>(E, par, st, false))) return rc;
    HIP_OK(hipStreamWaitEvent(st, g->join, 0));
    if ((rc = launch_q<T, D>(E, par, st))) return rc;
    cy->beta_pending = !check && more;
    if (!cy->beta_pending && (rc = launch_beta<T, D>(E, par, check, st, false))) return rc;
    if (check && (rc = check_iter<T, D>(E, par ^ 1, 1, st))) return rc;
    cy->rhs_ready = false;
    cy->cone_ready = false;
    return DOT_OK;
  }
  // kernel classes timed one by one run unfused
  const bool timing = E.prof && E.prof->cls >= 0;
  bool rhs_ready = cy->rhs_ready, cone_ready = cy->cone_ready;
  if (!rhs_ready && !cone_ready && E.ntri_long == 0 && !timing) {
    if ((rc = launch_cone_rhs<T, D>(E, par, st))) return rc;
    rhs_ready = cone_ready = true;
  }
  if ((rc = poisson_iter<T, D>(E, par, st, rhs_ready))) return rc;
  if (!cone_ready && (rc = launch_cone<T, D>(E, par, st))) return rc;
  if ((rc = launch_q<T, D>(E, par, st))) return rc;
  const bool fuse = !check && more && !timing;
  const bool fuse_cone = fuse && E.ntri_long == 0;
  if ((rc = launch_beta<T, D>(E, par, check, st, fuse, fuse_cone))) return rc;
  if (check && (rc = check_iter<T, D>(E, par ^ 1, 1, st))) return rc;
  cy->rhs_ready = fuse;
  cy->cone_ready = fuse_cone;
  cy->beta_pending = false;
  return DOT_OK;
}

// Capture n iterations (a multiple of kGraphIters) starting at an iteration
// count it (it % 10 == 0 keeps the check positions aligned) into a graph, on the cache's own
// stream (the caller's stream may be the legacy default stream, which cannot
// be captured); the graph is then launched on the caller's stream.
template <typename T, int D>
int capture_block(const Exec& E, int it, hipGraphExec_t* out, int n = kGraphIters) {
  DevLock lk(g_dev_mu);
  for (int f = g_fail_captures.load(); f > 0;)
    if (g_fail_captures.compare_exchange_weak(f, f - 1)) return fail(DOT_EDEVICE, "capture failed on purpose (test)");
  Exec Ec = E;
  Ec.prof = nullptr;  // no events inside a captured graph
  if (!E.graphs->cap) HIP_OK(hipStreamCreateWithFlags(&E.graphs->cap, hipStreamNonBlocking));
  hipStream_t st = E.graphs->cap;
  hipStream_t side = nullptr;
  if (overlapped(Ec)) {
    int rc0 = branch_streams(E.graphs);
    if (rc0) return rc0;
    side = E.graphs->cap_side;
  }
  hipGraph_t graph = nullptr;
  HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int rc = DOT_OK;
  Carry cy;
  for (int k = 0; k < n && !rc; ++k) rc = one_iter<T, D>(Ec, it + k, st, side, k + 1 < n, &cy);
  if (rc && side) {
    // a failure between fork and join: join the second branch back before the
    // capture ends (errors ignored; the capture is abandoned anyway)
    (void)hipEventRecord(E.graphs->join, side);
    (void)hipStreamWaitEvent(st, E.graphs->join, 0);
  }
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(DOT_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    *out = nullptr;
    return fail(DOT_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return DOT_OK;
}

// Run up to max_iters iterations of every instance of E in lockstep starting
// at iteration it0 (same for all instances); ctl_host (pinned, ninst entries
// at stride ctl_stride) is refreshed from ctl_dev every `poll` iterations and
// the loop ends once every instance has stopped. Whole blocks of 10
// iterations that start at a multiple of 10 replay a captured graph when the
// executor has a graph cache and no kernel class is being timed. on_poll runs
// after each poll that does not end the loop, with the fresh control blocks
// in ctl_host; it may lay the executor out anew (and drop its graph).
template <typename T, int D>
int run_iters(const Exec& E, int it0, int max_iters, const void* ctl_dev, size_t ctl_stride, void* ctl_host,
              hipStream_t st, int* done_iters, int nctl = -1, double time_limit = 0.0, bool* timed_out = nullptr,
              const std::function<int()>* on_poll = nullptr) {
  const int poll = 40;
  const auto t_start = std::chrono::steady_clock::now();
  if (nctl < 0) nctl = E.ninst;
  auto all_stopped = [&]() {
    for (int i = 0; i < nctl; ++i)
      if (!reinterpret_cast<const Ctl*>(static_cast<const char*>(ctl_host) + i * ctl_stride)->stop) return false;
    return true;
  };
  bool use_graphs = E.graphs && E.graphs->enabled && !(E.prof && E.prof->cls >= 0) && E.cadence == 5;
  int capture_failures = 0;
  hipStream_t side = nullptr;
  if (overlapped(E)) {
    int rc0 = branch_streams(E.graphs);
    if (rc0) return rc0;
    side = E.graphs->side;
  }
  int j = 0;
  int since_poll = 0;
  Carry cy;  // what the previous iteration left to this one
  while (j < max_iters) {
    const int it = it0 + j;
    int rc;
    const bool blk_ok = use_graphs && E.graphs->warm && it % kGraphIters == 0 && !cy.rhs_ready &&
                        !cy.cone_ready && !cy.beta_pending;
    // a block replays its captured graph; a capture that fails (nothing of
    // it ran) leaves the block to plain launches, and after two failures this
    // call launches plainly
    auto captured = [&](hipGraphExec_t& ex, int n) -> bool {
      if (ex) return true;
      if (capture_block<T, D>(E, it, &ex, n) == DOT_OK) return true;
      (void)hipGetLastError();
      if (++capture_failures >= 2) use_graphs = false;
      return false;
    };
    bool ran = false;
    if (blk_ok && since_poll == 0 && max_iters - j >= poll) {
      if (captured(E.graphs->exec_poll, poll)) {
        HIP_OK(hipGraphLaunch(E.graphs->exec_poll, st));
        j += poll;
        since_poll += poll;
        ran = true;
      }
    } else if (blk_ok && max_iters - j >= kGraphIters) {
      if (captured(E.graphs->exec, kGraphIters)) {
        HIP_OK(hipGraphLaunch(E.graphs->exec, st));
        // a block starts with its own right-hand side and ends with a check
        j += kGraphIters;
        since_poll += kGraphIters;
        ran = true;
      }
    }
    if (!ran) {
      // an iteration before a poll completes its iterate (nothing deferred)
      const bool more = j + 1 < max_iters && since_poll + 1 < poll;
      if ((rc = one_iter<T, D>(E, it, st, side, more, &cy))) return rc;
      if (E.graphs) E.graphs->warm = true;
      ++j;
      ++since_poll;
    }
    if (since_poll >= poll || j == max_iters) {
      since_poll = 0;
      HIP_OK(hipMemcpyAsync(ctl_host, ctl_dev, ctl_stride * nctl, hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      if (E.prof) E.prof->collect();
      if (all_stopped()) break;
      // wall-clock budget: return with the state as it is (resumable); a
      // call that has also done all its iterations is not cut short by it
      if (time_limit > 0.0 && j < max_iters &&
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count() >= time_limit) {
        if (timed_out) *timed_out = true;
        break;
      }
      // the executor's layout may change here (nothing is deferred at a poll)
      if (on_poll && j < max_iters) {
        if ((rc = (*on_poll)())) return rc;
        side = nullptr;
        if (overlapped(E)) {
          if ((rc = branch_streams(E.graphs))) return rc;
          side = E.graphs->side;
        }
      }
    }
  }
  HIP_OK(hipMemcpyAsync(ctl_host, ctl_dev, ctl_stride * nctl, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (E.prof) E.prof->collect();
  if (done_iters) *done_iters = j;
  return DOT_OK;
}

void fill_result(const Ctl& c, dot_result* res) {
  if (!res) return;
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

// Dispatch on (scalar type, D).
template <template <typename, int> class F, typename... A>
int dispatch(int precision, int D, A&&... args) {
  if (precision == DOT_FP64) {
    switch (D) {
      case 1: return F<double, 1>::run(std::forward<A>(args)...);
      case 2: return F<double, 2>::run(std::forward<A>(args)...);
      case 3: return F<double, 3>::run(std::forward<A>(args)...);
    }
  } else {
    switch (D) {
      case 1: return F<float, 1>::run(std::forward<A>(args)...);
      case 2: return F<float, 2>::run(std::forward<A>(args)...);
      case 3: return F<float, 3>::run(std::forward<A>(args)...);
    }
  }
  return fail(DOT_EINVAL, "unsupported D");
}

size_t inst_slot_bytes() { return align256(std::max(sizeof(Inst<double>), sizeof(Inst<float>))); }

// Single-instance executor of a plan; descriptor slot 0 (run) or 1 (steps).
Exec plan_exec(dot_plan* P, int slot) {
  Exec E;
  E.D = P->D;
  E.precision = P->precision;
  E.ninst = 1;
  E.nact = 1;
  E.cadence = P->cadence;
  E.d_inst = static_cast<char*>(P->d_inst) + slot * inst_slot_bytes();
  E.map_nodes = nullptr;  // one instance: blocks need no map
  E.grid_nodes = (unsigned)P->nblocks;
  E.ntri = P->tri ? 1 : 0;
  E.ntri_long = P->tri && P->g.N[P->D] > kTriPartMaxNodes ? 1 : 0;
  E.nstaged = P->nblocks >= kFinStageMinRows ? 1 : 0;
  E.nodes = P->g.nb;
  for (int a = 0; a <= P->D; ++a) {
    E.map_axis[a] = nullptr;
    const AxisGeom ag = P->precision == DOT_FP64 ? axis_geom<double>(&P, 1, a, P->sched)
                                                 : axis_geom<float>(&P, 1, a, P->sched);
    E.cw_axis[a] = ag.cw;
    E.grid_axis[a] = (unsigned)ag.tiles;
    E.smem_axis[a] = ag.smem;
    E.waves_axis[a] = ag.waves;
  }
  E.prof = &P->prof;
  E.device = P->device;
  E.graphs = slot == 0 ? &P->graphs : nullptr;
  return E;
}

template <typename T>
int upload_inst(const Exec& E, const Inst<T>& s, hipStream_t st) {
  HIP_OK(hipMemcpyAsync(E.d_inst, &s, sizeof(s), hipMemcpyHostToDevice, st));
  return DOT_OK;
}

template <typename T, int D>
struct RunF {
  static int run(dot_plan* P, void* state, int max_iters, hipStream_t st, dot_result* res) {
    Ctl* ctl = at<Ctl>(state, P->ctl_offset);
    HIP_OK(hipMemcpyAsync(P->host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const int it0 = P->host_ctl->iter;
    Exec E = plan_exec(P, 0);
    int rc = upload_inst(E, state_inst<T>(P, state, ctl), st);
    if (rc) return rc;
    if (!P->host_ctl->stop) {
      bool timed_out = false;
      rc = run_iters<T, D>(E, it0, max_iters, ctl, sizeof(Ctl), P->host_ctl, st, nullptr, -1, P->time_limit,
                           &timed_out);
      if (rc) return rc;
      fill_result(*P->host_ctl, res);
      if (timed_out && !P->host_ctl->stop && res) res->term = DOT_TIMEOUT;
      return DOT_OK;
    }
    fill_result(*P->host_ctl, res);
    return DOT_OK;
  }
};

// Step-level calls: a descriptor with the caller's planes in slot 1.
template <typename T>
Inst<T> step_inst(dot_plan* P, const void* phi, const void* q, const void* alpha, const void* beta, void* q_out,
                  void* W, Ctl* ctl) {
  // a caller's z-step workspace: 4D planes of the bulk type, then one FP64 plane
  double* dw = W ? reinterpret_cast<double*>(static_cast<char*>(W) + (size_t)(4 * P->D) * P->g.nb * sizeof(T))
                 : nullptr;
  return inst_of<T>(P, (double*)phi, (T*)P->step_scratch, (T*)q, (T*)q_out, (double*)alpha, (T*)beta, (T*)W, dw, ctl,
                    P->step_partials);
}

template <typename T, int D>
struct DivF {
  static int run(dot_plan* P, const void* q, const void* al, double sigma, void* b, hipStream_t st) {
    Exec E = plan_exec(P, 1);
    int rc = upload_inst(E, step_inst<T>(P, nullptr, q, al, nullptr, nullptr, nullptr, nullptr), st);
    if (rc) return rc;
    hipLaunchKernelGGL((kb_divergence<T, D>), dim3(flat_grid(P)), dim3(kBlock), 0, st, (const Inst<T>*)E.d_inst,
                       1.0 / sigma, (double*)b);
    HIP_OK(hipGetLastError());
    return DOT_OK;
  }
};

// Poisson solve of the step-level calls: from (q, alpha, sigma) if q is given,
// else from the right-hand side already in phi; result in phi.
template <typename T, int D>
struct PoissonF {
  static int run(dot_plan* P, void* phi, const void* q, const void* al, double sigma, hipStream_t st) {
    Exec E = plan_exec(P, 1);
    E.prof = nullptr;
    // c' checkpoints of the one-lane-per-line elimination (lines longer than the partitioned solve takes)
    if (P->tri && P->g.N[D] > kTriPartMaxNodes && !P->step_cbuf)
      HIP_OK(hipMalloc(&P->step_cbuf, (size_t)P->g.nb * sizeof(T)));
    int rc = upload_inst(E, step_inst<T>(P, phi, q, al, nullptr, nullptr, P->step_cbuf, nullptr), st);
    if (rc) return rc;
    if (q && (rc = launch_rhs<T, D, false>(E, 0, sigma, st))) return rc;
    if constexpr (std::is_same<T, double>::value) {
      return run_passes<double, D, kSrcPlane, kDstPlane>(E, 0, sigma, st);
    } else {
      if (q) return run_passes<T, D, kSrcPlane, kDstPhiSet>(E, 0, sigma, st);
      return run_passes<T, D, kSrcPlaneF64, kDstPhiSet>(E, 0, sigma, st);
    }
  }
};

template <typename T, int D>
struct ConeF {
  static int run(dot_plan* P, const void* q, const void* beta, double sigma, void* z, hipStream_t st) {
    Exec E = plan_exec(P, 1);
    int rc = upload_inst(E, step_inst<T>(P, nullptr, q, nullptr, beta, nullptr, nullptr, nullptr), st);
    if (rc) return rc;
    hipLaunchKernelGGL((kb_cone_out<T, D>), dim3(flat_grid(P)), dim3(kBlock), 0, st, (const Inst<T>*)E.d_inst,
                       1.0 / sigma, (T*)z);
    HIP_OK(hipGetLastError());
    return DOT_OK;
  }
};

template <typename T, int D>
struct UpdateF {
  static int run(dot_plan* P, const void* phi, const void* q, void* alpha, void* beta, double sigma, double tau,
                 void* qn, void* W, hipStream_t st) {
    Exec E = plan_exec(P, 1);
    E.prof = nullptr;
    Ctl h{};
    h.sigma = sigma;
    h.tau = tau;
    HIP_OK(hipMemcpyAsync(P->step_ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, st));
    int rc = upload_inst(E, step_inst<T>(P, phi, q, alpha, beta, qn, W, P->step_ctl), st);
    if (rc) return rc;
    rc = update_iter<T, D>(E, 0, 0, st);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(st));
    return DOT_OK;
  }
};

template <typename T, int D>
struct ResidF {
  static int run(dot_plan* P, const void* phi, const void* z, const void* q, const void* alpha, const void* beta,
                 hipStream_t st) {
    Exec E = plan_exec(P, 1);
    E.prof = nullptr;
    Ctl h{};  // stop = 0: the finalize block fills the residuals only
    HIP_OK(hipMemcpyAsync(P->step_ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, st));
    int rc = upload_inst(E, step_inst<T>(P, phi, q, alpha, beta, nullptr, nullptr, P->step_ctl), st);
    if (rc) return rc;
    hipLaunchKernelGGL((kb_zres<T, D>), dim3(E.grid_nodes), dim3(kBlock), 0, st, (const Inst<T>*)E.d_inst,
                       (const T*)z);
    HIP_OK(hipGetLastError());
    return check_iter<T, D>(E, 0, 0, st);
  }
};

// ---- residuals without allocation -------------------------------------------
// dot_step_residuals_noalloc keeps the control block that the finalize step
// writes and the per-workgroup partial sums of the residual sweep in this
// file-scope array instead of the plan's buffers. Each GPU the library runs on
// holds its own copy until the process ends. In host code the array's name is
// a host-side stand-in, not a device address: host code uses only the address
// that hipGetSymbolAddress returns for the current device, taken once per
// device and kept in noalloc_ptr.
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[DOT_NOALLOC_SCRATCH_BYTES];

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// Device address of this device's copy of `scratch` (device current).
int noalloc_ptr(int device, unsigned char** out) {
  if (device < 0 || device >= kNoAllocMaxDevices) return fail(DOT_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(DOT_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_noalloc_ptr[device] = p;
  }
  *out = static_cast<unsigned char*>(g_noalloc_ptr[device]);
  return DOT_OK;
}

// Bytes of the scratch array one residual evaluation of P takes: the control
// block, then kNumSums partial rows of one entry per workgroup and the
// kFinChunks stage rows of the reduction.
size_t noalloc_bytes(const dot_plan* P) {
  return align256(sizeof(Ctl)) + (size_t)kNumSums * (size_t)(P->nblocks + kFinChunks) * sizeof(double);
}

template <typename T, int D>
struct ResidNoAllocF {
  static int run(dot_plan* P, const void* phi, const void* z, const void* q, const void* alpha, const void* beta,
                 unsigned char* scr, hipStream_t st) {
    Ctl* ctl = reinterpret_cast<Ctl*>(scr);
    double* partials = reinterpret_cast<double*>(scr + align256(sizeof(Ctl)));
    Exec E = plan_exec(P, 1);
    E.prof = nullptr;
    // the control block starts zeroed (the finalize step reads it and, with
    // update_ctl = 0, only fills the residuals); a fill kernel rather than a
    // memset keeps the call capturable. Every partial slot of every workgroup
    // is written by the two sweeps below, so the partial rows need no clearing.
    hipLaunchKernelGGL(kb_clear_words, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(ctl),
                       (int)(sizeof(Ctl) / sizeof(uint32_t)));
    HIP_OK(hipGetLastError());
    int rc = upload_inst(E, inst_of<T>(P, (double*)phi, (T*)nullptr, (T*)q, (T*)nullptr, (double*)alpha, (T*)beta,
                                       (T*)nullptr, (double*)nullptr, ctl, partials),
                         st);
    if (rc) return rc;
    hipLaunchKernelGGL((kb_zres<T, D>), dim3(E.grid_nodes), dim3(kBlock), 0, st, (const Inst<T>*)E.d_inst,
                       (const T*)z);
    HIP_OK(hipGetLastError());
    if ((rc = check_iter<T, D>(E, 0, 0, st))) return rc;
    HIP_OK(hipMemcpyAsync(P->host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    return DOT_OK;
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
  if (p->sigma0 < 0 || !std::isfinite(p->sigma0)) return fail(DOT_EINVAL, "sigma0 must be > 0 (0 selects 30)");
  if (p->check_every < 0) return fail(DOT_EINVAL, "check_every must be >= 0");
  if (p->sigma_gap0 < 0 || p->sigma_growth < 0) return fail(DOT_EINVAL, "sigma schedule must be >= 0");
  if (!(p->time_limit_s >= 0) || !std::isfinite(p->time_limit_s))
    return fail(DOT_EINVAL, "time_limit_s must be >= 0 and finite");
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

int extract_impl(dot_plan* P, const void* state, double* rho_out, double* m_out, hipStream_t st) {
  // rho = alpha0 on the cells, m_d = alpha_d on G^s_d (alpha planes are FP64)
  const Geo& g = P->g;
  std::vector<double> buf(g.nb);
  const char* base = static_cast<const char*>(state) + P->off_alpha;
  if (rho_out) {
    HIP_OK(hipMemcpyAsync(buf.data(), base, g.nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const int64_t ncell = (int64_t)g.n[0] * g.nx;
    for (int64_t i = 0; i < ncell; ++i) rho_out[i] = buf[i];
  }
  if (m_out) {
    size_t o = 0;
    for (int d = 1; d <= P->D; ++d) {
      HIP_OK(hipMemcpyAsync(buf.data(), base + (size_t)d * g.nb * sizeof(double), g.nb * sizeof(double),
                            hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      for (int64_t i = 0; i < g.nb; ++i) {
        const int64_t r = i / g.stride[d];
        const int xd = (int)(r % g.N[d]);
        if (xd < g.n[d]) m_out[o++] = buf[i];
      }
    }
  }
  return DOT_OK;
}

}  // namespace

// A batch: one plan per instance, all instance states in one caller workspace
// (control blocks first, contiguous, so one copy polls every stop flag), and
// one executor whose launches cover every instance.
struct dot_batch {
  std::vector<dot_plan*> plans;
  int D = 0, precision = 0, cadence = 5;
  size_t ctl_stride = 256;
  std::vector<size_t> state_off;  // byte offset of each instance state in the workspace
  size_t ws_bytes = 0;
  void* d_inst = nullptr;
  uint16_t* d_maps = nullptr;  // node map, then one map per axis
  Sched sched;                 // transform schedule of the batch launches
  Exec E;
  Ctl* host_ctl = nullptr;     // pinned, one entry per instance at ctl_stride
  int it = 0;                  // iterations done (all instances in lockstep)
  std::vector<char> active;    // instances laid out in the launch grids (empty: all)
  Prof prof;
  GraphCache graphs;
};

namespace {

// Whether instance i of a batch has workgroups in its launch grids.
bool laid_out(const dot_batch* B, int i) { return B->active.empty() || B->active[i]; }

// Block maps (block -> instance; the node grid first, then one per axis) and
// the per-axis launch geometry of a batch under schedule s, over the
// instances marked in `act` (nullptr: those laid out now; empty: all). The
// new maps are uploaded before anything of the old layout changes, so on
// failure the batch keeps its previous layout and schedule; on success s
// becomes B->sched and `act` B->active. Which instances share the grids and
// the schedule change no computed value: an instance's workgroups index its
// own planes by their position among its own blocks.
int batch_layout(dot_batch* B, const Sched& s, const std::vector<char>* act = nullptr) {
  DevLock lk(g_dev_mu);
  const std::vector<char> on = act ? *act : B->active;
  const int count = (int)B->plans.size();
  std::vector<dot_plan*> plans;
  std::vector<int> idx;
  for (int i = 0; i < count; ++i)
    if (on.empty() || on[i]) {
      plans.push_back(B->plans[i]);
      idx.push_back(i);
    }
  if (plans.empty()) return fail(DOT_EINVAL, "a batch layout needs at least one instance");
  const int n = (int)plans.size();
  std::vector<uint16_t> maps;
  for (int k = 0; k < n; ++k) maps.insert(maps.end(), (size_t)plans[k]->nblocks, (uint16_t)idx[k]);
  size_t map_off[kMaxAxes] = {0, 0, 0, 0};
  AxisGeom ag[kMaxAxes];
  for (int a = 0; a <= B->D; ++a) {
    map_off[a] = maps.size();
    ag[a] = B->precision == DOT_FP64 ? axis_geom<double>(plans.data(), n, a, s)
                                     : axis_geom<float>(plans.data(), n, a, s);
    for (int k = 0; k < n; ++k)
      maps.insert(maps.end(), (size_t)tiles_for(plans[k]->lines[a], ag[a].cw), (uint16_t)idx[k]);
  }
  uint16_t* fresh = nullptr;
  HIP_OK(hipMalloc((void**)&fresh, maps.size() * sizeof(uint16_t)));
  const hipError_t e = hipMemcpy(fresh, maps.data(), maps.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(fresh);
    return fail(DOT_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  if (B->d_maps) {
    HIP_OK(hipDeviceSynchronize());  // no launch of the old layout is still reading its maps
    (void)hipFree(B->d_maps);
  }
  B->d_maps = fresh;
  B->sched = s;
  B->active = on;
  Exec& E = B->E;
  E.nact = n;
  E.grid_nodes = (unsigned)map_off[0];
  E.ntri = 0;
  E.ntri_long = 0;
  E.nstaged = 0;
  E.nodes = 0;
  for (dot_plan* P : plans) {
    E.ntri += P->tri ? 1 : 0;
    E.ntri_long += P->tri && P->g.N[P->D] > kTriPartMaxNodes ? 1 : 0;
    E.nstaged += P->nblocks >= kFinStageMinRows ? 1 : 0;
    E.nodes += P->g.nb;
  }
  E.map_nodes = B->d_maps;
  for (int a = 0; a <= B->D; ++a) {
    E.map_axis[a] = B->d_maps + map_off[a];
    E.cw_axis[a] = ag[a].cw;
    E.grid_axis[a] = (unsigned)ag[a].tiles;
    E.smem_axis[a] = ag[a].smem;
    E.waves_axis[a] = ag[a].waves;
  }
  return DOT_OK;
}

template <typename T>
int batch_descriptors(dot_batch* B, void* ws, hipStream_t st) {
  const int count = (int)B->plans.size();
  std::vector<Inst<T>> host(count);
  uint32_t blk = 0;
  uint32_t tile[kMaxAxes] = {0, 0, 0, 0};
  for (int i = 0; i < count; ++i) {
    dot_plan* P = B->plans[i];
    Ctl* ctl = reinterpret_cast<Ctl*>(static_cast<char*>(ws) + (size_t)i * B->ctl_stride);
    host[i] = state_inst<T>(P, static_cast<char*>(ws) + B->state_off[i], ctl);
    if (!laid_out(B, i)) continue;  // no workgroup maps to it (blk0 and tile0 stay 0)
    host[i].blk0 = blk;
    blk += (uint32_t)P->nblocks;
    for (int a = 0; a <= B->D; ++a) {
      host[i].tile0[a] = tile[a];
      tile[a] += (uint32_t)tiles_for(P->lines[a], B->E.cw_axis[a]);
    }
  }
  HIP_OK(hipMemcpyAsync(B->d_inst, host.data(), sizeof(Inst<T>) * count, hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  return DOT_OK;
}

// Compaction: lays the batch out over the instances that have not stopped,
// by the control blocks in B->host_ctl, so that a stopped instance's
// workgroups (each reads its descriptor and stop flag, then returns) stop
// taking dispatch slots. With `any_change` the layout follows every change of
// that set (instances that run again after a reset come back); otherwise it
// drops stopped instances once they hold at least 1/8 of the node-grid
// workgroups. Keeps the layout when no instance runs.
template <typename T>
int batch_compact(dot_batch* B, void* ws, hipStream_t st, bool any_change) {
  const int count = (int)B->plans.size();
  std::vector<char> now(count);
  int64_t dropped = 0, kept = 0;
  int live = 0;
  bool differs = false;
  for (int i = 0; i < count; ++i) {
    const Ctl* c = reinterpret_cast<const Ctl*>(reinterpret_cast<const char*>(B->host_ctl) + (size_t)i * B->ctl_stride);
    now[i] = c->stop ? 0 : 1;
    live += now[i];
    const bool was = laid_out(B, i);
    differs = differs || (was != (now[i] != 0));
    if (was && !now[i]) dropped += B->plans[i]->nblocks;
    if (now[i]) kept += B->plans[i]->nblocks;
    if (!was && now[i]) any_change = true;  // an instance to bring back: always
  }
  if (live == 0 || !differs) return DOT_OK;
  if (!any_change && dropped * 8 < dropped + kept) return DOT_OK;
  drop_graph(B->graphs);
  int rc = batch_layout(B, B->sched, &now);
  if (rc) return rc;
  return batch_descriptors<T>(B, ws, st);
}

template <typename T, int D>
struct BatchRunF {
  static int run(dot_batch* B, void* ws, int max_iters, hipStream_t st, int* done, bool* timed_out) {
    const int count = (int)B->plans.size();
    HIP_OK(hipMemcpyAsync(B->host_ctl, ws, B->ctl_stride * count, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const char* hc = reinterpret_cast<const char*>(B->host_ctl);
    bool any_running = false;
    for (int i = 0; i < count; ++i)
      any_running = any_running || !reinterpret_cast<const Ctl*>(hc + (size_t)i * B->ctl_stride)->stop;
    if (!any_running) {  // nothing to iterate: no launch at all
      if (done) *done = 0;
      return DOT_OK;
    }
    int rc = batch_compact<T>(B, ws, st, true);
    if (rc || (rc = batch_descriptors<T>(B, ws, st))) return rc;
    // the smallest time budget of the instances bounds the call
    double limit = 0.0;
    for (auto* P : B->plans)
      if (P->time_limit > 0.0) limit = limit > 0.0 ? std::min(limit, P->time_limit) : P->time_limit;
    const std::function<int()> compact = [&]() { return batch_compact<T>(B, ws, st, false); };
    return run_iters<T, D>(B->E, B->it, max_iters, ws, B->ctl_stride, B->host_ctl, st, done, -1, limit, timed_out,
                           &compact);
  }
};

// ---- transform schedule autotuning ----------------------------------------

// Whether every instance of a launch can run the passes over axis a with
// tiles of cw lines and `waves` waves per workgroup.
template <typename T>
bool schedule_ok(dot_plan* const* plans, int count, int a, int cw, int waves, int max_smem) {
  bool all_tri = true;
  for (int i = 0; i < count; ++i) all_tri = all_tri && plans[i]->tri;
  if (waves < 1 || waves > kMaxWaves) return false;
  if (a == plans[0]->D && all_tri) return tri_cw_ok(plans, count, cw);
  if (cw != kCWNarrow && cw != kCWMid && cw != kCW) return false;
  for (int i = 0; i < count; ++i) {
    if (a == plans[i]->D && plans[i]->tri) continue;  // only the tridiagonal solve runs there
    const int L = plans[i]->g.N[a];
    if (!axis_fits<T>(L, cw, max_smem)) return false;
    if (waves * wave_items<T>(cw) < pass_items(L, cw)) return false;
  }
  return true;
}

// A caller's schedule (zeros: the rule's) checked against the instances.
template <typename T>
int schedule_from(dot_plan* const* plans, int count, const dot_schedule* in, Sched* out) {
  Sched s;
  if (in) {
    int max_smem = 0;
    HIP_OK(hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, plans[0]->device));
    for (int a = 0; a <= plans[0]->D; ++a) {
      if (!in->cw[a] && !in->waves[a]) continue;
      Sched t;
      t.cw[a] = in->cw[a];
      const AxisGeom ag = axis_geom<T>(plans, count, a, t);
      const int cw = ag.cw, w = in->waves[a] ? in->waves[a] : ag.waves;
      if (!schedule_ok<T>(plans, count, a, cw, w, max_smem))
        return fail(DOT_EINVAL, "axis " + std::to_string(a) + ": no launch of " + std::to_string(cw) +
                                    "-line tiles with " + std::to_string(w) + " waves for these instances");
      s.cw[a] = cw;
      s.waves[a] = w;
    }
  }
  *out = s;
  return DOT_OK;
}

// One transform sequence of an executor (every pass of one phi-step, as an
// iteration launches them), timed with HIP events on its stream: one warm-up
// sequence, then the fastest of three runs of about 2 ms each.
template <typename T, int D>
int time_passes(const Exec& E, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double* us) {
  auto seq = [&]() -> int {
    if constexpr (std::is_same<T, double>::value)
      return run_passes<double, D, kSrcPlane, kDstPlane>(E, 0, 0.0, st);
    else
      return run_passes<T, D, kSrcPlane, kDstPhiAdd>(E, 0, 0.0, st);
  };
  int rc = seq();
  if (rc) return rc;
  float ms = 0.f;
  HIP_OK(hipEventRecord(e0, st));
  if ((rc = seq())) return rc;
  HIP_OK(hipEventRecord(e1, st));
  HIP_OK(hipEventSynchronize(e1));
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  const int reps = std::max(3, std::min(64, (int)(2.0 / std::max(1e-3, (double)ms))));
  double best = 1e300;
  for (int trial = 0; trial < 3; ++trial) {
    HIP_OK(hipEventRecord(e0, st));
    for (int r = 0; r < reps && !rc; ++r) rc = seq();
    HIP_OK(hipEventRecord(e1, st));
    HIP_OK(hipEventSynchronize(e1));
    if (rc) return rc;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, 1000.0 * ms / reps);
  }
  *us = best;
  return DOT_OK;
}

struct EventPair {
  hipEvent_t e[2] = {nullptr, nullptr};
  ~EventPair() {
    for (auto x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

// Coordinate descent over the axes: on each axis in turn every candidate is
// timed with the other axes at their best so far; the result is compared
// once more with the rule's schedule, alternating, and the rule is kept
// unless the measured schedule is faster. apply(s, &E) installs s on the
// executor under test and returns its geometry.
template <typename T, int D, typename Apply>
int tune_schedule(Apply&& apply, const std::vector<std::vector<std::pair<int, int>>>& cands, hipStream_t st,
                  Sched* out) {
  EventPair ev;
  HIP_OK(hipEventCreate(&ev.e[0]));
  HIP_OK(hipEventCreate(&ev.e[1]));
  Exec E;
  const Sched rule;
  int rc = apply(rule, &E);
  double t_best = 0.0;
  if (rc || (rc = time_passes<T, D>(E, st, ev.e[0], ev.e[1], &t_best))) return rc;
  Sched rule_x;  // the rule's schedule written out
  for (int a = 0; a <= D; ++a) {
    rule_x.cw[a] = E.cw_axis[a];
    rule_x.waves[a] = E.waves_axis[a];
  }
  Sched best = rule_x;
  int n = 1;
  for (int a = 0; a <= D; ++a) {
    for (const auto& c : cands[a]) {
      if (c.first == best.cw[a] && c.second == best.waves[a]) continue;
      Sched s = best;
      s.cw[a] = c.first;
      s.waves[a] = c.second;
      double t = 0.0;
      if ((rc = apply(s, &E)) || (rc = time_passes<T, D>(E, st, ev.e[0], ev.e[1], &t))) return rc;
      ++n;
      if (t < t_best) {
        t_best = t;
        best = s;
      }
    }
  }
  double t_rule = 1e300, t_tuned = 1e300;
  for (int k = 0; k < 2; ++k) {
    double t = 0.0;
    if ((rc = apply(rule_x, &E)) || (rc = time_passes<T, D>(E, st, ev.e[0], ev.e[1], &t))) return rc;
    t_rule = std::min(t_rule, t);
    if ((rc = apply(best, &E)) || (rc = time_passes<T, D>(E, st, ev.e[0], ev.e[1], &t))) return rc;
    t_tuned = std::min(t_tuned, t);
  }
  if (!(t_tuned < t_rule)) {
    best = rule_x;
    t_tuned = t_rule;
  }
  best.tuned = true;
  best.candidates = n;
  best.us = t_tuned;
  best.us_rule = t_rule;
  if ((rc = apply(best, &E))) return rc;
  *out = best;
  return DOT_OK;
}

template <typename T>
std::vector<std::vector<std::pair<int, int>>> all_candidates(dot_plan* const* plans, int count) {
  int max_smem = 0;
  (void)hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, plans[0]->device);
  std::vector<std::vector<std::pair<int, int>>> c;
  for (int a = 0; a <= plans[0]->D; ++a) c.push_back(axis_candidates<T>(plans, count, a, max_smem));
  return c;
}

template <typename T, int D>
struct PlanTuneF {
  static int run(dot_plan* P, void* state, hipStream_t st) {
    Ctl* ctl = at<Ctl>(state, P->ctl_offset);
    int rc = upload_inst(plan_exec(P, 0), state_inst<T>(P, state, ctl), st);
    if (rc) return rc;
    auto apply = [&](const Sched& s, Exec* E) -> int {
      P->sched = s;
      *E = plan_exec(P, 0);
      E->prof = nullptr;
      E->graphs = nullptr;
      return DOT_OK;
    };
    Sched out;
    rc = tune_schedule<T, D>(apply, all_candidates<T>(&P, 1), st, &out);
    if (rc) return rc;
    P->sched = out;
    return DOT_OK;
  }
};

template <typename T, int D>
struct BatchTuneF {
  static int run(dot_batch* B, void* ws, hipStream_t st) {
    auto apply = [&](const Sched& s, Exec* E) -> int {
      int rc = batch_layout(B, s);
      if (rc || (rc = batch_descriptors<T>(B, ws, st))) return rc;
      *E = B->E;
      E->prof = nullptr;
      E->graphs = nullptr;
      return DOT_OK;
    };
    Sched out;
    int rc = tune_schedule<T, D>(apply, all_candidates<T>(B->plans.data(), (int)B->plans.size()), st, &out);
    if (rc) return rc;
    B->sched = out;  // the layout of `out` is in place (tune_schedule applies it last)
    return DOT_OK;
  }
};

void schedule_out(const Sched& s, const Exec& E, int D, dot_schedule* o) {
  std::memset(o, 0, sizeof(*o));
  for (int a = 0; a <= D; ++a) {
    o->cw[a] = E.cw_axis[a];
    o->waves[a] = E.waves_axis[a];
  }
  o->tuned = s.tuned ? 1 : 0;
  o->candidates = s.candidates;
  o->us = s.us;
  o->us_rule = s.us_rule;
}

}  // namespace

extern "C" {

const char* dot_last_error(void) { return g_err.c_str(); }

void dot_plan_destroy(dot_plan* P) {
  DevLock lk(g_dev_mu);
  if (!P) return;
  (void)hipFree(P->sw_sp);
  (void)hipFree(P->om_sp);
  (void)hipFree(P->c_lo);
  (void)hipFree(P->c_hi);
  (void)hipFree(P->lam_other);
  (void)hipFree(P->lam_last);
  for (auto* b : P->axis_buf) (void)hipFree(b);
  (void)hipFree(P->d_inst);
  (void)hipFree(P->step_ctl);
  (void)hipFree(P->step_partials);
  (void)hipFree(P->step_cbuf);
  (void)hipFree(P->step_scratch);
  (void)hipHostFree(P->host_ctl);
  delete P;
}

int dot_plan_create(const dot_problem* p, dot_plan** out) {
  DevLock lk(g_dev_mu);
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
  P->sigma0 = p->sigma0 > 0 ? p->sigma0 : 30.0;
  P->tol = p->tol;
  P->max_iter = p->max_iter;
  P->cadence = p->check_every > 0 ? p->check_every : 5;
  P->adapt = p->adapt_sigma;
  P->gap0 = p->sigma_gap0 > 0 ? p->sigma_gap0 : 10;
  P->growth = p->sigma_growth > 0 ? p->sigma_growth : 1.2;
  P->time_limit = p->time_limit_s;
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
  P->tri = g.N[D] >= kTriMinNodes;
  for (int a = 0; a <= D; ++a) {
    P->lines[a] = g.nb / g.N[a];
    // a last axis solved by tridiagonal elimination is never transformed,
    // whatever its length: no tile limits apply to it
    if (a == D && P->tri) continue;
    auto fits = [&](int cw) {
      return P->precision == DOT_FP64 ? axis_fits<double>(g.N[a], cw, max_smem)
                                      : axis_fits<float>(g.N[a], cw, max_smem);
    };
    if (!fits(kCWNarrow))
      return fail(DOT_EINVAL, "axis of " + std::to_string(g.N[a]) + " nodes exceeds the transform tile capacity");
    P->wide_ok[a] = fits(kCW);
    P->mid_ok[a] = fits(kCWMid) && pass_smem(g.N[a], P->scalar_bytes, kCWMid) <= kMidLds;
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
    if (a == D && P->tri) continue;  // no transform tables for an eliminated axis
    rc = P->precision == DOT_FP64 ? build_axis<double>(P.get(), a, &P->axis_buf[a], &P->tab64[a])
                                  : build_axis<float>(P.get(), a, &P->axis_buf[a], &P->tab32[a]);
    if (rc) return rc;
  }
  rc = P->precision == DOT_FP64 ? build_eigs<double>(P.get()) : build_eigs<float>(P.get());
  if (rc) return rc;
  const size_t pb = (size_t)g.nb * P->scalar_bytes;
  const StateLayout lay = state_layout(D, g.nb, P->precision);
  P->off_phi = lay.off_phi;
  P->off_scr = lay.off_scr;
  P->off_q = lay.off_q;
  P->off_qn = lay.off_qn;
  P->off_alpha = lay.off_alpha;
  P->off_beta = lay.off_beta;
  P->off_w = lay.off_w;
  P->n_planes = 2 * (D + 1) + P->K + 4 * D;
  set_sweep(g, default_tc(g.nx, g.N[0]));
  P->nblocks = g.nsweep;
  P->partial_rows = (int64_t)g.nxb * g.N[0];
  P->off_dw = lay.off_dw;
  P->ctl_offset = lay.ctl_offset;
  P->partials_offset = P->ctl_offset + align256(sizeof(Ctl));
  // partial rows, then the stage rows of their first reduction stage
  const size_t partial_bytes = (size_t)(P->partial_rows + kFinChunks) * kNumSums * sizeof(double);
  P->state_bytes = P->partials_offset + align256(partial_bytes);
  if (P->precision == DOT_MIXED) HIP_OK(hipMalloc(&P->step_scratch, pb));
  HIP_OK(hipMalloc((void**)&P->step_ctl, sizeof(Ctl)));
  HIP_OK(hipMalloc((void**)&P->step_partials, partial_bytes));
  HIP_OK(hipMemset(P->step_partials, 0, partial_bytes));
  HIP_OK(hipHostMalloc((void**)&P->host_ctl, sizeof(Ctl), hipHostMallocDefault));
  HIP_OK(hipMalloc(&P->d_inst, 2 * inst_slot_bytes()));
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
  *P->host_ctl = initial_ctl(P);
  HIP_OK(hipMemcpyAsync(at<Ctl>(state, P->ctl_offset), P->host_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  return DOT_OK;
}

int dot_run(dot_plan* P, void* state, int32_t max_iters, void* stream, dot_result* res) {
  if (!P || !state || max_iters < 0) return fail(DOT_EINVAL, "bad argument");
  return dispatch<RunF>(P->precision, P->D, P, state, (int)max_iters, (hipStream_t)stream, res);
}

int dot_extract(dot_plan* P, const void* state, double* rho_out, double* m_out, void* stream) {
  if (!P || !state) return fail(DOT_EINVAL, "null argument");
  return extract_impl(P, state, rho_out, m_out, (hipStream_t)stream);
}

int dot_step_divergence(dot_plan* P, const void* q, const void* alpha, double sigma, void* b, void* stream) {
  if (!P || !q || !alpha || !b || !(sigma > 0)) return fail(DOT_EINVAL, "bad argument");
  return dispatch<DivF>(P->precision, P->D, P, q, alpha, sigma, b, (hipStream_t)stream);
}

int dot_step_poisson(dot_plan* P, void* b, void* stream) {
  if (!P || !b) return fail(DOT_EINVAL, "bad argument");
  return dispatch<PoissonF>(P->precision, P->D, P, b, (const void*)nullptr, (const void*)nullptr, 1.0,
                            (hipStream_t)stream);
}

int dot_step_rhs_poisson(dot_plan* P, const void* q, const void* alpha, double sigma, void* phi, void* stream) {
  if (!P || !q || !alpha || !phi || !(sigma > 0)) return fail(DOT_EINVAL, "bad argument");
  return dispatch<PoissonF>(P->precision, P->D, P, phi, q, alpha, sigma, (hipStream_t)stream);
}

int dot_step_cone(dot_plan* P, const void* q, const void* beta, double sigma, void* z, void* stream) {
  if (!P || !q || !beta || !z || !(sigma > 0)) return fail(DOT_EINVAL, "bad argument");
  return dispatch<ConeF>(P->precision, P->D, P, q, beta, sigma, z, (hipStream_t)stream);
}

int dot_step_update(dot_plan* P, const void* phi, const void* q, void* alpha, void* beta, double sigma, double tau,
                    void* q_out, void* w_scratch, void* stream) {
  if (!P || !phi || !q || !alpha || !beta || !q_out || !w_scratch || !(sigma > 0) || !(tau > 0))
    return fail(DOT_EINVAL, "bad argument");
  return dispatch<UpdateF>(P->precision, P->D, P, phi, q, alpha, beta, sigma, tau, q_out, w_scratch,
                           (hipStream_t)stream);
}

int dot_step_residuals(dot_plan* P, const void* phi, const void* z, const void* q, const void* alpha,
                       const void* beta, dot_result* res, void* stream) {
  if (!P || !phi || !z || !q || !alpha || !beta || !res) return fail(DOT_EINVAL, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = dispatch<ResidF>(P->precision, P->D, P, phi, z, q, alpha, beta, st);
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(P->host_ctl, P->step_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  std::memset(res, 0, sizeof(*res));
  fill_result(*P->host_ctl, res);
  res->iters = 0;
  res->checks = 0;
  res->term = DOT_RUNNING;
  return DOT_OK;
}

int dot_step_residuals_noalloc(dot_plan* P, const void* phi, const void* z, const void* q, const void* alpha,
                               const void* beta, dot_result* res, void* stream) {
  if (!P || !phi || !z || !q || !alpha || !beta || !res) return fail(DOT_EINVAL, "bad argument");
  if (noalloc_bytes(P) > (size_t)DOT_NOALLOC_SCRATCH_BYTES)
    return fail(DOT_EINVAL, "the residual sweep of this grid needs " + std::to_string(noalloc_bytes(P)) +
                                " bytes of scratch, more than the " + std::to_string((size_t)DOT_NOALLOC_SCRATCH_BYTES) +
                                " of dot_step_residuals_noalloc");
  int cur = -1;
  HIP_OK(hipGetDevice(&cur));
  if (cur != P->device) return fail(DOT_EINVAL, "the plan's device must be the current device");
  unsigned char* scr = nullptr;
  int rc = noalloc_ptr(cur, &scr);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  rc = dispatch<ResidNoAllocF>(P->precision, P->D, P, phi, z, q, alpha, beta, scr, st);
  if (rc) return rc;
  HIP_OK(hipStreamSynchronize(st));
  std::memset(res, 0, sizeof(*res));
  fill_result(*P->host_ctl, res);
  res->iters = 0;
  res->checks = 0;
  res->term = DOT_RUNNING;
  return DOT_OK;
}

int dot_profile_select(dot_plan* P, int32_t kernel_class) {
  if (!P || kernel_class < -1 || kernel_class > DOT_K_RHS) return fail(DOT_EINVAL, "bad kernel class");
  P->prof.cls = kernel_class;
  P->prof.used = 0;
  P->prof.ms = 0.0;
  P->prof.launches = 0;
  return DOT_OK;
}

int dot_profile_read(dot_plan* P, double* total_ms, int64_t* launches) {
  if (!P) return fail(DOT_EINVAL, "null plan");
  if (total_ms) *total_ms = P->prof.ms;
  if (launches) *launches = P->prof.launches;
  P->prof.ms = 0.0;
  P->prof.launches = 0;
  return DOT_OK;
}

int dot_test_fail_captures(int32_t count) {
  if (count < 0) return fail(DOT_EINVAL, "count must be >= 0");
  g_fail_captures.store(count);
  return DOT_OK;
}

int dot_plan_set_graphs(dot_plan* P, int32_t enable) {
  if (!P) return fail(DOT_EINVAL, "null plan");
  P->graphs.enabled = enable != 0;
  drop_graph(P->graphs);  // the next run captures anew
  return DOT_OK;
}

int dot_solve(const dot_problem* p, double* rho_out, double* m_out, dot_result* res) {
  dot_plan* P = nullptr;
  int rc = dot_plan_create(p, &P);
  if (rc) return rc;
  void* state = nullptr;
  hipError_t e;
  {
    DevLock lk(g_dev_mu);
    e = hipMalloc(&state, P->state_bytes);
  }
  if (e != hipSuccess) {
    dot_plan_destroy(P);
    return fail(DOT_ENOMEM, "state allocation failed");
  }
  rc = dot_state_reset(P, state, nullptr);
  if (!rc) rc = dot_run(P, state, p->max_iter, nullptr, res);
  if (!rc) rc = dot_extract(P, state, rho_out, m_out, nullptr);
  {
    DevLock lk(g_dev_mu);
    (void)hipFree(state);
  }
  dot_plan_destroy(P);
  return rc;
}

// ---- batches ---------------------------------------------------------------

void dot_batch_destroy(dot_batch* B) {
  DevLock lk(g_dev_mu);
  if (!B) return;
  for (auto* p : B->plans) dot_plan_destroy(p);
  (void)hipFree(B->d_inst);
  (void)hipFree(B->d_maps);
  (void)hipHostFree(B->host_ctl);
  delete B;
}

int dot_batch_create(const dot_problem* probs, int32_t count, dot_batch** out) {
  DevLock lk(g_dev_mu);
  if (!out || !probs || count < 1 || count > 65535) return fail(DOT_EINVAL, "bad batch arguments");
  *out = nullptr;
  std::unique_ptr<dot_batch, void (*)(dot_batch*)> B(new (std::nothrow) dot_batch(), dot_batch_destroy);
  if (!B) return fail(DOT_ENOMEM, "host allocation failed");
  auto cad = [](const dot_problem& p) { return p.check_every > 0 ? p.check_every : 5; };
  // every problem is checked before any device work
  for (int i = 0; i < count; ++i) {
    if (probs[i].D != probs[0].D || probs[i].precision != probs[0].precision || cad(probs[i]) != cad(probs[0]))
      return fail(DOT_EINVAL, "all problems of a batch need the same D, precision and check cadence");
    const int rc = validate(&probs[i]);
    if (rc) return fail(rc, "problem " + std::to_string(i) + ": " + g_err);
  }
  for (int i = 0; i < count; ++i) {
    dot_plan* P = nullptr;
    int rc = dot_plan_create(&probs[i], &P);
    if (rc) return fail(rc, "problem " + std::to_string(i) + ": " + g_err);
    B->plans.push_back(P);
  }
  const int D = probs[0].D;
  B->D = D;
  B->precision = probs[0].precision;
  B->cadence = B->plans[0]->cadence;
  B->ctl_stride = align256(sizeof(Ctl));
  size_t off = align256(B->ctl_stride * count);
  for (auto* P : B->plans) {
    B->state_off.push_back(off);
    off += align256(P->state_bytes);
  }
  B->ws_bytes = off;
  Exec& E = B->E;
  E.D = D;
  E.precision = B->precision;
  E.ninst = count;
  E.cadence = B->cadence;
  E.device = B->plans[0]->device;
  int rc = batch_layout(B.get(), Sched());
  if (rc) return rc;
  const size_t isz = B->precision == DOT_FP64 ? sizeof(Inst<double>) : sizeof(Inst<float>);
  HIP_OK(hipMalloc(&B->d_inst, isz * count));
  E.d_inst = B->d_inst;
  E.prof = &B->prof;
  E.graphs = &B->graphs;
  HIP_OK(hipHostMalloc((void**)&B->host_ctl, B->ctl_stride * count, hipHostMallocDefault));
  *out = B.release();
  return DOT_OK;
}

size_t dot_batch_workspace_bytes(const dot_batch* B) { return B ? B->ws_bytes : 0; }

int32_t dot_batch_size(const dot_batch* B) { return B ? (int32_t)B->plans.size() : 0; }

int32_t dot_batch_laid_out(const dot_batch* B) {
  if (!B) return -1;
  if (B->active.empty()) return (int32_t)B->plans.size();
  int32_t n = 0;
  for (char a : B->active) n += a ? 1 : 0;
  return n;
}

int dot_batch_reset(dot_batch* B, void* ws, void* stream) {
  if (!B || !ws) return fail(DOT_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const int count = (int)B->plans.size();
  for (int i = 0; i < count; ++i) {
    dot_plan* P = B->plans[i];
    HIP_OK(hipMemsetAsync(static_cast<char*>(ws) + B->state_off[i], 0, P->ctl_offset, st));
    *reinterpret_cast<Ctl*>(reinterpret_cast<char*>(B->host_ctl) + (size_t)i * B->ctl_stride) = initial_ctl(P);
  }
  HIP_OK(hipMemcpyAsync(ws, B->host_ctl, B->ctl_stride * count, hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  B->it = 0;
  if (!B->active.empty()) {
    // every instance runs again: lay them all out (a compacted layout left some out)
    drop_graph(B->graphs);
    const std::vector<char> all;
    return batch_layout(B, B->sched, &all);
  }
  return DOT_OK;
}

int dot_batch_run(dot_batch* B, void* ws, int32_t max_iters, void* stream, dot_result* results) {
  if (!B || !ws || max_iters < 0) return fail(DOT_EINVAL, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  int done = 0;
  bool timed_out = false;
  const auto t0 = std::chrono::steady_clock::now();
  int rc = dispatch<BatchRunF>(B->precision, B->D, B, ws, (int)max_iters, st, &done, &timed_out);
  if (rc) return rc;
  const double elapsed = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  B->it += done;
  if (results)
    for (size_t i = 0; i < B->plans.size(); ++i) {
      const Ctl& c = *reinterpret_cast<const Ctl*>(reinterpret_cast<char*>(B->host_ctl) + i * B->ctl_stride);
      fill_result(c, &results[i]);
      // the call ended early at the smallest budget: instances whose own
      // budget ran out report DOT_TIMEOUT, the other unfinished ones
      // DOT_RUNNING (their state is resumable as well)
      if (timed_out && !c.stop) {
        const double own = B->plans[i]->time_limit;
        results[i].term = own > 0.0 && elapsed >= own ? DOT_TIMEOUT : DOT_RUNNING;
      }
    }
  return DOT_OK;
}

int dot_batch_extract(dot_batch* B, const void* ws, int32_t index, double* rho_out, double* m_out, void* stream) {
  if (!B || !ws || index < 0 || index >= (int)B->plans.size()) return fail(DOT_EINVAL, "bad argument");
  return extract_impl(B->plans[index], static_cast<const char*>(ws) + B->state_off[index], rho_out, m_out,
                      (hipStream_t)stream);
}

int dot_batch_set_graphs(dot_batch* B, int32_t enable) {
  if (!B) return fail(DOT_EINVAL, "null batch");
  B->graphs.enabled = enable != 0;
  drop_graph(B->graphs);  // the next run captures anew
  return DOT_OK;
}

int dot_plan_set_schedule(dot_plan* P, const dot_schedule* s) {
  if (!P) return fail(DOT_EINVAL, "null plan");
  Sched x;
  int rc = P->precision == DOT_FP64 ? schedule_from<double>(&P, 1, s, &x) : schedule_from<float>(&P, 1, s, &x);
  if (rc) return rc;
  P->sched = x;
  drop_graph(P->graphs);
  return DOT_OK;
}

int dot_plan_get_schedule(const dot_plan* P, dot_schedule* out) {
  if (!P || !out) return fail(DOT_EINVAL, "null argument");
  schedule_out(P->sched, plan_exec(const_cast<dot_plan*>(P), 0), P->D, out);
  return DOT_OK;
}

int dot_plan_autotune(dot_plan* P, void* state, void* stream, dot_schedule* out) {
  if (!P || !state) return fail(DOT_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = dot_state_reset(P, state, stream);
  if (rc) return rc;
  drop_graph(P->graphs);
  const Sched keep = P->sched;
  rc = dispatch<PlanTuneF>(P->precision, P->D, P, state, st);
  if (rc) {
    P->sched = keep;
    return rc;
  }
  if ((rc = dot_state_reset(P, state, stream))) return rc;
  if (out) return dot_plan_get_schedule(P, out);
  return DOT_OK;
}

int dot_batch_set_schedule(dot_batch* B, const dot_schedule* s) {
  if (!B) return fail(DOT_EINVAL, "null batch");
  dot_plan* const* plans = B->plans.data();
  const int count = (int)B->plans.size();
  Sched x;
  int rc = B->precision == DOT_FP64 ? schedule_from<double>(plans, count, s, &x)
                                    : schedule_from<float>(plans, count, s, &x);
  if (rc) return rc;
  drop_graph(B->graphs);
  return batch_layout(B, x);
}

int dot_batch_get_schedule(const dot_batch* B, dot_schedule* out) {
  if (!B || !out) return fail(DOT_EINVAL, "null argument");
  schedule_out(B->sched, B->E, B->D, out);
  return DOT_OK;
}

int dot_batch_autotune(dot_batch* B, void* ws, void* stream, dot_schedule* out) {
  if (!B || !ws) return fail(DOT_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = dot_batch_reset(B, ws, stream);
  if (rc) return rc;
  drop_graph(B->graphs);
  const Sched keep = B->sched;
  rc = dispatch<BatchTuneF>(B->precision, B->D, B, ws, st);
  if (rc) {
    (void)batch_layout(B, keep);  // back to the schedule in use before the call
    return rc;
  }
  if ((rc = dot_batch_reset(B, ws, stream))) return rc;
  if (out) return dot_batch_get_schedule(B, out);
  return DOT_OK;
}

int dot_batch_profile_select(dot_batch* B, int32_t kernel_class) {
  if (!B || kernel_class < -1 || kernel_class > DOT_K_RHS) return fail(DOT_EINVAL, "bad kernel class");
  B->prof.cls = kernel_class;
  B->prof.used = 0;
  B->prof.ms = 0.0;
  B->prof.launches = 0;
  return DOT_OK;
}

int dot_batch_profile_read(dot_batch* B, double* total_ms, int64_t* launches) {
  if (!B) return fail(DOT_EINVAL, "null batch");
  if (total_ms) *total_ms = B->prof.ms;
  if (launches) *launches = B->prof.launches;
  B->prof.ms = 0.0;
  B->prof.launches = 0;
  return DOT_OK;
}

// ---- multilevel initialisation ------------------------------------------

int dot_coarsen_data(int32_t D, const int32_t* n, const double* rho0, const double* rho1, const uint8_t* mask,
                     double* rho0_out, double* rho1_out, uint8_t* mask_out) {
  if (D < 1 || D > 3 || !n || !rho0 || !rho1 || !rho0_out || !rho1_out || (mask && !mask_out))
    return fail(DOT_EINVAL, "bad coarsening arguments");
  for (int d = 0; d <= D; ++d)
    if (n[d] < 2 || n[d] % 2) return fail(DOT_EINVAL, "segment counts must be even (>= 2) to coarsen");
  // spatial node counts, fine and coarse; C order, last axis fastest
  std::vector<int64_t> Nf(D), Nc(D);
  for (int d = 0; d < D; ++d) {
    Nf[d] = n[d + 1] + 1;
    Nc[d] = n[d + 1] / 2 + 1;
  }
  int64_t cf = 1, cc = 1;
  for (int d = 0; d < D; ++d) {
    cf *= Nf[d];
    cc *= Nc[d];
  }
  // restrict one axis at a time: coarse i <- fine 2i (weight 1), 2i-1 and 2i+1 (weight 1/2)
  auto restrict_all = [&](const double* in, double* out) {
    std::vector<double> cur(in, in + cf), nxt;
    std::vector<int64_t> shape(Nf.begin(), Nf.end());
    for (int ax = 0; ax < D; ++ax) {
      int64_t outer = 1, inner = 1;
      for (int d = 0; d < ax; ++d) outer *= shape[d];
      for (int d = ax + 1; d < D; ++d) inner *= shape[d];
      const int64_t lf = shape[ax], lc = Nc[ax];
      nxt.assign((size_t)(outer * lc * inner), 0.0);
      for (int64_t o = 0; o < outer; ++o)
        for (int64_t j = 0; j < lf; ++j) {
          const double* srow = cur.data() + (o * lf + j) * inner;
          auto add = [&](int64_t ci, double wgt) {
            double* drow = nxt.data() + (o * lc + ci) * inner;
            for (int64_t k = 0; k < inner; ++k) drow[k] += wgt * srow[k];
          };
          if (j % 2 == 0) {
            add(j / 2, 1.0);
          } else {
            add((j - 1) / 2, 0.5);
            add((j + 1) / 2, 0.5);
          }
        }
      cur.swap(nxt);
      shape[ax] = lc;
    }
    std::copy(cur.begin(), cur.end(), out);
  };
  restrict_all(rho0, rho0_out);
  restrict_all(rho1, rho1_out);
  if (mask) {
    // coarse node i is an obstacle node when fine node 2i is; no mass there
    double s0 = 0.0, s1 = 0.0;
    for (int64_t c = 0; c < cc; ++c) {
      int64_t r = c, f = 0, mul = 1;
      for (int d = D - 1; d >= 0; --d) {
        const int64_t x = r % Nc[d];
        r /= Nc[d];
        f += 2 * x * mul;
        mul *= Nf[d];
      }
      mask_out[c] = mask[f];
      if (mask_out[c]) rho0_out[c] = rho1_out[c] = 0.0;
      s0 += rho0_out[c];
      s1 += rho1_out[c];
    }
    if (!(s0 > 0.0) || !(s1 > 0.0)) return fail(DOT_EINVAL, "coarse data has no mass outside the obstacles");
    for (int64_t c = 0; c < cc; ++c) {
      rho0_out[c] /= s0;
      rho1_out[c] /= s1;
    }
  }
  return DOT_OK;
}

}  // extern "C"

namespace {

template <typename T, int D>
struct ProlongF {
  static int run(const dot_plan* C, const void* cs, dot_plan* F, void* fs, hipStream_t st) {
    const char* c = static_cast<const char*>(cs);
    char* f = static_cast<char*>(fs);
    const dim3 blk(kBlock);
    const unsigned gx = (unsigned)((F->g.nb + kBlock - 1) / kBlock);
    // q0 / alpha0 / beta: cells (staggered in time); q_d / alpha_d: staggered on axis d
    hipLaunchKernelGGL((kb_prolong<T, D>), dim3(gx, 1), blk, 0, st, C->g, F->g,
                       (const T*)(c + C->off_q), (T*)(f + F->off_q), 1);
    hipLaunchKernelGGL((kb_prolong<double, D>), dim3(gx, 1), blk, 0, st, C->g, F->g,
                       (const double*)(c + C->off_alpha), (double*)(f + F->off_alpha), 1);
    hipLaunchKernelGGL((kb_prolong<T, D>), dim3(gx, (unsigned)C->K), blk, 0, st, C->g, F->g,
                       (const T*)(c + C->off_beta), (T*)(f + F->off_beta), 1);
    for (int d = 1; d <= D; ++d) {
      hipLaunchKernelGGL((kb_prolong<T, D>), dim3(gx, 1), blk, 0, st, C->g, F->g,
                         (const T*)(c + C->off_q) + (size_t)d * C->g.nb, (T*)(f + F->off_q) + (size_t)d * F->g.nb,
                         1 << d);
      hipLaunchKernelGGL((kb_prolong<double, D>), dim3(gx, 1), blk, 0, st, C->g, F->g,
                         (const double*)(c + C->off_alpha) + (size_t)d * C->g.nb,
                         (double*)(f + F->off_alpha) + (size_t)d * F->g.nb, 1 << d);
    }
    HIP_OK(hipGetLastError());
    return DOT_OK;
  }
};

// Fine state from a coarse one: phi, z and the work planes cleared, q,
// alpha and beta interpolated (the control block is left to the caller).
int prolong_planes(const dot_plan* C, const void* coarse_state, dot_plan* F, void* fine_state, hipStream_t st) {
  HIP_OK(hipMemsetAsync(fine_state, 0, F->ctl_offset, st));
  return dispatch<ProlongF>(C->precision, C->D, C, coarse_state, F, fine_state, st);
}

}  // namespace

namespace {

// Whether node i of the padded box lies in a plane of kind `axis`: 0 for cell
// planes (time slices t < n0), d >= 1 for the G^s_d planes of q_d / alpha_d
// (x_d < n_d).
bool in_plane(const Geo& g, int axis, int64_t i) {
  if (axis == 0) return i / g.stride[0] < g.n[0];
  return (i / g.stride[axis]) % g.N[axis] < g.n[axis];
}

// The sigma changes held in a control block, oldest first (at most cap).
int sigma_history(const Ctl& c, double* sigma, int32_t* at_iter, int32_t cap, int32_t* count) {
  if (cap < 0) return fail(DOT_EINVAL, "cap must be >= 0");
  const int n = c.sigma_changes;
  const int kept = std::min(n, kSigmaHist), first = n - kept;
  const int out = std::min(kept, (int)cap);
  for (int j = 0; j < out; ++j) {
    const int slot = (first + kept - out + j) % kSigmaHist;  // the newest `out` changes
    if (sigma) sigma[j] = c.hist_sigma[slot];
    if (at_iter) at_iter[j] = c.hist_iter[slot];
  }
  if (count) *count = n;
  return DOT_OK;
}

}  // namespace

extern "C" {

int dot_state_export(const dot_plan* P, const void* state, double* q, double* alpha, double* beta, double* sigma,
                     void* stream) {
  if (!P || !state) return fail(DOT_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const char* s = static_cast<const char*>(state);
  HIP_OK(hipMemcpyAsync(P->host_ctl, s + P->ctl_offset, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  const Ctl c = *P->host_ctl;
  const int64_t nb = P->g.nb;
  // after k iterations the newest q is the buffer k & 1 (q, then q_new)
  auto fetch = [&](size_t off, int planes, double* out) -> int {
    if (!out) return DOT_OK;
    const size_t n = (size_t)planes * nb;
    if (P->precision == DOT_FP64) {
      HIP_OK(hipMemcpyAsync(out, s + off, n * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
    } else {
      std::vector<float> tmp(n);
      HIP_OK(hipMemcpyAsync(tmp.data(), s + off, n * sizeof(float), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      for (size_t i = 0; i < n; ++i) out[i] = (double)tmp[i];
    }
    return DOT_OK;
  };
  int rc = fetch((c.iter & 1) ? P->off_qn : P->off_q, P->D + 1, q);
  if (rc || (rc = fetch(P->off_beta, P->K, beta))) return rc;
  if (alpha) {
    HIP_OK(hipMemcpyAsync(alpha, s + P->off_alpha, (size_t)(P->D + 1) * nb * sizeof(double), hipMemcpyDeviceToHost,
                          st));
    HIP_OK(hipStreamSynchronize(st));
  }
  if (sigma) *sigma = c.sigma;
  return DOT_OK;
}

int dot_sigma_history(const dot_plan* P, const void* state, double* sigma, int32_t* at_iter, int32_t cap,
                      int32_t* count, void* stream) {
  if (!P || !state) return fail(DOT_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(P->host_ctl, static_cast<const char*>(state) + P->ctl_offset, sizeof(Ctl),
                        hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return sigma_history(*P->host_ctl, sigma, at_iter, cap, count);
}

int dot_batch_sigma_history(const dot_batch* B, const void* ws, int32_t index, double* sigma, int32_t* at_iter,
                            int32_t cap, int32_t* count, void* stream) {
  if (!B || !ws || index < 0 || index >= (int)B->plans.size()) return fail(DOT_EINVAL, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  Ctl c;
  HIP_OK(hipMemcpyAsync(&c, static_cast<const char*>(ws) + (size_t)index * B->ctl_stride, sizeof(Ctl),
                        hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return sigma_history(c, sigma, at_iter, cap, count);
}

int dot_state_import(dot_plan* P, void* state, const double* q, const double* alpha, const double* beta, double sigma,
                     void* stream) {
  if (!P || !state || !q || !alpha || !beta) return fail(DOT_EINVAL, "null argument");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(DOT_EINVAL, "sigma must be positive and finite");
  const Geo& g = P->g;
  const int64_t nb = g.nb;
  const int D = P->D;
  for (const auto& arr : {std::make_pair(q, D + 1), std::make_pair(alpha, D + 1), std::make_pair(beta, P->K)})
    for (int64_t i = 0; i < (int64_t)arr.second * nb; ++i)
      if (!std::isfinite(arr.first[i])) return fail(DOT_EINVAL, "non-finite value in the iterate");
  hipStream_t st = (hipStream_t)stream;
  int rc = dot_state_reset(P, state, stream);
  if (rc) return rc;
  char* s = static_cast<char*>(state);
  // planes in the storage type, positions outside each plane's set zeroed
  auto put = [&](size_t off, int planes, const double* src, bool is_q_or_alpha, bool fp64) -> int {
    const size_t n = (size_t)planes * nb;
    std::vector<double> v(n);
    for (int p = 0; p < planes; ++p) {
      const int kind = is_q_or_alpha ? p : 0;
      for (int64_t i = 0; i < nb; ++i) v[(size_t)p * nb + i] = in_plane(g, kind, i) ? src[(size_t)p * nb + i] : 0.0;
    }
    if (fp64) {
      HIP_OK(hipMemcpyAsync(s + off, v.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
      HIP_OK(hipStreamSynchronize(st));
    } else {
      std::vector<float> f(n);
      for (size_t i = 0; i < n; ++i) f[i] = (float)v[i];
      HIP_OK(hipMemcpyAsync(s + off, f.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
      HIP_OK(hipStreamSynchronize(st));
    }
    return DOT_OK;
  };
  const bool fp64 = P->precision == DOT_FP64;
  if ((rc = put(P->off_q, D + 1, q, true, fp64)) || (rc = put(P->off_alpha, D + 1, alpha, true, true)) ||
      (rc = put(P->off_beta, P->K, beta, false, fp64)))
    return rc;
  Ctl c = initial_ctl(P);
  c.sigma = sigma;
  *P->host_ctl = c;
  HIP_OK(hipMemcpyAsync(s + P->ctl_offset, P->host_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  return DOT_OK;
}

}  // extern "C"

namespace {

// Promotion of the mixed iterate in `mixed_state` (layout of M) whose control
// block is at `mctl` (the state's own, or a batch member's) into fp64_state.
// Control block of an FP64 continuation of a mixed-precision iterate: the
// FP64 plan's parameters, the iterate's sigma, residuals, counters and sigma
// schedule.
Ctl promoted_ctl(const dot_plan* F, const Ctl& m) {
  Ctl f = initial_ctl(F);
  f.sigma = m.sigma;
  for (int k = 0; k < 8; ++k) f.eta[k] = m.eta[k];
  f.objective = m.objective;
  f.dual_objective = m.dual_objective;
  f.iter = m.iter;
  f.checks = m.checks;
  f.sigma_changes = m.sigma_changes;
  f.next_update = m.next_update;
  f.gap = m.gap;
  for (int k = 0; k < kSigmaHist; ++k) {
    f.hist_sigma[k] = m.hist_sigma[k];
    f.hist_iter[k] = m.hist_iter[k];
  }
  return f;
}

int promote_impl(const dot_plan* M, const void* mixed_state, const Ctl* mctl, dot_plan* F, void* fp64_state,
                 hipStream_t st) {
  if (M->precision != DOT_MIXED || F->precision != DOT_FP64)
    return fail(DOT_EINVAL, "promotion goes from a mixed-precision plan to an FP64 plan");
  bool same = M->D == F->D && M->cadence == F->cadence;
  for (int a = 0; a <= M->D; ++a) same = same && M->n[a] == F->n[a];
  if (!same) return fail(DOT_EINVAL, "the two plans differ in grid or check cadence");
  const int D = M->D;
  const int64_t nb = M->g.nb;
  const char* ms = static_cast<const char*>(mixed_state);
  char* fs = static_cast<char*>(fp64_state);
  // phi and alpha are FP64 in both layouts
  HIP_OK(hipMemcpyAsync(fs + F->off_phi, ms + M->off_phi, (size_t)nb * 8, hipMemcpyDeviceToDevice, st));
  HIP_OK(hipMemcpyAsync(fs + F->off_alpha, ms + M->off_alpha, (size_t)(D + 1) * nb * 8, hipMemcpyDeviceToDevice, st));
  // q and q_new (adjacent in both layouts), then beta: widened
  auto widen = [&](size_t src_off, size_t dst_off, int64_t n) -> int {
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(kb_widen, dim3(std::max(1u, grid)), dim3(256), 0, st,
                       reinterpret_cast<const float*>(ms + src_off), reinterpret_cast<double*>(fs + dst_off), n);
    HIP_OK(hipGetLastError());
    return DOT_OK;
  };
  int rc = widen(M->off_q, F->off_q, (int64_t)(2 * (D + 1)) * nb);
  if (rc || (rc = widen(M->off_beta, F->off_beta, (int64_t)M->K * nb))) return rc;
  // the W planes only carry values inside an iteration
  HIP_OK(hipMemsetAsync(fs + F->off_w, 0, F->ctl_offset - F->off_w, st));
  // control block: the FP64 plan's parameters, the iterate's sigma, counters
  // and sigma schedule
  HIP_OK(hipMemcpyAsync(M->host_ctl, mctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  *F->host_ctl = promoted_ctl(F, *M->host_ctl);
  HIP_OK(hipMemcpyAsync(fs + F->ctl_offset, F->host_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  return DOT_OK;
}

}  // namespace

extern "C" {

int dot_state_promote(const dot_plan* M, const void* mixed_state, dot_plan* F, void* fp64_state, void* stream) {
  if (!M || !mixed_state || !F || !fp64_state) return fail(DOT_EINVAL, "null argument");
  return promote_impl(M, mixed_state, at<const Ctl>(const_cast<void*>(mixed_state), M->ctl_offset), F, fp64_state,
                      (hipStream_t)stream);
}

int dot_batch_promote(const dot_batch* B, const void* ws, int32_t index, dot_plan* F, void* fp64_state,
                      void* stream) {
  if (!B || !ws || !F || !fp64_state) return fail(DOT_EINVAL, "null argument");
  if (index < 0 || index >= (int)B->plans.size()) return fail(DOT_EINVAL, "instance index out of range");
  const char* base = static_cast<const char*>(ws);
  return promote_impl(B->plans[index], base + B->state_off[index],
                      reinterpret_cast<const Ctl*>(base + (size_t)index * B->ctl_stride), F, fp64_state,
                      (hipStream_t)stream);
}

int dot_batch_promote_member(const dot_batch* Bm, const void* ws_m, int32_t index, dot_batch* Bf, void* ws_f,
                             int32_t slot, void* stream) {
  if (!Bm || !ws_m || !Bf || !ws_f) return fail(DOT_EINVAL, "null argument");
  if (index < 0 || index >= (int)Bm->plans.size()) return fail(DOT_EINVAL, "instance index out of range");
  if (slot < 0 || slot >= (int)Bf->plans.size()) return fail(DOT_EINVAL, "slot index out of range");
  if (Bf->it != 0 && Bf->it != Bm->it)
    return fail(DOT_EINVAL, "the FP64 batch is at iteration " + std::to_string(Bf->it) + ", the mixed one at " +
                                std::to_string(Bm->it) + ": its members iterate in lockstep");
  hipStream_t st = (hipStream_t)stream;
  const char* bm = static_cast<const char*>(ws_m);
  char* bf = static_cast<char*>(ws_f);
  dot_plan* F = Bf->plans[slot];
  int rc = promote_impl(Bm->plans[index], bm + Bm->state_off[index],
                        reinterpret_cast<const Ctl*>(bm + (size_t)index * Bm->ctl_stride), F, bf + Bf->state_off[slot],
                        st);
  if (rc) return rc;
  // a batch keeps its members' control blocks at the head of its workspace
  Ctl* hc = reinterpret_cast<Ctl*>(reinterpret_cast<char*>(Bf->host_ctl) + (size_t)slot * Bf->ctl_stride);
  *hc = *F->host_ctl;
  HIP_OK(hipMemcpyAsync(bf + (size_t)slot * Bf->ctl_stride, hc, sizeof(Ctl), hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  Bf->it = Bm->it;
  return DOT_OK;
}

int dot_prolong(const dot_plan* C, const void* coarse_state, dot_plan* F, void* fine_state, void* stream) {
  if (!C || !F || !coarse_state || !fine_state) return fail(DOT_EINVAL, "null argument");
  if (C->D != F->D || C->precision != F->precision) return fail(DOT_EINVAL, "plans differ in D or precision");
  for (int d = 0; d <= C->D; ++d)
    if (F->n[d] != 2 * C->n[d]) return fail(DOT_EINVAL, "the fine grid must have twice the segments per axis");
  hipStream_t st = (hipStream_t)stream;
  // sigma of the coarse iterate carries over; counters and schedule restart
  Ctl cc{};
  HIP_OK(hipMemcpyAsync(&cc, static_cast<const char*>(coarse_state) + C->ctl_offset, sizeof(Ctl),
                        hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  int rc = prolong_planes(C, coarse_state, F, fine_state, st);
  if (rc) return rc;
  Ctl h = initial_ctl(F);
  h.sigma = cc.sigma;
  *F->host_ctl = h;
  HIP_OK(hipMemcpyAsync(static_cast<char*>(fine_state) + F->ctl_offset, F->host_ctl, sizeof(Ctl),
                        hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  return DOT_OK;
}

int dot_solve_multilevel(const dot_problem* p, int32_t levels, double* rho_out, double* m_out, dot_result* res,
                         dot_result* level_results) {
  if (!p || levels < 0 || levels > 8) return fail(DOT_EINVAL, "bad multilevel arguments");
  int rc = validate(p);
  if (rc) return rc;
  const int D = p->D;
  // data of every level, finest first
  struct Level {
    int32_t n[4];
    std::vector<double> r0, r1;
    std::vector<uint8_t> mask;
  };
  std::vector<Level> L(levels + 1);
  size_t nx = 1;
  for (int d = 1; d <= D; ++d) nx *= (size_t)p->n[d] + 1;
  for (int d = 0; d < 4; ++d) L[0].n[d] = p->n[d];
  L[0].r0.assign(p->rho0, p->rho0 + nx);
  L[0].r1.assign(p->rho1, p->rho1 + nx);
  if (p->mask) L[0].mask.assign(p->mask, p->mask + nx);
  for (int v = 1; v <= levels; ++v) {
    Level& a = L[v - 1];
    Level& b = L[v];
    size_t ncx = 1;
    for (int d = 0; d < 4; ++d) b.n[d] = d <= D ? a.n[d] / 2 : 0;
    for (int d = 1; d <= D; ++d) ncx *= (size_t)b.n[d] + 1;
    b.r0.resize(ncx);
    b.r1.resize(ncx);
    if (!a.mask.empty()) b.mask.resize(ncx);
    rc = dot_coarsen_data(D, a.n, a.r0.data(), a.r1.data(), a.mask.empty() ? nullptr : a.mask.data(), b.r0.data(),
                          b.r1.data(), b.mask.empty() ? nullptr : b.mask.data());
    if (rc) return rc;
  }
  std::vector<dot_plan*> plans(levels + 1, nullptr);
  std::vector<void*> states(levels + 1, nullptr);
  auto cleanup = [&]() {
    DevLock lk(g_dev_mu);
    for (auto* s : states) (void)hipFree(s);
    for (auto* P : plans) dot_plan_destroy(P);
  };
  for (int v = levels; v >= 0; --v) {
    dot_problem q = *p;
    for (int d = 0; d < 4; ++d) q.n[d] = L[v].n[d];
    q.rho0 = L[v].r0.data();
    q.rho1 = L[v].r1.data();
    q.mask = L[v].mask.empty() ? nullptr : L[v].mask.data();
    // coarse level v: max{tol 10^-v, 1e-6}; the target level: tol
    if (v > 0) q.tol = std::max(p->tol * std::pow(10.0, -v), 1e-6);
    rc = dot_plan_create(&q, &plans[v]);
    if (!rc) {
      DevLock lk(g_dev_mu);
      if (hipMalloc(&states[v], plans[v]->state_bytes) != hipSuccess) rc = fail(DOT_ENOMEM, "state allocation failed");
    }
    if (!rc) rc = v == levels ? dot_state_reset(plans[v], states[v], nullptr)
                              : dot_prolong(plans[v + 1], states[v + 1], plans[v], states[v], nullptr);
    dot_result r{};
    if (!rc) rc = dot_run(plans[v], states[v], p->max_iter, nullptr, &r);
    if (rc) {
      cleanup();
      return rc;
    }
    if (level_results) level_results[levels - v] = r;
    if (v == 0 && res) *res = r;
  }
  rc = dot_extract(plans[0], states[0], rho_out, m_out, nullptr);
  cleanup();
  return rc;
}

// ---- serving: continuous batching with admission by HBM footprint ---------

}  // extern "C"

namespace {

// First-fit allocator over one device arena (host-side bookkeeping; blocks
// are 256-byte aligned; freed neighbours coalesce).
struct Arena {
  size_t size = 0;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, length), sorted by offset
  void init(size_t n) {
    size = n;
    free_list.assign(1, {0, n});
  }
  bool alloc(size_t n, size_t* off) {
    n = align256(n);
    for (size_t k = 0; k < free_list.size(); ++k) {
      if (free_list[k].second >= n) {
        *off = free_list[k].first;
        free_list[k].first += n;
        free_list[k].second -= n;
        if (free_list[k].second == 0) free_list.erase(free_list.begin() + k);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align256(n);
    auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, (size_t)0));
    it = free_list.insert(it, {off, n});
    size_t k = it - free_list.begin();
    if (k + 1 < free_list.size() && free_list[k].first + free_list[k].second == free_list[k + 1].first) {
      free_list[k].second += free_list[k + 1].second;
      free_list.erase(free_list.begin() + k + 1);
    }
    if (k > 0 && free_list[k - 1].first + free_list[k - 1].second == free_list[k].first) {
      free_list[k - 1].second += free_list[k].second;
      free_list.erase(free_list.begin() + k);
    }
  }
  size_t free_bytes() const {
    size_t t = 0;
    for (auto& f : free_list) t += f.second;
    return t;
  }
};

enum { kQueued = 0, kRunning = 1, kDone = 2 };

// A request: one plan per level (coarsest first; one level for a plain
// solve), all level states in one arena block.
struct Request {
  uint64_t ticket = 0;
  std::vector<dot_plan*> plans;
  std::vector<size_t> lvl_off;  // state offset of each level inside the block
  size_t bytes = 0;             // block size
  int level = 0;                // level being iterated
  dot_plan* plan = nullptr;     // plans[level]
  int status = kQueued;
  int slot = -1;
  size_t block = 0;             // arena offset of the block
  size_t off = 0;               // arena offset of the current level's state
  std::vector<double> rho, m;
  dot_result res{};
  std::chrono::steady_clock::time_point admitted;  // start of the time budget
  // imported checkpoint (dot_ctx_import): installed at admission instead of
  // the initial point; empty for a plain submission
  int ck_level = 0;
  std::vector<unsigned char> ck_planes;  // the level's state up to its control block
  Ctl ck_ctl{};
  // checkpoint of the final state of a request that stopped at its iteration
  // cap in a context that keeps them (dot_ctx_keep_capped); freed by fetch
  std::vector<unsigned char> final_ck;
  ~Request() {
    for (auto* P : plans) dot_plan_destroy(P);
  }
};

}  // namespace

struct dot_ctx {
  int D = 0, precision = 0, max_slots = 0;
  size_t budget = 0;
  void* arena_mem = nullptr;
  Arena arena;
  Ctl* d_ctl = nullptr;     // max_slots control blocks
  Ctl* h_ctl = nullptr;     // pinned mirror
  size_t ctl_stride = 0;
  std::vector<Request*> slots;          // active request per slot (nullptr: free)
  std::vector<Request*> queue;          // FIFO of queued requests
  std::vector<std::unique_ptr<Request>> all;
  uint64_t next_ticket = 1;
  int it = 0;                           // iterations done by the executor (multiple of 10)
  bool dirty = true;                    // active set changed: rebuild descriptors and maps
  bool warm = false;                    // plain launches have run once (graph capture allowed)
  void* d_inst = nullptr;
  size_t d_inst_cap = 0;
  uint16_t* d_maps = nullptr;
  size_t d_maps_cap = 0;
  Exec E;
  GraphCache* graphs = nullptr;
  Prof prof;
  int device = 0;
  int64_t admitted = 0, retired = 0;
  bool keep_capped = false;             // keep checkpoints of requests retired at their iteration cap
  mutable std::mutex mu;                // every dot_ctx_* call holds it
  mutable std::string err;              // message of the last failed call on this context
  ~dot_ctx() { delete graphs; }
};

namespace {

Request* find_req(dot_ctx* C, uint64_t ticket) {
  for (auto& r : C->all)
    if (r && r->ticket == ticket) return r.get();
  return nullptr;
}

template <typename T>
int ctx_rebuild(dot_ctx* C, hipStream_t st) {
  DevLock lk(g_dev_mu);
  std::vector<Inst<T>> host;
  std::vector<uint16_t> maps;
  std::vector<dot_plan*> act;
  for (int sl = 0; sl < C->max_slots; ++sl)
    if (C->slots[sl]) act.push_back(C->slots[sl]->plan);
  Exec& E = C->E;
  E = Exec();
  E.D = C->D;
  E.precision = C->precision;
  E.ninst = 0;
  E.cadence = 5;
  E.device = C->device;
  E.prof = &C->prof;
  delete C->graphs;
  C->graphs = new GraphCache();
  C->graphs->warm = C->warm;  // kernel attributes already set by earlier plain launches
  E.graphs = C->graphs;
  if (act.empty()) {
    C->dirty = false;
    return DOT_OK;
  }
  // transform tile width per axis, from the lines of all active instances
  for (int a = 0; a <= C->D; ++a) {
    int64_t all_lines = 0;
    bool wide_ok = true, mid_ok = true, all_tri = true;
    for (dot_plan* P : act) {
      all_lines += P->lines[a];
      wide_ok = wide_ok && P->wide_ok[a];
      mid_ok = mid_ok && P->mid_ok[a];
      all_tri = all_tri && P->tri;
    }
    E.cw_axis[a] = (a == C->D && all_tri) ? tri_default_cw(act.data(), (int)act.size())
                                           : choose_cw(all_lines, wide_ok, mid_ok);
  }
  // descriptors of the active instances, in slot order
  uint32_t blk = 0;
  uint32_t tile[kMaxAxes] = {0, 0, 0, 0};
  int idx = 0;
  for (int sl = 0; sl < C->max_slots; ++sl) {
    Request* r = C->slots[sl];
    if (!r) continue;
    dot_plan* P = r->plan;
    Ctl* ctl = reinterpret_cast<Ctl*>(reinterpret_cast<char*>(C->d_ctl) + (size_t)sl * C->ctl_stride);
    Inst<T> s = state_inst<T>(P, static_cast<char*>(C->arena_mem) + r->off, ctl);
    s.blk0 = blk;
    blk += (uint32_t)P->nblocks;
    for (int a = 0; a <= C->D; ++a) {
      s.tile0[a] = tile[a];
      tile[a] += (uint32_t)tiles_for(P->lines[a], E.cw_axis[a]);
    }
    host.push_back(s);
    maps.insert(maps.end(), (size_t)P->nblocks, (uint16_t)idx);
    ++idx;
  }
  E.ninst = idx;
  E.nact = idx;
  E.grid_nodes = blk;
  for (dot_plan* P : act) {
    E.ntri += P->tri ? 1 : 0;
    E.ntri_long += P->tri && P->g.N[P->D] > kTriPartMaxNodes ? 1 : 0;
    E.nstaged += P->nblocks >= kFinStageMinRows ? 1 : 0;
    E.nodes += P->g.nb;
  }
  size_t map_off[kMaxAxes] = {0, 0, 0, 0};
  for (int a = 0; a <= C->D; ++a) {
    map_off[a] = maps.size();
    size_t smem = 0;
    int waves = 1, k = 0;
    const int cw = E.cw_axis[a];
    int64_t all_tiles = 0;
    for (dot_plan* P : act) all_tiles += tiles_for(P->lines[a], cw);
    for (int sl = 0; sl < C->max_slots; ++sl) {
      Request* r = C->slots[sl];
      if (!r) continue;
      dot_plan* P = r->plan;
      maps.insert(maps.end(), (size_t)tiles_for(P->lines[a], cw), (uint16_t)k);
      ++k;
      if (a == C->D && P->tri) continue;  // takes the tridiagonal solve on this axis
      smem = std::max(smem, pass_smem(P->g.N[a], P->scalar_bytes, cw));
      waves = std::max(waves, pass_waves<T>(P->g.N[a], all_tiles, cw));
    }
    E.grid_axis[a] = (unsigned)(maps.size() - map_off[a]);
    E.smem_axis[a] = smem;
    E.waves_axis[a] = waves;
  }
  if (host.size() * sizeof(Inst<T>) > C->d_inst_cap) {
    (void)hipFree(C->d_inst);
    C->d_inst_cap = host.size() * sizeof(Inst<T>) * 2;
    HIP_OK(hipMalloc(&C->d_inst, C->d_inst_cap));
  }
  if (maps.size() * sizeof(uint16_t) > C->d_maps_cap) {
    (void)hipFree(C->d_maps);
    C->d_maps_cap = maps.size() * sizeof(uint16_t) * 2;
    HIP_OK(hipMalloc((void**)&C->d_maps, C->d_maps_cap));
  }
  HIP_OK(hipMemcpyAsync(C->d_inst, host.data(), host.size() * sizeof(Inst<T>), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(C->d_maps, maps.data(), maps.size() * sizeof(uint16_t), hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  E.d_inst = C->d_inst;
  E.map_nodes = C->d_maps;
  for (int a = 0; a <= C->D; ++a) E.map_axis[a] = C->d_maps + map_off[a];
  C->dirty = false;
  return DOT_OK;
}

// Iterations of the active set; the executor's counter advances by the
// iterations run (a multiple of 10 unless every instance stopped early).
template <typename T, int D>
struct CtxStepF {
  static int run(dot_ctx* C, int iters, hipStream_t st) {
    int rc;
    if (C->dirty && (rc = ctx_rebuild<T>(C, st))) return rc;
    if (C->E.ninst == 0) return DOT_OK;
    int done = 0;
    // the control blocks of every slot are polled; free slots hold stop = 1
    rc = run_iters<T, D>(C->E, C->it, iters, C->d_ctl, C->ctl_stride, C->h_ctl, st, &done, C->max_slots);
    if (rc) return rc;
    C->it += done;
    C->warm = C->warm || C->E.graphs->warm;
    return DOT_OK;
  }
};

// Admit queued requests in arrival order while a slot and arena space exist.
int ctx_admit(dot_ctx* C, hipStream_t st) {
  while (!C->queue.empty()) {
    Request* r = C->queue.front();
    int sl = -1;
    for (int k = 0; k < C->max_slots; ++k)
      if (!C->slots[k]) {
        sl = k;
        break;
      }
    size_t off = 0;
    if (sl < 0 || !C->arena.alloc(r->bytes, &off)) break;  // head-of-line waits for space
    C->queue.erase(C->queue.begin());
    r->slot = sl;
    r->block = off;
    r->level = r->ck_planes.empty() ? 0 : r->ck_level;
    r->plan = r->plans[r->level];
    r->off = off + r->lvl_off[r->level];
    off = r->off;
    r->status = kRunning;
    r->admitted = std::chrono::steady_clock::now();
    C->slots[sl] = r;
    dot_plan* P = r->plan;
    char* slot_ctl = reinterpret_cast<char*>(C->d_ctl) + (size_t)sl * C->ctl_stride;
    if (r->ck_planes.empty()) {
      HIP_OK(hipMemsetAsync(static_cast<char*>(C->arena_mem) + off, 0, P->ctl_offset, st));
      Ctl h = initial_ctl(P);
      h.iter_limit = P->max_iter;
      HIP_OK(hipMemcpyAsync(slot_ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, st));
    } else {
      // the checkpointed iterate continues exactly where it was exported
      HIP_OK(hipMemcpyAsync(static_cast<char*>(C->arena_mem) + off, r->ck_planes.data(), r->ck_planes.size(),
                            hipMemcpyHostToDevice, st));
      HIP_OK(hipMemcpyAsync(slot_ctl, &r->ck_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));
    }
    HIP_OK(hipStreamSynchronize(st));
    if (!r->ck_planes.empty()) std::vector<unsigned char>().swap(r->ck_planes);
    C->dirty = true;
    C->admitted += 1;
  }
  return DOT_OK;
}

int write_checkpoint(dot_ctx* C, Request* r, unsigned char* out, hipStream_t st);
size_t checkpoint_bytes(const Request* r);

// Retire instances that stopped or reached their iteration cap: results to
// host, arena block and slot freed.
int ctx_retire(dot_ctx* C, hipStream_t st) {
  HIP_OK(hipMemcpyAsync(C->h_ctl, C->d_ctl, C->ctl_stride * C->max_slots, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (int sl = 0; sl < C->max_slots; ++sl) {
    Request* r = C->slots[sl];
    if (!r) continue;
    Ctl c = *reinterpret_cast<Ctl*>(reinterpret_cast<char*>(C->h_ctl) + (size_t)sl * C->ctl_stride);
    // a request's time budget runs from its admission and applies on its
    // target level (a multilevel request always finishes its coarse levels)
    const bool last = r->level + 1 == (int)r->plans.size();
    const double limit = r->plans.back()->time_limit;
    const bool out_of_time =
        last && limit > 0.0 &&
        std::chrono::duration<double>(std::chrono::steady_clock::now() - r->admitted).count() >= limit;
    if (!c.stop && c.iter < r->plan->max_iter && !out_of_time) continue;
    if (!last) {
      // multilevel: the next finer level starts from the interpolated
      // iterate, whatever the coarse level's stop reason (as solved alone)
      dot_plan* Pc = r->plans[r->level];
      dot_plan* Pf = r->plans[r->level + 1];
      char* cs = static_cast<char*>(C->arena_mem) + r->off;
      char* fs = static_cast<char*>(C->arena_mem) + r->block + r->lvl_off[r->level + 1];
      int rc = prolong_planes(Pc, cs, Pf, fs, st);
      if (rc) return rc;
      Ctl h = initial_ctl(Pf);
      h.sigma = c.sigma;
      h.iter_limit = Pf->max_iter;
      HIP_OK(hipMemcpyAsync(reinterpret_cast<char*>(C->d_ctl) + (size_t)sl * C->ctl_stride, &h, sizeof(Ctl),
                            hipMemcpyHostToDevice, st));
      HIP_OK(hipStreamSynchronize(st));
      r->level += 1;
      r->plan = Pf;
      r->off = r->block + r->lvl_off[r->level];
      C->dirty = true;
      continue;
    }
    dot_plan* P = r->plan;
    const void* state = static_cast<char*>(C->arena_mem) + r->off;
    r->rho.assign((size_t)P->g.n[0] * P->g.nx, 0.0);
    size_t nm = 0;
    for (int d = 1; d <= P->D; ++d) nm += (size_t)(P->g.nb / P->g.N[d]) * P->g.n[d];
    r->m.assign(nm, 0.0);
    int rc = extract_impl(P, state, r->rho.data(), r->m.data(), st);
    if (rc) return rc;
    fill_result(c, &r->res);
    if (!c.stop && c.iter < r->plan->max_iter) r->res.term = DOT_TIMEOUT;
    if (C->keep_capped && c.stop == 2) {
      r->final_ck.resize(checkpoint_bytes(r));
      if ((rc = write_checkpoint(C, r, r->final_ck.data(), st))) return rc;
    }
    r->status = kDone;
    C->arena.release(r->block, r->bytes);
    C->slots[sl] = nullptr;
    // a free slot keeps stop = 1 so that polling ignores it
    Ctl dead{};
    dead.stop = 1;
    HIP_OK(hipMemcpyAsync(reinterpret_cast<char*>(C->d_ctl) + (size_t)sl * C->ctl_stride, &dead, sizeof(Ctl),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    C->dirty = true;
    C->retired += 1;
  }
  return DOT_OK;
}

}  // namespace

extern "C" {

size_t dot_footprint_bytes(const dot_problem* p) {
  if (!p || p->D < 1 || p->D > 3) return 0;
  const int D = p->D;
  const size_t w = p->precision == DOT_FP64 ? 8 : 4;
  size_t nb = 1;
  for (int d = 0; d <= D; ++d) nb *= (size_t)p->n[d] + 1;
  const size_t pb = nb * w;
  size_t s = align256(nb * 8);                               // phi
  if (p->precision == DOT_MIXED) s += align256(pb);          // transform scratch
  s = align256(s + (size_t)(2 * (D + 1)) * pb);              // q, q_new
  s += (size_t)(D + 1) * nb * 8;                             // alpha (FP64)
  s += (size_t)(4 * D + 2 + 4 * D) * pb;                     // beta, W
  s = align256(s) + nb * 8;                                  // w_{K-1} - w_0 (FP64)
  s = align256(s) + align256(sizeof(Ctl));
  // partial rows (one per workgroup at one slice each), then the reduction's stage rows
  const size_t rows = (nb / ((size_t)p->n[0] + 1) + kBlock - 1) / kBlock * ((size_t)p->n[0] + 1) + kFinChunks;
  s += align256(rows * kNumSums * sizeof(double));
  return s;
}

void dot_ctx_destroy(dot_ctx* C) {
  DevLock lk(g_dev_mu);
  if (!C) return;
  int prev = -1;
  const bool other = hipGetDevice(&prev) == hipSuccess && prev != C->device && hipSetDevice(C->device) == hipSuccess;
  C->all.clear();  // requests destroy their plans
  (void)hipFree(C->arena_mem);
  (void)hipFree(C->d_ctl);
  (void)hipHostFree(C->h_ctl);
  (void)hipFree(C->d_inst);
  (void)hipFree(C->d_maps);
  delete C;
  if (other) (void)hipSetDevice(prev);
}

}  // extern "C"

namespace {

int ctx_create_impl(int32_t device, int32_t D, int32_t precision, size_t hbm_budget_bytes, int32_t max_slots,
                    dot_ctx** out) {
  if (!out || D < 1 || D > 3 || (precision != DOT_FP64 && precision != DOT_MIXED) || max_slots < 1 ||
      max_slots > 4096 || hbm_budget_bytes < 4096)
    return fail(DOT_EINVAL, "bad serving context arguments");
  *out = nullptr;
  std::unique_ptr<dot_ctx, void (*)(dot_ctx*)> C(new (std::nothrow) dot_ctx(), dot_ctx_destroy);
  if (!C) return fail(DOT_ENOMEM, "host allocation failed");
  C->D = D;
  C->precision = precision;
  C->max_slots = max_slots;
  C->budget = hbm_budget_bytes;
  C->device = device;
  if (hipMalloc(&C->arena_mem, hbm_budget_bytes) != hipSuccess)
    return fail(DOT_ENOMEM, "cannot reserve the HBM budget");
  C->arena.init(hbm_budget_bytes);
  C->ctl_stride = align256(sizeof(Ctl));
  HIP_OK(hipMalloc((void**)&C->d_ctl, C->ctl_stride * max_slots));
  HIP_OK(hipHostMalloc((void**)&C->h_ctl, C->ctl_stride * max_slots, hipHostMallocDefault));
  for (int k = 0; k < max_slots; ++k) {
    Ctl* h = reinterpret_cast<Ctl*>(reinterpret_cast<char*>(C->h_ctl) + (size_t)k * C->ctl_stride);
    *h = Ctl{};
    h->stop = 1;
  }
  HIP_OK(hipMemcpy(C->d_ctl, C->h_ctl, C->ctl_stride * max_slots, hipMemcpyHostToDevice));
  C->slots.assign(max_slots, nullptr);
  *out = C.release();
  return DOT_OK;
}

int ctx_submit_impl(dot_ctx* C, const dot_problem* p, int32_t levels, uint64_t* ticket, Request** made = nullptr) {
  if (!C || !p || !ticket) return fail(DOT_EINVAL, "null argument");
  if (levels < 0 || levels > 8) return fail(DOT_EINVAL, "levels must be in 0..8");
  if (p->D != C->D || p->precision != C->precision) return fail(DOT_EINVAL, "problem D / precision differ from the context");
  if ((p->check_every > 0 ? p->check_every : 5) != 5) return fail(DOT_EINVAL, "serving needs the 5-iteration check cadence");
  if (p->max_iter % 5 != 0) return fail(DOT_EINVAL, "serving needs max_iter to be a multiple of 5");
  int rc = validate(p);
  if (rc) return rc;
  // problems of every level, coarsest first, as dot_solve_multilevel builds them
  const int D = p->D;
  std::vector<std::array<int32_t, 4>> n(levels + 1);
  std::vector<std::vector<double>> r0(levels + 1), r1(levels + 1);
  std::vector<std::vector<uint8_t>> mk(levels + 1);
  size_t nx = 1;
  for (int d = 1; d <= D; ++d) nx *= (size_t)p->n[d] + 1;
  for (int d = 0; d < 4; ++d) n[levels][d] = p->n[d];
  r0[levels].assign(p->rho0, p->rho0 + nx);
  r1[levels].assign(p->rho1, p->rho1 + nx);
  if (p->mask) mk[levels].assign(p->mask, p->mask + nx);
  for (int l = levels - 1; l >= 0; --l) {
    size_t ncx = 1;
    for (int d = 0; d < 4; ++d) n[l][d] = d <= D ? n[l + 1][d] / 2 : 0;
    for (int d = 1; d <= D; ++d) ncx *= (size_t)n[l][d] + 1;
    r0[l].resize(ncx);
    r1[l].resize(ncx);
    if (!mk[l + 1].empty()) mk[l].resize(ncx);
    rc = dot_coarsen_data(D, n[l + 1].data(), r0[l + 1].data(), r1[l + 1].data(),
                          mk[l + 1].empty() ? nullptr : mk[l + 1].data(), r0[l].data(), r1[l].data(),
                          mk[l].empty() ? nullptr : mk[l].data());
    if (rc) return rc;
  }
  auto r = std::make_unique<Request>();
  size_t total = 0;
  for (int l = 0; l <= levels; ++l) {
    dot_problem q = *p;
    for (int d = 0; d < 4; ++d) q.n[d] = n[l][d];
    q.rho0 = r0[l].data();
    q.rho1 = r1[l].data();
    q.mask = mk[l].empty() ? nullptr : mk[l].data();
    const int v = levels - l;  // coarse level v: max{tol 10^-v, 1e-6}
    if (v > 0) q.tol = std::max(p->tol * std::pow(10.0, -v), 1e-6);
    dot_plan* P = nullptr;
    rc = dot_plan_create(&q, &P);
    if (rc) return rc;
    r->plans.push_back(P);
    r->lvl_off.push_back(total);
    total += align256(P->state_bytes);
  }
  if (total > C->budget) return fail(DOT_EBUSY, "problem can never fit the HBM budget");
  r->bytes = total;
  r->plan = r->plans[0];
  r->ticket = C->next_ticket++;
  *ticket = r->ticket;
  if (made) *made = r.get();
  C->queue.push_back(r.get());
  C->all.push_back(std::move(r));
  return DOT_OK;
}

int ctx_step_impl(dot_ctx* C, int32_t iters, void* stream, int32_t* n_active, int32_t* n_queued) {
  if (!C || iters < 0 || iters % kGraphIters != 0) return fail(DOT_EINVAL, "iters must be a multiple of 10");
  hipStream_t st = (hipStream_t)stream;
  int rc = ctx_admit(C, st);
  if (rc) return rc;
  rc = dispatch<CtxStepF>(C->precision, C->D, C, (int)iters, st);
  if (rc) return rc;
  rc = ctx_retire(C, st);
  if (rc) return rc;
  int a = 0;
  for (auto* r : C->slots) a += r != nullptr;
  // admissions happen at multiples of 10 of the executor's counter, so each
  // instance's parity and check positions match those of a solve alone; with
  // nothing active the counter restarts
  if (a == 0) C->it = 0;
  if (n_active) *n_active = a;
  if (n_queued) *n_queued = (int32_t)C->queue.size();
  return DOT_OK;
}

int ctx_poll_impl(dot_ctx* C, uint64_t ticket, int32_t* status) {
  if (!C || !status) return fail(DOT_EINVAL, "null argument");
  Request* r = find_req(C, ticket);
  if (!r) return fail(DOT_EINVAL, "unknown ticket");
  *status = r->status;
  return DOT_OK;
}

int ctx_fetch_impl(dot_ctx* C, uint64_t ticket, double* rho_out, double* m_out, dot_result* res) {
  if (!C) return fail(DOT_EINVAL, "null argument");
  for (auto it = C->all.begin(); it != C->all.end(); ++it) {
    Request* r = it->get();
    if (!r || r->ticket != ticket) continue;
    if (r->status != kDone) return fail(DOT_EINVAL, "request not finished");
    if (rho_out) std::memcpy(rho_out, r->rho.data(), r->rho.size() * sizeof(double));
    if (m_out) std::memcpy(m_out, r->m.data(), r->m.size() * sizeof(double));
    if (res) *res = r->res;
    C->all.erase(it);
    return DOT_OK;
  }
  return fail(DOT_EINVAL, "unknown ticket");
}

int ctx_stats_impl(const dot_ctx* C, size_t* free_bytes, int64_t* admitted, int64_t* retired) {
  if (!C) return fail(DOT_EINVAL, "null context");
  if (free_bytes) *free_bytes = C->arena.free_bytes();
  if (admitted) *admitted = C->admitted;
  if (retired) *retired = C->retired;
  return DOT_OK;
}


// ---- checkpoint of a running request --------------------------------------
// Layout of a checkpoint (host bytes): CkHeader, the state of the request's
// current level up to its control block (every plane: phi, transform
// scratch, q, q_new, alpha, beta, W), then the control block.
constexpr uint64_t kCkMagic = 0x31544B4354534F44ull;  // "DOSTCKT1"
struct CkHeader {
  uint64_t magic;
  int32_t D, precision, levels, level;
  int32_t n[4];           // target grid of the request
  int32_t level_n[4];     // grid of the exported level
  uint64_t plane_bytes;   // state bytes before the control block
  uint64_t ctl_bytes;
};

// Checkpoint of request r's current level (running, between steps) into out
// (sizeof(CkHeader) + ctl_offset + sizeof(Ctl) bytes).
int write_checkpoint(dot_ctx* C, Request* r, unsigned char* out, hipStream_t st) {
  dot_plan* P = r->plan;
  CkHeader h{};
  h.magic = kCkMagic;
  h.D = C->D;
  h.precision = C->precision;
  h.levels = (int32_t)r->plans.size() - 1;
  h.level = r->level;
  for (int d = 0; d < 4; ++d) {
    h.n[d] = r->plans.back()->n[d];
    h.level_n[d] = P->n[d];
  }
  h.plane_bytes = P->ctl_offset;
  h.ctl_bytes = sizeof(Ctl);
  std::memcpy(out, &h, sizeof(h));
  HIP_OK(hipMemcpyAsync(out + sizeof(h), static_cast<char*>(C->arena_mem) + r->off, P->ctl_offset,
                        hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(out + sizeof(h) + P->ctl_offset,
                        reinterpret_cast<char*>(C->d_ctl) + (size_t)r->slot * C->ctl_stride, sizeof(Ctl),
                        hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return DOT_OK;
}

size_t checkpoint_bytes(const Request* r) { return sizeof(CkHeader) + r->plan->ctl_offset + sizeof(Ctl); }

int ctx_export_impl(dot_ctx* C, uint64_t ticket, void* buf, size_t cap, size_t* bytes, hipStream_t st) {
  Request* r = find_req(C, ticket);
  if (!r) return fail(DOT_EINVAL, "unknown ticket");
  const bool kept = r->status == kDone && !r->final_ck.empty();
  if (r->status != kRunning && !kept)
    return fail(DOT_EINVAL, "only a running request, or one kept at its iteration cap, can be exported");
  const size_t need = kept ? r->final_ck.size() : checkpoint_bytes(r);
  if (bytes) *bytes = need;
  if (!buf) return DOT_OK;
  if (cap < need) return fail(DOT_EINVAL, "checkpoint buffer too small");
  if (kept) {
    std::memcpy(buf, r->final_ck.data(), need);
    return DOT_OK;
  }
  return write_checkpoint(C, r, static_cast<unsigned char*>(buf), st);
}

int ctx_import_impl(dot_ctx* C, const dot_problem* p, int32_t levels, const void* buf, size_t bytes,
                    uint64_t* ticket) {
  if (!buf || bytes < sizeof(CkHeader)) return fail(DOT_EINVAL, "checkpoint too short");
  CkHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kCkMagic) return fail(DOT_EINVAL, "not a serving checkpoint");
  // a mixed-precision checkpoint may continue in an FP64 context (promoted)
  const bool promote = h.precision == DOT_MIXED && C->precision == DOT_FP64;
  if (h.D != C->D || (h.precision != C->precision && !promote))
    return fail(DOT_EINVAL, "checkpoint D / precision differ from the context");
  if (h.levels != levels || h.level < 0 || h.level > levels)
    return fail(DOT_EINVAL, "checkpoint levels differ from the request's");
  for (int d = 0; d <= p->D && d < 4; ++d)
    if (p->n[d] != h.n[d]) return fail(DOT_EINVAL, "checkpoint grid differs from the problem's");
  if (h.ctl_bytes != sizeof(Ctl) || bytes != sizeof(CkHeader) + h.plane_bytes + h.ctl_bytes)
    return fail(DOT_EINVAL, "checkpoint size does not match its header");
  Request* r = nullptr;
  uint64_t t = 0;
  int rc = ctx_submit_impl(C, p, levels, &t, &r);
  if (rc) return rc;
  dot_plan* P = r->plans[h.level];
  const StateLayout src = state_layout(h.D, P->g.nb, h.precision);
  bool same = src.ctl_offset == h.plane_bytes;
  for (int d = 0; d < 4; ++d) same = same && P->n[d] == h.level_n[d];
  const unsigned char* in = static_cast<const unsigned char*>(buf) + sizeof(CkHeader);
  Ctl ck;
  std::memcpy(&ck, in + h.plane_bytes, sizeof(Ctl));
  // the q planes of an imported state are read with the parity of an
  // admission, which holds for iteration counts that are multiples of 10
  const bool aligned = ck.iter % 10 == 0;
  if (!same || !aligned) {
    // undo the submission: the request was queued last
    C->queue.pop_back();
    C->all.pop_back();
    return fail(DOT_EINVAL, !same ? "checkpoint state layout differs from the problem's"
                                  : "checkpoint not at a multiple of 10 iterations");
  }
  r->ck_level = h.level;
  if (!promote) {
    r->ck_planes.assign(in, in + h.plane_bytes);
    r->ck_ctl = ck;
  } else {
    // the FP64 state of the iterate (as dot_state_promote): phi and alpha
    // copied, q, q_new and beta widened exactly, the z-step planes zero
    const int64_t nb = P->g.nb;
    const int D = h.D, K = 4 * D + 2;
    r->ck_planes.assign(P->ctl_offset, 0);
    unsigned char* out = r->ck_planes.data();
    std::memcpy(out + P->off_phi, in + src.off_phi, (size_t)nb * sizeof(double));
    std::memcpy(out + P->off_alpha, in + src.off_alpha, (size_t)(D + 1) * nb * sizeof(double));
    auto widen = [&](size_t from, size_t to, int64_t n) {
      const float* a = reinterpret_cast<const float*>(in + from);
      double* b = reinterpret_cast<double*>(out + to);
      for (int64_t i = 0; i < n; ++i) b[i] = (double)a[i];
    };
    widen(src.off_q, P->off_q, (int64_t)2 * (D + 1) * nb);
    widen(src.off_beta, P->off_beta, (int64_t)K * nb);
    r->ck_ctl = promoted_ctl(P, ck);
  }
  // the request continues to its own max_iter (a request stopped at an
  // earlier cap runs on)
  r->ck_ctl.iter_limit = P->max_iter;
  if (r->ck_ctl.stop == 2 && r->ck_ctl.iter < P->max_iter) r->ck_ctl.stop = 0;
  *ticket = t;
  return DOT_OK;
}

// Makes the context's device current for one call and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  int dev = -1;
  int rc = DOT_OK;
  explicit DeviceGuard(int device) : dev(device) {
    if (hipGetDevice(&prev) != hipSuccess) {
      rc = fail(DOT_EDEVICE, "hipGetDevice failed");
      prev = -1;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) rc = fail(DOT_EDEVICE, "cannot select the context's device");
  }
  ~DeviceGuard() {
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
  }
};

// Keeps the message of a failed call in the context.
int ctx_ret(const dot_ctx* C, int rc) {
  if (rc) C->err = g_err;
  return rc;
}

}  // namespace

extern "C" {

int dot_ctx_create(int32_t device, int32_t D, int32_t precision, size_t hbm_budget_bytes, int32_t max_slots,
                   dot_ctx** out) {
  if (!out) return fail(DOT_EINVAL, "null output pointer");
  *out = nullptr;
  // host-side checks first (no device call before the arguments are valid)
  if (D < 1 || D > 3 || (precision != DOT_FP64 && precision != DOT_MIXED) || max_slots < 1 || max_slots > 4096 ||
      hbm_budget_bytes < 4096)
    return fail(DOT_EINVAL, "bad serving context arguments");
  int count = 0;
  if (device < -1) return fail(DOT_EINVAL, "device must be >= -1");
  DevLock lk(g_dev_mu);
  if (device == -1) {
    HIP_OK(hipGetDevice(&device));
  } else {
    HIP_OK(hipGetDeviceCount(&count));
    if (device >= count) return fail(DOT_EINVAL, "no such device: " + std::to_string(device));
  }
  DeviceGuard g(device);
  if (g.rc) return g.rc;
  return ctx_create_impl(device, D, precision, hbm_budget_bytes, max_slots, out);
}

#define CTX_ENTER(C)                            \
  if (!(C)) return fail(DOT_EINVAL, "null context"); \
  std::lock_guard<std::mutex> lk_((C)->mu);     \
  DeviceGuard dg_((C)->device);                 \
  if (dg_.rc) return ctx_ret((C), dg_.rc)

int dot_ctx_submit_ml(dot_ctx* C, const dot_problem* p, int32_t levels, uint64_t* ticket) {
  CTX_ENTER(C);
  return ctx_ret(C, ctx_submit_impl(C, p, levels, ticket));
}

int dot_ctx_submit(dot_ctx* C, const dot_problem* p, uint64_t* ticket) {
  CTX_ENTER(C);
  return ctx_ret(C, ctx_submit_impl(C, p, 0, ticket));
}

int dot_ctx_step(dot_ctx* C, int32_t iters, void* stream, int32_t* n_active, int32_t* n_queued) {
  CTX_ENTER(C);
  return ctx_ret(C, ctx_step_impl(C, iters, stream, n_active, n_queued));
}

int dot_ctx_poll(dot_ctx* C, uint64_t ticket, int32_t* status) {
  CTX_ENTER(C);
  return ctx_ret(C, ctx_poll_impl(C, ticket, status));
}

int dot_ctx_fetch(dot_ctx* C, uint64_t ticket, double* rho_out, double* m_out, dot_result* res) {
  CTX_ENTER(C);
  return ctx_ret(C, ctx_fetch_impl(C, ticket, rho_out, m_out, res));
}

int dot_ctx_stats(const dot_ctx* C, size_t* free_bytes, int64_t* admitted, int64_t* retired) {
  CTX_ENTER(C);
  return ctx_ret(C, ctx_stats_impl(C, free_bytes, admitted, retired));
}

int dot_ctx_export(dot_ctx* C, uint64_t ticket, void* buf, size_t cap, size_t* bytes, void* stream) {
  CTX_ENTER(C);
  return ctx_ret(C, ctx_export_impl(C, ticket, buf, cap, bytes, (hipStream_t)stream));
}

int dot_ctx_import(dot_ctx* C, const dot_problem* p, int32_t levels, const void* buf, size_t bytes,
                   uint64_t* ticket) {
  CTX_ENTER(C);
  if (!p || !ticket) return ctx_ret(C, fail(DOT_EINVAL, "null argument"));
  return ctx_ret(C, ctx_import_impl(C, p, levels, buf, bytes, ticket));
}

int dot_ctx_keep_capped(dot_ctx* C, int32_t keep) {
  CTX_ENTER(C);
  C->keep_capped = keep != 0;
  return DOT_OK;
}

const char* dot_ctx_last_error(const dot_ctx* C) { return C ? C->err.c_str() : ""; }

}  // extern "C"
