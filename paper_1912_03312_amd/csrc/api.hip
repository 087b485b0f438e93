// C ABI of the REXI step (declared in include/rexi.h): handle, validation,
// the (sigma, beta) -> (s, w) mapping of eq. rational-evaluation, workspace
// planning and the host control loop of the batched restarted GMRES.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rexi.h"
#include "kernels.hip"

using rexi::FastDiv;
using rexi::InstDesc;
using rexi::SysDesc;
using rexi::SysState_t;
using rexi::Work;
using cplx = std::complex<double>;

namespace {

thread_local std::string g_setup_error;

enum ProfClass {
  PC_START = 0, PC_ARNOLDI_A, PC_REDUCE, PC_ARNOLDI_B, PC_REORTH_A, PC_REORTH_B,
  PC_UPDATE_X, PC_RESIDUAL, PC_POLESUM, PC_APPLY_H, PC_GRAD, PC_LANCZOS, PC_NCLASS
};
const char* kProfNames[PC_NCLASS] = {"start", "arnoldi_matvec_dots", "per_system_reduce", "arnoldi_update",
                                     "reorth_dots", "reorth_update", "update_x", "residual",
                                     "polesum", "apply_h", "grad_v", "lanczos_step"};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Restarted GMRES over a set of shifted systems that share one tiling scheme.
struct Solver {
  int S = 0, m = 0, max_cycles = 0, prec = 0, tile = 0, grid = 0, reorth = 1, ppt = 8;
  double eta = 1e-2;
  double inner_rtol = 0.0;
  std::vector<SysDesc> hsys;
  std::vector<int32_t> htile;
  int total_tiles = 0;
  std::vector<DevBuf> bufs;
  Work W{};
  SysDesc* dsys = nullptr;
  int32_t* dtile = nullptr;
  int32_t* dtsys = nullptr;   // system of each tile (sized for the smallest tile; null for capacity builds)
  // column-marching Lanczos pass (0: the row-staged pass)
  int col_kh = 0, col_L = 0, col_total = 0;
  bool col_strip = false;  // tiled pass over strips of rows (2D instances relabelled (rows, 1, columns))
  std::vector<int32_t> hcol;
  int32_t* dcol = nullptr;
  int32_t* dcolsys = nullptr;  // system of each marching item (sized for any plan that fits)
  int64_t colsys_cap = 0;
  // a solver whose systems change between runs (fallback solves) is built
  // for at most cap_S systems of cap_pts points in total
  int cap_S = 0;
  int64_t cap_pts = 0;
  // per-pole finite-difference solves: the basis is stored tile-interleaved
  // (the points of one work tile of all m + 1 vectors contiguous)
  bool ilv = false;
  bool ready = false;
};

// log2 of a power of two
inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
// points of a system's vector in an interleaved basis (room for any tile of
// at most 8 TPB points)
inline int64_t ilv_points(int64_t n) { return (n + 8 * rexi::TPB - 1) / (8 * rexi::TPB) * (8 * rexi::TPB); }

struct Prof {
  bool on = false;
  int64_t launches[PC_NCLASS] = {};
  double ms[PC_NCLASS] = {};
  double bytes[PC_NCLASS] = {};
  std::vector<hipEvent_t> ev;      // pool, pairs
  std::vector<int> cls;            // class per recorded pair
  std::vector<double> pbytes;      // bytes per recorded pair
  std::vector<int> pcount;         // launches per recorded pair
  size_t used = 0;
  int suspend = 0;                 // > 0: record nothing (a stream is being captured)
};

}  // namespace

struct rexi_handle {
  rexi_options opt{};
  int ninst = 0;
  int64_t N = 0;
  std::vector<InstDesc> hinst;
  std::vector<int32_t> hitile;
  int itotal = 0;
  InstDesc* dinst = nullptr;
  int32_t* ditile = nullptr;
  double* V64 = nullptr;
  float* V32 = nullptr;
  std::vector<cplx> s, w;             // per system (pole), instance order
  std::vector<double> tol_sys, dist_sys, lam_lo, lam_hi;  // spectrum bound of the solved operator
  std::vector<double> center;         // per instance: the solves use H - center I
  std::vector<int> Kinst;
  Solver fwd, adj;
  Solver fb;                          // per-pole solves of poles the shared basis missed
  int fb_cycles = 0;                  // most cycles of those solves (last step)
  int fb_poles = 0;                   // poles they took over (last step)
  int64_t fb_its = 0;                 // their iterations (last step)
  double2* fb_rhs = nullptr;          // a copy of psi when the step is in place (out = psi)
  // restarts on the shared basis (fallback = 1): the cycles' view of SW,
  // their right-hand side and per-pole / per-instance bookkeeping
  bool rs_ready = false;
  rexi::ShiftWork SWR{};
  double2* rs_rhs = nullptr;
  int32_t *rs_miss = nullptr, *rs_kbase = nullptr, *rs_hasmiss = nullptr;
  double *rs_gam = nullptr, *rs_bn0 = nullptr;
  int rs_k_hint = 0, rs_reorth = 0;
  int rs_cycles = 0;                  // restart cycles of the last step
  int64_t rs_its = 0;                 // their iterations summed over instances
  std::vector<rexi::SysState_t> st0;  // per-instance states after the first cycle of the last solve
  // shared-basis solver: fwd holds one system (H, shift 0) per instance
  bool shifted = false;
  rexi::ShiftWork SW{};
  rexi::ShiftWork noshift{};          // K = 0: per-pole Givens in pass B
  std::vector<DevBuf> sbufs;
  int32_t* hpin = nullptr;            // pinned counters read-back
  SysState_t* hst = nullptr;          // pinned system states read with each convergence check
  int hst_cap = 0;
  // capture-safe steps: no host reads, fixed schedule (set while launching one)
  bool syncfree = false;
  hipStream_t cap_stream = nullptr;   // internal stream for graph capture
  struct GraphEntry {
    const void* in;
    void* out;
    int nsteps;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  // iteration-chunk graphs of the shared-basis loop, keyed by (first, count)
  struct ChunkGraph {
    int j0, len;
    hipGraphExec_t exec;
  };
  std::vector<ChunkGraph> chunks;
  std::vector<ChunkGraph> rs_chunks;  // the same for the restart cycles (their own ShiftWork)
  int k_hint = 0;                     // iterations the last shared-basis solve took
  int reorth_passes = 0;              // second passes of the last shared-basis solve
  // shared-basis adjoint: a second basis for the solves with conjugate shifts
  Solver fwdA;
  rexi::ShiftWork SWA{};
  std::vector<ChunkGraph> chunksA;
  int k_hintA = 0, reorth_passesA = 0;
  double2* adj_coef = nullptr;        // [m][m] coefficients of the gradient's bilinear form
  double* dnorm = nullptr;            // scratch partials for norms
  double2* mrhs = nullptr;            // Q1 elements: M psi (per pole), L^T psi (shared basis)
  // Q1 elements with the shared basis: M = L L^T, the solves run on
  // Ahat = L^-1 A L^-T (one instance); chol holds the factors of L per axis,
  // fem_y the operator's intermediate vector
  bool fem_shared = false;
  double* chol = nullptr;
  double2* fem_y = nullptr;
  double2* fem_z = nullptr;           // second intermediate (the sweeps run out of place)
  int fem_warm[3] = {0, 0, 0};        // warm-up entries of a segment per axis
  std::string err;
  Prof prof;
  int64_t ws_bytes = 0;
  void* scratch = nullptr;            // device address of the allocation-free workspace on this device
  // explicit pole solutions of the shared-basis solver (finite differences):
  // x_p of every pole at X + xoff[p] (FP64), the tile partials and norms of
  // their residuals, and a copy of psi for in-place steps
  double2* X = nullptr;
  int64_t* dxoff = nullptr;
  std::vector<int64_t> hxoff;
  int32_t* dpoff = nullptr;
  double* xpart = nullptr;
  double* xrn = nullptr;
  double2* xb = nullptr;
  bool want_x = false;                // this solve forms the solutions
  bool want_res = false;              // ... and their explicit residuals
  bool x_valid = false;               // X holds the solutions of the last step
  bool x_res = false;                 // xrn holds their residual norms
  bool stepped = false;               // a step has run (per pole: W.x holds its solutions)
  int32_t* jdev = nullptr;            // device iteration indices of captured schedules (2 ints)
};

namespace {

rexi_status fail(rexi_handle* h, rexi_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf; else g_setup_error = buf;
  return st;
}

#define HIPCHK(h, call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((h), REXI_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));           \
  } while (0)

bool is_fin(double v) { return std::isfinite(v); }

void free_solver(Solver& sv) {
  for (auto& b : sv.bufs)
    if (b.p) (void)hipFree(b.p);
  sv.bufs.clear();
  sv.ready = false;
}

void destroy_handle(rexi_handle* h) {
  if (!h) return;
  free_solver(h->fwd);
  free_solver(h->adj);
  free_solver(h->fb);
  free_solver(h->fwdA);
  for (auto& g : h->chunksA) (void)hipGraphExecDestroy(g.exec);
  if (h->adj_coef) (void)hipFree(h->adj_coef);
  for (auto& b : h->sbufs)
    if (b.p) (void)hipFree(b.p);
  if (h->dinst) (void)hipFree(h->dinst);
  if (h->ditile) (void)hipFree(h->ditile);
  if (h->V64) (void)hipFree(h->V64);
  if (h->V32) (void)hipFree(h->V32);
  if (h->dnorm) (void)hipFree(h->dnorm);
  if (h->mrhs) (void)hipFree(h->mrhs);
  if (h->chol) (void)hipFree(h->chol);
  if (h->fem_y) (void)hipFree(h->fem_y);
  if (h->fem_z) (void)hipFree(h->fem_z);
  if (h->fb_rhs) (void)hipFree(h->fb_rhs);
  if (h->hpin) (void)hipHostFree(h->hpin);
  if (h->hst) (void)hipHostFree(h->hst);
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  for (auto& g : h->chunks) (void)hipGraphExecDestroy(g.exec);
  for (auto& g : h->rs_chunks) (void)hipGraphExecDestroy(g.exec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (auto& e : h->prof.ev) (void)hipEventDestroy(e);
  delete h;
}

// ---------------------------------------------------------------- profiling
struct Timed {
  rexi_handle* h;
  int slot = -1;
  hipStream_t st;
  // count: launches of the class between the two events (a graph of several)
  Timed(rexi_handle* hh, int cls, double bytes, hipStream_t s, int count = 1) : h(hh), st(s) {
    Prof& P = h->prof;
    if (!P.on || h->syncfree || P.suspend) return;
    if (P.used + 2 > P.ev.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        P.ev.push_back(e);
      }
    }
    slot = (int)P.used;
    P.used += 2;
    P.cls.push_back(cls);
    P.pbytes.push_back(bytes);
    P.pcount.push_back(count);
    (void)hipEventRecord(P.ev[slot], st);
  }
  ~Timed() {
    if (slot >= 0) (void)hipEventRecord(h->prof.ev[slot + 1], st);
  }
};

void prof_collect(rexi_handle* h, hipStream_t st) {
  Prof& P = h->prof;
  if (!P.on || P.used == 0) return;
  (void)hipStreamSynchronize(st);
  for (size_t k = 0; k < P.cls.size(); ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P.ev[2 * k], P.ev[2 * k + 1]) == hipSuccess) {
      P.ms[P.cls[k]] += ms;
      P.launches[P.cls[k]] += P.pcount[k];
      P.bytes[P.cls[k]] += P.pbytes[k];
    }
  }
  P.cls.clear();
  P.pbytes.clear();
  P.pcount.clear();
  P.used = 0;
}

// ---------------------------------------------------------------- planning
template <typename X>
rexi_status dalloc(rexi_handle* h, Solver& sv, X** out, size_t count) {
  DevBuf b;
  b.bytes = std::max<size_t>(count * sizeof(X), 256);
  hipError_t e = hipMalloc(&b.p, b.bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, REXI_E_NO_MEMORY, "hipMalloc of %zu bytes failed: %s", b.bytes, hipGetErrorString(e));
  }
  sv.bufs.push_back(b);
  h->ws_bytes += (int64_t)b.bytes;
  *out = reinterpret_cast<X*>(b.p);
  return REXI_OK;
}

size_t solver_bytes(const std::vector<SysDesc>& sys, int m, int prec, int max_cycles, int total_tiles,
                    bool ilv) {
  size_t e = prec ? 8 : 16, tot = 0;
  for (auto& d : sys)
    tot += (size_t)(m + 1) * (ilv ? ilv_points(d.n) : d.n) * e + (size_t)d.n * 16 + (size_t)(m + 1) * d.ntiles * 16;
  size_t S = sys.size();
  tot += S * ((size_t)(m + 1) * m * 16 + (m + 1) * 16 * 2 + m * 16 * 3 + (m + 1) * 8 + sizeof(SysState_t));
  tot += (size_t)total_tiles * 8 + (size_t)(max_cycles * (m + 1) + max_cycles + 4) * 4;
  return tot;
}

// Build the system table of a solver: for each (instance, pole) in `order`.
void layout_systems(Solver& sv, int m) {
  int64_t basis = 0, xo = 0;
  int tile0 = 0, pbase = 0;
  sv.htile.clear();
  for (auto& d : sv.hsys) {
    d.ntiles = (d.n + sv.tile - 1) / sv.tile;
    d.tile0 = tile0;
    d.basis = basis;
    d.xoff = xo;
    d.pbase = pbase;
    sv.htile.push_back(tile0);
    tile0 += d.ntiles;
    basis += (int64_t)(m + 1) * (sv.ilv ? (int64_t)d.ntiles * sv.tile : d.n);
    xo += d.n;
    pbase += (m + 1) * d.ntiles;
  }
  sv.htile.push_back(tile0);
  sv.total_tiles = tile0;
  sv.S = (int)sv.hsys.size();
}

constexpr int TPB_ = rexi::TPB;

// Column-marching Lanczos pass: kh slots per thread cover a band of rows of
// the (i1, i2) plane and one halo row on each side; an item spans L planes.
// Fills the descriptors and the item prefix; false (nothing changed) if a
// system's rows do not fit or its six partial-sum slots (two parities of
// three, max(ntiles, items) entries each) exceed its partial-sum block of
// (m + 1) ntiles entries.
// kh = 2: the tiled pass, tiles of ZT_R x ZT_C points of the plane, or (strip)
// strips of ZS_C points of a row (any grid fits; tiles at the edges are clipped).
bool plan_columns(Solver& sv, int kh, int L, bool strip) {
  struct Plan { int rows, Lc, nr, n; };
  std::vector<Plan> pl;
  for (auto& d : sv.hsys) {
    const bool tiled = kh == 2;
    const int tr = strip ? 1 : rexi::ZT_R, tc = strip ? rexi::ZS_C : rexi::ZT_C;
    const int rows = tiled ? tr : std::min(d.n1, TPB_ * kh / d.n2 - 2);
    if (rows < 1) return false;
    // the tiled pass addresses a vector with 32-bit byte offsets below 2^31
    if (tiled && (int64_t)d.n * 16 >= ((int64_t)1 << 31)) return false;
    const int nb = tiled ? ((d.n1 + tr - 1) / tr) * ((d.n2 + tc - 1) / tc) : (d.n1 + rows - 1) / rows;
    const int Lc = std::min(L, d.n0);
    const int nr = (d.n0 + Lc - 1) / Lc;
    const int64_t items = (int64_t)nb * nr;
    if (6 * std::max<int64_t>(d.ntiles, items) > (int64_t)(sv.m + 1) * d.ntiles) return false;
    pl.push_back({rows, Lc, nr, (int)items});
  }
  sv.hcol.clear();
  int total = 0;
  for (size_t i = 0; i < sv.hsys.size(); ++i) {
    SysDesc& d = sv.hsys[i];
    d.col_rows = pl[i].rows;
    d.col_L = pl[i].Lc;
    d.col_nr = pl[i].nr;
    d.col_n = pl[i].n;
    d.col_cs = std::max(d.ntiles, pl[i].n);
    sv.hcol.push_back(total);
    total += pl[i].n;
  }
  sv.hcol.push_back(total);
  sv.col_total = total;
  sv.col_kh = kh;
  sv.col_L = L;
  sv.col_strip = strip;
  return true;
}

// The per-tile system table of a solver (after its layout changed).
rexi_status upload_tile_sys(rexi_handle* h, Solver& sv, hipStream_t stream) {
  sv.W.tile_sys = nullptr;
  if (!sv.dtsys || sv.S == 0) return REXI_OK;
  std::vector<int32_t> t((size_t)sv.total_tiles);
  for (int q = 0; q < sv.S; ++q)
    for (int it = sv.htile[q]; it < sv.htile[q + 1]; ++it) t[it] = q;
  HIPCHK(h, hipMemcpyAsync(sv.dtsys, t.data(), t.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipStreamSynchronize(stream));
  sv.W.tile_sys = sv.dtsys;
  return REXI_OK;
}

rexi_status build_solver(rexi_handle* h, Solver& sv, hipStream_t stream) {
  const int m = sv.m, S = sv.S;
  const int SA = sv.cap_S > 0 ? sv.cap_S : S;  // systems allocated for
  Work& W = sv.W;
  W = Work{};
  rexi_status st;
#define ALLOC(ptr, type, count) \
  if ((st = dalloc(h, sv, (type**)&(ptr), (size_t)(count))) != REXI_OK) return st
  ALLOC(sv.dsys, SysDesc, SA);
  ALLOC(sv.dtile, int32_t, SA + 1);
  ALLOC(sv.dcol, int32_t, SA + 1);
  SysState_t* dst;
  ALLOC(dst, SysState_t, SA);
  W.st = dst;
  ALLOC(W.H, double, (size_t)SA * (m + 1) * m * 2);
  ALLOC(W.hcur, double, (size_t)SA * (m + 1) * 2);
  ALLOC(W.gvec, double, (size_t)SA * (m + 1) * 2);
  ALLOC(W.gc, double, (size_t)SA * m * 2);
  ALLOC(W.gs, double, (size_t)SA * m * 2);
  ALLOC(W.cscale, double, (size_t)SA * (m + 1));
  ALLOC(W.y, double, (size_t)SA * m * 2);
  // partial sums sized for the smallest tile, so the tuner may switch tilings
  size_t npart = 0, nx = 0, nb = 0, ntmax = 0;
  if (sv.cap_S > 0) {
    // any set of cap_S systems of cap_pts points: each system adds at most one
    // partial tile of the smallest tile (512 points)
    ntmax = (size_t)(sv.cap_pts / (2 * TPB_)) + (size_t)sv.cap_S;
    npart = (size_t)(m + 1) * ntmax;
    nx = (size_t)sv.cap_pts;
    nb = (size_t)(m + 1) * sv.cap_pts;
  }
  for (auto& d : sv.hsys) {
    if (sv.cap_S > 0) break;
    const size_t nt = (size_t)(d.n + 2 * TPB_ - 1) / (2 * TPB_);
    npart += (size_t)(m + 1) * nt;
    ntmax += nt;
    nx += d.n;
    nb += (size_t)(m + 1) * (sv.ilv ? ilv_points(d.n) : d.n);
  }
  ALLOC(W.part, double, npart * 2);
  ALLOC(W.pnorm, double, ntmax);
  if (sv.cap_S == 0) ALLOC(sv.dtsys, int32_t, ntmax);
  if (sv.cap_S == 0) {
    // a marching plan fits when 6 max(ntiles, items) <= (m + 1) ntiles per system
    int64_t cap = 0;
    for (auto& d : sv.hsys) cap += (int64_t)(m + 1) * ((d.n + 2 * TPB_ - 1) / (2 * TPB_)) / 6 + 1;
    sv.colsys_cap = cap;
    ALLOC(sv.dcolsys, int32_t, cap);
  }
  ALLOC(W.counters, int32_t, sv.max_cycles * (m + 1) + sv.max_cycles + 4);
  ALLOC(W.x, double, nx * 2);
  if (sv.prec) {
    float* b;
    ALLOC(b, float, nb * 2);
    W.basis = b;
  } else {
    double* b;
    ALLOC(b, double, nb * 2);
    W.basis = b;
  }
#undef ALLOC
  if (S > 0) {
    HIPCHK(h, hipMemcpyAsync(sv.dsys, sv.hsys.data(), S * sizeof(SysDesc), hipMemcpyHostToDevice, stream));
    HIPCHK(h, hipMemcpyAsync(sv.dtile, sv.htile.data(), (S + 1) * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  }
  HIPCHK(h, hipStreamSynchronize(stream));
  W.sys = sv.dsys;
  W.tile_start = sv.dtile;
  W.V64 = h->V64;
  W.V32 = h->V32;
  W.S = S;
  W.m = m;
  W.total_tiles = sv.total_tiles;
  W.reorth_mode = sv.reorth;
  W.inner_rtol = sv.inner_rtol;
  W.eta2 = sv.eta * sv.eta;  // DGKS: second pass when ||w - V h|| < eta ||w||
  W.max_cycles = sv.max_cycles;
  W.tile = sv.tile;
  W.ilv = sv.ilv ? ilog2(sv.tile) : 0;
  if ((st = upload_tile_sys(h, sv, stream)) != REXI_OK) return st;
  sv.ready = true;
  return REXI_OK;
}

int default_grid(int total_tiles, int opt_grid) {
  if (opt_grid > 0) return opt_grid;
  return std::max(1, std::min(total_tiles, 2048));
}

// ---------------------------------------------------------------- solve
constexpr int TPB = rexi::TPB;
constexpr int INST_PPT = 8;  // points per thread of the instance-level kernels
constexpr int INST_TILE = TPB * INST_PPT;  // points per tile of the instance tiling (itotal, ditile)

// Restarted cycles of the per-pole solver from the current state: `active`
// systems are iterating, `total_restarts` restarts were counted so far.
template <typename T, int PPT>
rexi_status run_cycles(rexi_handle* h, Solver& sv, const double2* r0, const double2* r1, hipStream_t stream,
                       int active, int total_restarts, int* restarts_out) {
  Work& W = sv.W;
  const int G = sv.grid, S = sv.S, m = sv.m;
  const double e = sizeof(T);
  const double eV = sv.prec ? 4.0 : 8.0;
  double npts = 0;  // points per system (uniform tiling assumed for byte counts)
  for (auto& d : sv.hsys) npts += d.n;
  const double n_avg = npts / std::max(1, S);
  for (int c = 0; c < sv.max_cycles; ++c) {
    for (int j = 0; j < m; ++j) {
      {
        Timed t(h, PC_ARNOLDI_A, active * n_avg * ((j + 2) * e + eV), stream);
        hipLaunchKernelGGL((rexi::k_arnoldi_a<T, PPT, true>), dim3(G), dim3(TPB), 0, stream, W, j, 0, 0);
      }
      {
        Timed t(h, PC_REDUCE, 0, stream);
        hipLaunchKernelGGL(rexi::k_reduce_dots, dim3(S, j + 2), dim3(TPB), 0, stream, W, j, 0, 0);
      }
      {
        Timed t(h, PC_ARNOLDI_B, active * n_avg * (j + 3) * e, stream);
        hipLaunchKernelGGL((rexi::k_arnoldi_b<T, PPT>), dim3(G), dim3(TPB), 0, stream, W, j, 0, 0);
      }
      {
        Timed t(h, PC_REDUCE, 0, stream);
        hipLaunchKernelGGL(rexi::k_end_iter, dim3(S), dim3(TPB), 0, stream, W, h->noshift, j, 0, c);
      }
      if (sv.reorth) {
        {
          Timed t(h, PC_REORTH_A, 0, stream);
          hipLaunchKernelGGL((rexi::k_arnoldi_a<T, PPT, false>), dim3(G), dim3(TPB), 0, stream, W, j, 0, 0);
        }
        {
          Timed t(h, PC_REDUCE, 0, stream);
          hipLaunchKernelGGL(rexi::k_reduce_dots, dim3(S, j + 2), dim3(TPB), 0, stream, W, j, 1, 0);
        }
        {
          Timed t(h, PC_REORTH_B, 0, stream);
          hipLaunchKernelGGL((rexi::k_arnoldi_b<T, PPT>), dim3(G), dim3(TPB), 0, stream, W, j, 1, 0);
        }
        {
          Timed t(h, PC_REDUCE, 0, stream);
          hipLaunchKernelGGL(rexi::k_end_iter, dim3(S), dim3(TPB), 0, stream, W, h->noshift, j, 1, c);
        }
      }
      HIPCHK(h, hipGetLastError());
      if (h->syncfree) continue;  // fixed schedule: finished systems skip on the device
      HIPCHK(h, hipMemcpyAsync(h->hpin, W.counters + c * (m + 1) + j, sizeof(int32_t), hipMemcpyDeviceToHost,
                               stream));
      HIPCHK(h, hipStreamSynchronize(stream));
      active = h->hpin[0];
      if (active == 0) break;
    }
    // finishing systems: all that were active in this cycle
    {
      Timed t(h, PC_UPDATE_X, 0, stream);
      hipLaunchKernelGGL((rexi::k_update_x<T, PPT>), dim3(G), dim3(TPB), 0, stream, W);
    }
    {
      Timed t(h, PC_RESIDUAL, 0, stream);
      hipLaunchKernelGGL((rexi::k_residual<T, PPT>), dim3(G), dim3(TPB), 0, stream, W, r0, r1);
    }
    {
      Timed t(h, PC_REDUCE, 0, stream);
      hipLaunchKernelGGL(rexi::k_restart, dim3(S), dim3(TPB), 0, stream, W, c);
    }
    HIPCHK(h, hipGetLastError());
    if (h->syncfree) {
      if (c + 1 >= (h->opt.capture_cycles > 0 ? h->opt.capture_cycles : sv.prec ? 16 : 4)) break;
      continue;
    }
    // restarted count of this cycle: counters[max_cycles*(m+1)] accumulates; read the total
    HIPCHK(h, hipMemcpyAsync(h->hpin, W.counters + sv.max_cycles * (m + 1), 2 * sizeof(int32_t),
                             hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    const int restarted_total = h->hpin[0];
    const int restarted = restarted_total - total_restarts;
    total_restarts = restarted_total;
    if (restarted == 0) break;
    active = restarted;
  }
  if (restarts_out) *restarts_out = total_restarts;
  return REXI_OK;
}

template <typename T, int PPT>
rexi_status run_solve(rexi_handle* h, Solver& sv, const double2* r0, const double2* r1, hipStream_t stream,
                      int* restarts_out) {
  Work& W = sv.W;
  const int G = sv.grid, S = sv.S;
  double npts = 0;
  for (auto& d : sv.hsys) npts += d.n;
  {
    Timed t(h, PC_START, npts * (16.0 + sizeof(T)), stream);
    hipLaunchKernelGGL((rexi::k_start<T, PPT>), dim3(G), dim3(TPB), 0, stream, W, r0, r1);
  }
  {
    Timed t(h, PC_REDUCE, 0, stream);
    hipLaunchKernelGGL(rexi::k_start_reduce, dim3(S), dim3(TPB), 0, stream, W);
  }
  return run_cycles<T, PPT>(h, sv, r0, r1, stream, S, 0, restarts_out);
}

rexi_status solve(rexi_handle* h, Solver& sv, const double2* r0, const double2* r1, hipStream_t stream,
                  int* restarts) {
  switch (sv.ppt * 2 + sv.prec) {
    case 16: return run_solve<double2, 8>(h, sv, r0, r1, stream, restarts);
    case 17: return run_solve<float2, 8>(h, sv, r0, r1, stream, restarts);
    case 8: return run_solve<double2, 4>(h, sv, r0, r1, stream, restarts);
    case 9: return run_solve<float2, 4>(h, sv, r0, r1, stream, restarts);
    case 4: return run_solve<double2, 2>(h, sv, r0, r1, stream, restarts);
    case 5: return run_solve<float2, 2>(h, sv, r0, r1, stream, restarts);
  }
  return fail(h, REXI_E_INVALID_ARG, "unsupported tiling");
}

// Points per thread: the largest of 8, 4, 2 that still gives >= 1024 work
// tiles (four or more 4-wave blocks per compute unit).
int choose_ppt(int64_t points) {
  for (int p : {8, 4}) if (points / (TPB * p) >= 1024) return p;
  return 2;
}

void copy_fem(SysDesc& d, const InstDesc& in);

// Fill the system table for a set of poles of the handle's instances.
void make_systems(rexi_handle* h, Solver& sv, bool conj_shift, int rhs_sel) {
  int sidx = 0;
  for (int i = 0; i < h->ninst; ++i) {
    const InstDesc& in = h->hinst[i];
    for (int k = 0; k < h->Kinst[i]; ++k, ++sidx) {
      SysDesc d{};
      d.off = in.off;
      d.n = in.n;
      d.n0 = in.n0;
      d.n1 = in.n1;
      d.n2 = in.n2;
      d.d2 = in.d2;
      d.d1 = in.d1;
      d.c0 = in.c0;
      d.c1 = in.c1;
      d.c2 = in.c2;
      d.diag = in.diag - h->center[i];
      copy_fem(d, in);
      const cplx s = conj_shift ? std::conj(h->s[sidx]) : h->s[sidx];
      d.sre = s.real();
      d.sim = s.imag();
      d.wre = h->w[sidx].real();
      d.wim = h->w[sidx].imag();
      d.tol = h->tol_sys[sidx];
      d.dist = h->dist_sys[sidx];
      d.inst = i;
      d.rhs_sel = rhs_sel;
      sv.hsys.push_back(d);
    }
  }
}

rexi_status init_solver(rexi_handle* h, Solver& sv, int copies, hipStream_t stream) {
  sv.hsys.clear();
  if (copies == 0) {
    // shared-basis solver: one unshifted system per instance
    for (int i = 0; i < h->ninst; ++i) {
      const InstDesc& in = h->hinst[i];
      SysDesc d{};
      d.off = in.off;
      d.n = in.n;
      d.n0 = in.n0;
      d.n1 = in.n1;
      d.n2 = in.n2;
      d.d2 = in.d2;
      d.d1 = in.d1;
      d.c0 = in.c0;
      d.c1 = in.c1;
      d.c2 = in.c2;
      d.diag = in.diag - h->center[i];
      d.tol = 0.0;
      d.dist = 1.0;
      d.inst = i;
      sv.hsys.push_back(d);
    }
  }
  for (int c = 0; c < copies; ++c) make_systems(h, sv, c == 1, c);
  // per-pole finite-difference solves store their bases tile-interleaved
  // (Q1 element sweeps address whole vectors: they keep the plain layout)
  sv.ilv = copies > 0;
  for (auto& d : sv.hsys)
    if (d.fem) sv.ilv = false;
  sv.prec = h->opt.precision == REXI_PREC_C64_REFINE ? 1 : 0;
  int64_t pts = 0;
  for (auto& d : sv.hsys) pts += d.n;
  sv.ppt = choose_ppt(pts);
  if (h->opt.tile == 2 * TPB || h->opt.tile == 4 * TPB || h->opt.tile == 8 * TPB) sv.ppt = h->opt.tile / TPB;
  sv.tile = TPB * sv.ppt;
  sv.eta = h->opt.reorth_eta;
  sv.reorth = h->opt.reorth;
  sv.inner_rtol = sv.prec ? h->opt.inner_rtol : 0.0;
  sv.max_cycles = h->opt.max_cycles;
  // restart length: as asked, reduced until the workspace fits the budget
  size_t budget = (size_t)h->opt.max_workspace_bytes;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(h, REXI_E_HIP, "hipMemGetInfo failed");
    budget = (size_t)(0.9 * (double)fr);
  }
  // restart length: the option, except for the per-pole (adjoint) solves of a
  // shared-basis handle, whose m is the basis dimension: they restart at fallback_m
  int m = (h->shifted && copies > 0) ? h->opt.fallback_m : h->opt.m;
  for (;;) {
    layout_systems(sv, m);
    if (solver_bytes(sv.hsys, m, sv.prec, sv.max_cycles, sv.total_tiles, sv.ilv) <= budget) break;
    if (copies == 0) return fail(h, REXI_E_NO_MEMORY, "shared Krylov basis of dimension %d does not fit", m);
    if (m <= 4) return fail(h, REXI_E_NO_MEMORY, "Krylov workspace does not fit the %zu-byte budget", budget);
    m = std::max(4, m * 3 / 4);
  }
  sv.m = m;
  sv.grid = default_grid(sv.total_tiles, h->opt.grid_blocks);
  return build_solver(h, sv, stream);
}


// Shared-basis solver: one Krylov system per instance plus per-pole Givens data.
// conj: the poles' conjugates (s_j -> conj s_j, w_j -> conj w_j), for R^H.
rexi_status init_shifted(rexi_handle* h, Solver& sv, rexi::ShiftWork& SW, bool conj, hipStream_t stream) {
  rexi_status st = init_solver(h, sv, 0, stream);
  if (st != REXI_OK) return st;
  const int S = h->ninst, m = sv.m;
  int K = 0;
  for (int i = 0; i < S; ++i) K += h->Kinst[i];
  SW.K = K;
  auto al = [&](void** p, size_t bytes) -> rexi_status {
    DevBuf b;
    b.bytes = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, b.bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, REXI_E_NO_MEMORY, "hipMalloc failed: %s", hipGetErrorString(e));
    }
    h->sbufs.push_back(b);
    h->ws_bytes += (int64_t)b.bytes;
    *p = b.p;
    return REXI_OK;
  };
  const size_t c16 = 16, d8 = 8, i4 = 4;
  void *s = nullptr, *w = nullptr, *tol = nullptr, *its = nullptr, *pole0 = nullptr, *pinst = nullptr;
  void *R = nullptr, *g = nullptr, *gc = nullptr, *gs = nullptr, *y = nullptr, *z = nullptr, *res = nullptr;
  void *alpha = nullptr, *beta = nullptr, *omega = nullptr, *flags = nullptr, *full = nullptr, *reo = nullptr;
  if ((st = al(&s, K * c16)) || (st = al(&w, K * c16)) || (st = al(&tol, K * d8)) || (st = al(&its, K * i4)) ||
      (st = al(&pole0, (S + 1) * i4)) || (st = al(&pinst, K * i4)) ||
      (st = al(&R, (size_t)K * (m + 1) * m * c16)) || (st = al(&g, (size_t)K * (m + 1) * c16)) ||
      (st = al(&gc, (size_t)K * m * c16)) || (st = al(&gs, (size_t)K * m * c16)) ||
      (st = al(&y, (size_t)K * m * c16)) || (st = al(&z, (size_t)S * m * c16)) || (st = al(&res, K * d8)) ||
      (st = al(&alpha, (size_t)S * m * d8)) || (st = al(&beta, (size_t)S * (m + 1) * d8)) ||
      (st = al(&omega, (size_t)S * 2 * (m + 1) * d8)) || (st = al(&flags, (size_t)S * 4 * i4)) ||
      (st = al(&full, (size_t)S * m * i4)) || (st = al(&reo, (size_t)(m + 1) * i4)))
    return st;
  void* gp = nullptr;
  if ((st = al(&gp, i4))) return st;
  SW.gpause = (int32_t*)gp;
  if (!h->jdev) {
    void* jd = nullptr;
    if ((st = al(&jd, 2 * i4))) return st;
    h->jdev = (int32_t*)jd;
  }
  // certified policy: the weights of the instance-wide stopping test
  SW.cw = nullptr;
  SW.tau = h->opt.tol;
  if (h->opt.tol_policy == REXI_TOL_CERTIFIED) {
    void* cw = nullptr;
    if ((st = al(&cw, K * d8))) return st;
    std::vector<double> hc((size_t)K);
    for (int k = 0; k < K; ++k) hc[(size_t)k] = std::abs(h->w[(size_t)k]) / h->dist_sys[(size_t)k];
    HIPCHK(h, hipMemcpyAsync(cw, hc.data(), hc.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    SW.cw = (const double*)cw;
  }
  sv.W.reo_any = (int32_t*)reo;
  SW.s = (const double*)s;
  SW.w = (const double*)w;
  SW.tol = (const double*)tol;
  SW.its = (int32_t*)its;
  SW.pole0 = (const int32_t*)pole0;
  SW.pinst = (const int32_t*)pinst;
  SW.R = (double*)R;
  SW.g = (double*)g;
  SW.gc = (double*)gc;
  SW.gs = (double*)gs;
  SW.y = (double*)y;
  SW.z = (double*)z;
  SW.res = (double*)res;
  SW.alpha = (double*)alpha;
  SW.beta = (double*)beta;
  SW.omega = (double*)omega;
  SW.flags = (int32_t*)flags;
  SW.full = (int32_t*)full;
  SW.lanczos = h->opt.lanczos ? 1 : 0;
  if (h->opt.lanczos == 1) {
    // pipelined recurrence: two z buffers of all instances' points
    int64_t tot = 0;
    for (auto& d : sv.hsys) tot += d.n;
    void* zb = nullptr;
    if ((st = al(&zb, (size_t)2 * tot * c16))) return st;
    SW.zb = (double*)zb;
    SW.zstride = tot;
  }
  if (SW.lanczos) {
    // the orthogonality estimate decides the second passes; the DGKS test is off
    sv.W.reorth_mode = 3;
  }
  std::vector<double> hs(2 * K), hw(2 * K), ht(K);
  std::vector<int32_t> hp0(S + 1), hpi(K);
  int q = 0;
  for (int i = 0; i < S; ++i) {
    hp0[i] = q;
    for (int k = 0; k < h->Kinst[i]; ++k, ++q) hpi[q] = i;
  }
  hp0[S] = q;
  for (int k = 0; k < K; ++k) {
    const double sg = conj ? -1.0 : 1.0;
    hs[2 * k] = h->s[k].real();
    hs[2 * k + 1] = sg * h->s[k].imag();
    hw[2 * k] = h->w[k].real();
    hw[2 * k + 1] = sg * h->w[k].imag();
    ht[k] = h->tol_sys[k];
  }
  HIPCHK(h, hipMemcpyAsync(s, hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipMemcpyAsync(w, hw.data(), hw.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipMemcpyAsync(tol, ht.data(), ht.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipMemcpyAsync(pole0, hp0.data(), hp0.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipMemcpyAsync(pinst, hpi.data(), hpi.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipMemsetAsync(flags, 0, (size_t)S * 4 * i4, stream));
  HIPCHK(h, hipMemsetAsync(full, 0, (size_t)S * m * i4, stream));
  HIPCHK(h, hipStreamSynchronize(stream));
  return REXI_OK;
}

// The fused Lanczos pass of iteration j: the marching pass when a column plan
// is selected, else the row-staged pass (n2 <= 512) or the plain one.
// Restart cycles on the shared basis (forward solver): the cycles' view of
// the shared-basis data (own weights, targets, iteration counts and
// residuals; the rest shared) and their bookkeeping.
rexi_status init_restart(rexi_handle* h, hipStream_t stream) {
  const int K = h->SW.K, S = h->fwd.S;
  void *gnext = nullptr, *miss = nullptr, *gam = nullptr, *w = nullptr, *tol = nullptr, *its = nullptr,
       *res = nullptr, *bn0 = nullptr, *kbase = nullptr, *hasmiss = nullptr, *rhs = nullptr;
  auto al = [&](void** p, size_t bytes) -> rexi_status {
    DevBuf b;
    b.bytes = std::max<size_t>(bytes, 256);
    if (hipMalloc(&b.p, b.bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, REXI_E_NO_MEMORY, "restart workspace (%zu bytes)", b.bytes);
    }
    h->sbufs.push_back(b);
    h->ws_bytes += (int64_t)b.bytes;
    *p = b.p;
    return REXI_OK;
  };
  rexi_status st;
  if ((st = al(&gnext, (size_t)K * 16)) || (st = al(&miss, (size_t)K * 4)) || (st = al(&gam, (size_t)K * 16)) ||
      (st = al(&w, (size_t)K * 16)) || (st = al(&tol, (size_t)K * 8)) || (st = al(&its, (size_t)K * 4)) ||
      (st = al(&res, (size_t)K * 8)) || (st = al(&bn0, (size_t)S * 8)) || (st = al(&kbase, (size_t)S * 4)) ||
      (st = al(&hasmiss, (size_t)S * 4)) || (st = al(&rhs, (size_t)h->N * 16)))
    return st;
  h->SW.gnext = (double*)gnext;
  rexi::ShiftWork R = h->SW;
  R.w = (const double*)w;
  R.tol = (const double*)tol;
  R.its = (int32_t*)its;
  R.res = (double*)res;
  R.fom = 1;
  R.fb_skip = 0;
  R.restart = 1;
  R.cw = nullptr;  // restart cycles: per-pole targets (weights scaled by gam)
  R.miss = (const int32_t*)miss;
  R.gam = (const double*)gam;
  R.w0 = h->SW.w;
  R.tol0 = h->SW.tol;
  R.bn0 = (const double*)bn0;
  h->SWR = R;
  h->rs_miss = (int32_t*)miss;
  h->rs_gam = (double*)gam;
  h->rs_bn0 = (double*)bn0;
  h->rs_kbase = (int32_t*)kbase;
  h->rs_hasmiss = (int32_t*)hasmiss;
  h->rs_rhs = (double2*)rhs;
  h->rs_ready = true;
  (void)stream;
  return REXI_OK;
}

// Explicit pole solutions of the shared-basis solver (finite differences): x_p
// of every pole ([sum_i K_i n_i] complex128), the per-tile residual partials
// and norms, and a copy of psi for in-place steps. Planned last at setup (the
// partials follow the final tiling). keep_solutions = 1 requires them; else
// they are planned when they take at most half of the free memory, and steps
// with info then report explicit residuals.
rexi_status init_solutions(rexi_handle* h, hipStream_t stream) {
  Solver& sv = h->fwd;
  const int K = h->SW.K;
  std::vector<int64_t> xo((size_t)K);
  std::vector<int32_t> po((size_t)K);
  int64_t xtot = 0, ptot = 0;
  int q = 0;
  for (int i = 0; i < sv.S; ++i)
    for (int k = 0; k < h->Kinst[i]; ++k, ++q) {
      xo[q] = xtot;
      po[q] = (int32_t)ptot;
      xtot += sv.hsys[i].n;
      ptot += sv.hsys[i].ntiles;
    }
  if (ptot > INT32_MAX) return h->opt.keep_solutions ? fail(h, REXI_E_NO_MEMORY, "too many solution tiles") : REXI_OK;
  const size_t bx = (size_t)xtot * sizeof(double2), bp = (size_t)std::max<int64_t>(ptot, 1) * sizeof(double);
  const size_t total = bx + bp + (size_t)K * 20 + (size_t)h->N * sizeof(double2);
  if (!h->opt.keep_solutions) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(h, REXI_E_HIP, "hipMemGetInfo failed");
    if (total > fr / 2) return REXI_OK;
  }
  auto al = [&](void** p, size_t bytes) -> rexi_status {
    DevBuf b;
    b.bytes = std::max<size_t>(bytes, 256);
    if (hipMalloc(&b.p, b.bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, REXI_E_NO_MEMORY, "pole solutions (%zu bytes)", total);
    }
    h->sbufs.push_back(b);
    h->ws_bytes += (int64_t)b.bytes;
    *p = b.p;
    return REXI_OK;
  };
  void *X = nullptr, *xoff = nullptr, *poff = nullptr, *part = nullptr, *rn = nullptr, *xb = nullptr;
  rexi_status st;
  if ((st = al(&X, bx)) || (st = al(&xoff, (size_t)K * 8)) || (st = al(&poff, (size_t)K * 4)) ||
      (st = al(&part, bp)) || (st = al(&rn, (size_t)K * 8)) || (st = al(&xb, (size_t)h->N * sizeof(double2))))
    return st;
  HIPCHK(h, hipMemcpyAsync(xoff, xo.data(), (size_t)K * 8, hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipMemcpyAsync(poff, po.data(), (size_t)K * 4, hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipStreamSynchronize(stream));
  h->X = (double2*)X;
  h->dxoff = (int64_t*)xoff;
  h->hxoff = xo;
  h->dpoff = (int32_t*)poff;
  h->xpart = (double*)part;
  h->xrn = (double*)rn;
  h->xb = (double2*)xb;
  return REXI_OK;
}

// x_p (+)= V a_p y_p for all poles (gam, miss: a restart cycle), XG poles per launch.
template <int PPT>
rexi_status form_x(rexi_handle* h, const rexi::ShiftWork& SWc, const double* gam, const int32_t* miss,
                   hipStream_t stream) {
  Solver& sv = h->fwd;
  int kmax = 0;
  for (int k : h->Kinst) kmax = std::max(kmax, k);
  const size_t lds = (size_t)rexi::XG * sv.m * sizeof(double2);
  for (int g0 = 0; g0 < kmax; g0 += rexi::XG)
    hipLaunchKernelGGL((rexi::k_form_x<PPT>), dim3(sv.grid), dim3(TPB), lds, stream, sv.W, SWc, h->X,
                       (const int64_t*)h->dxoff, g0, gam, miss);
  HIPCHK(h, hipGetLastError());
  return REXI_OK;
}

// Explicit FP64 residual norms ||b - (H - s_p) x_p|| of the solutions in X.
template <int PPT>
rexi_status explicit_residuals(rexi_handle* h, const double2* b, hipStream_t stream) {
  Solver& sv = h->fwd;
  hipLaunchKernelGGL((rexi::k_x_resid<PPT>), dim3(sv.grid), dim3(TPB), 0, stream, sv.W, h->SW, b,
                     (const double2*)h->X, (const int64_t*)h->dxoff, (const int32_t*)h->dpoff, h->xpart);
  hipLaunchKernelGGL(rexi::k_x_resid_norm, dim3(h->SW.K), dim3(TPB), 0, stream, sv.W, h->SW,
                     (const double*)h->xpart, (const int32_t*)h->dpoff, h->xrn);
  HIPCHK(h, hipGetLastError());
  h->x_res = true;
  return REXI_OK;
}

// Workspace of the per-pole solves that finish poles the shared basis missed:
// complex64 basis + FP64 refinement, restart length fallback_m, for at most
// cap_pts points over at most cap_S systems (one wave of those poles).
// points per thread of the fallback solves (their tiles are TPB * FB_PPT points)
constexpr int FB_PPT = 4;

rexi_status init_fallback(rexi_handle* h, hipStream_t stream) {
  Solver& fb = h->fb;
  fb.hsys.clear();
  fb.m = h->opt.fallback_m;
  fb.prec = 1;
  fb.ppt = FB_PPT;
  fb.tile = TPB_ * fb.ppt;
  fb.eta = h->opt.reorth_eta;
  fb.reorth = h->opt.reorth;
  fb.inner_rtol = h->opt.inner_rtol;
  fb.max_cycles = h->opt.max_cycles;
  int64_t nmax = 0, all = 0;
  for (int i = 0; i < h->ninst; ++i) {
    nmax = std::max<int64_t>(nmax, h->hinst[i].n);
    all += (int64_t)h->hinst[i].n * h->Kinst[i];
  }
  const double per_pt = (fb.m + 1) * 8.0 + 16.0 + 8.0 * (fb.m + 1) / (2 * TPB_) * 2.0;
  size_t budget = (size_t)h->opt.fallback_bytes;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(h, REXI_E_HIP, "hipMemGetInfo failed");
    budget = std::min<size_t>((size_t)16 << 30, fr / 4);
  }
  fb.cap_pts = std::min<int64_t>(all, (int64_t)((double)budget / per_pt));
  if (fb.cap_pts < nmax) return REXI_OK;  // no room for one solve of the largest instance: no fallback
  fb.cap_S = (int)std::min<int64_t>((int64_t)h->s.size(), 4096);
  fb.S = 0;
  fb.total_tiles = 0;
  fb.htile.assign(1, 0);
  rexi_status st = build_solver(h, fb, stream);
  if (st != REXI_OK) return st;
  fb.grid = 1;
  // in-place steps overwrite psi with the shared-basis sum before these
  // solves read it: they read this copy instead
  if (hipMalloc(&h->fb_rhs, (size_t)h->N * sizeof(double2)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, REXI_E_NO_MEMORY, "fallback right-hand side");
  }
  h->ws_bytes += h->N * (int64_t)sizeof(double2);
  return REXI_OK;
}

// Finish the poles p of `poles` (all missed their target in the shared basis,
// whose iterates y_p are current) by per-pole solves in waves, and add
// sum_p w_p x_p to out.
rexi_status run_fallback(rexi_handle* h, const std::vector<int>& poles, const double2* b, double2* out,
                         hipStream_t stream) {
  Solver& fb = h->fb;
  Solver& sv = h->fwd;
  std::vector<int> pinst(h->s.size());
  {
    int q = 0;
    for (int i = 0; i < h->ninst; ++i)
      for (int k = 0; k < h->Kinst[i]; ++k) pinst[q++] = i;
  }
  int kshared = 0;
  {
    std::vector<SysState_t> sst((size_t)sv.S);
    HIPCHK(h, hipMemcpyAsync(sst.data(), sv.W.st, sv.S * sizeof(SysState_t), hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    for (auto& x : sst) kshared = std::max(kshared, x.kcyc);
  }
  h->fb_cycles = 0;
  h->fb_its = 0;
  size_t next = 0;
  while (next < poles.size()) {
    // one wave: as many poles as fit the workspace
    fb.hsys.clear();
    int64_t pts = 0;
    while (next < poles.size() && (int)fb.hsys.size() < fb.cap_S) {
      const int p = poles[next];
      const InstDesc& in = h->hinst[pinst[p]];
      if (pts + in.n > fb.cap_pts) break;
      SysDesc d{};
      d.off = in.off;
      d.n = in.n;
      d.n0 = in.n0;
      d.n1 = in.n1;
      d.n2 = in.n2;
      d.d2 = in.d2;
      d.d1 = in.d1;
      d.c0 = in.c0;
      d.c1 = in.c1;
      d.c2 = in.c2;
      d.diag = in.diag - h->center[pinst[p]];
      d.sre = h->s[p].real();
      d.sim = h->s[p].imag();
      d.wre = h->w[p].real();
      d.wim = h->w[p].imag();
      d.tol = h->tol_sys[p];
      d.dist = h->dist_sys[p];
      d.inst = pinst[p];
      d.pole = p;
      fb.hsys.push_back(d);
      pts += in.n;
      ++next;
    }
    layout_systems(fb, fb.m);
    fb.W.S = fb.S;
    fb.W.total_tiles = fb.total_tiles;
    fb.W.tile = fb.tile;
    fb.grid = default_grid(fb.total_tiles, 0);
    HIPCHK(h, hipMemcpyAsync(fb.dsys, fb.hsys.data(), fb.S * sizeof(SysDesc), hipMemcpyHostToDevice, stream));
    HIPCHK(h, hipMemcpyAsync(fb.dtile, fb.htile.data(), (fb.S + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                             stream));
    Work& F = fb.W;
    // warm start: x = V y_p, then the explicit residual and restart decision
    hipLaunchKernelGGL(rexi::k_fb_init_x, dim3(fb.grid), dim3(TPB), 0, stream, F, sv.W, h->SW);
    hipLaunchKernelGGL(rexi::k_fb_state, dim3(fb.S), dim3(TPB), 0, stream, F, sv.W);
    hipLaunchKernelGGL((rexi::k_residual<float2, FB_PPT>), dim3(fb.grid), dim3(TPB), 0, stream, F, b, b);
    hipLaunchKernelGGL(rexi::k_restart, dim3(fb.S), dim3(TPB), 0, stream, F, 0);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(h->hpin, F.counters + fb.max_cycles * (fb.m + 1), sizeof(int32_t),
                             hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    const int active = h->hpin[0];
    if (active > 0) {
      rexi_status rs = run_cycles<float2, FB_PPT>(h, fb, b, b, stream, active, active, nullptr);
      if (rs != REXI_OK) return rs;
    }
    hipLaunchKernelGGL(rexi::k_fb_report, dim3(fb.S), dim3(64), 0, stream, F, h->SW, kshared);
    for (int q = 0; q < fb.S; ++q)
      hipLaunchKernelGGL(rexi::k_fb_accumulate, dim3(256), dim3(TPB), 0, stream, F, q, out);
    HIPCHK(h, hipGetLastError());
    if (h->want_x && h->X)
      for (const SysDesc& d : fb.hsys)
        HIPCHK(h, hipMemcpyAsync(h->X + h->hxoff[(size_t)d.pole], reinterpret_cast<const double2*>(fb.W.x) + d.xoff,
                                 (size_t)d.n * sizeof(double2), hipMemcpyDeviceToDevice, stream));
    std::vector<SysState_t> fst((size_t)fb.S);
    HIPCHK(h, hipMemcpyAsync(fst.data(), F.st, fb.S * sizeof(SysState_t), hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    for (auto& x : fst) {
      h->fb_cycles = std::max(h->fb_cycles, x.cycles);
      h->fb_its += x.its;
    }
  }
  return REXI_OK;
}

// fused (marching pass only): the pass of iteration j also ends iteration j - 1
template <int KH>
void launch_col(const Solver& sv, const rexi::Work& W, const rexi::ShiftWork& SW, int j, bool fused,
                hipStream_t strm) {
  if (fused) {
    const dim3 g((j < sv.m ? sv.col_total : 0) + sv.S);
    hipLaunchKernelGGL((rexi::k_lz_step_col<KH, true>), g, dim3(TPB), 0, strm, W, SW, j);
  } else {
    hipLaunchKernelGGL((rexi::k_lz_step_col<KH, false>), dim3(sv.col_total), dim3(TPB), 0, strm, W, SW, j);
  }
}

template <int TR, int TC, int NT>
void launch_tile(const Solver& sv, const rexi::Work& W, const rexi::ShiftWork& SW, int j, bool fused,
                 hipStream_t strm) {
  if (fused) {
    const dim3 g((j < sv.m ? sv.col_total : 0) + sv.S);
    hipLaunchKernelGGL((rexi::k_lz_step_tile<TR, TC, NT, true>), g, dim3(NT), 0, strm, W, SW, j);
  } else {
    hipLaunchKernelGGL((rexi::k_lz_step_tile<TR, TC, NT, false>), dim3(sv.col_total), dim3(NT), 0, strm, W, SW, j);
  }
}

template <int PPT>
void launch_lz_step(const Solver& sv, const rexi::Work& W, const rexi::ShiftWork& SW, int j, hipStream_t strm,
                    bool fused = false) {
  if (sv.col_kh) {
    switch (sv.col_kh) {
      case 2:
        if (sv.col_strip) launch_tile<1, rexi::ZS_C, rexi::ZS_T>(sv, W, SW, j, fused, strm);
        else launch_tile<rexi::ZT_R, rexi::ZT_C, rexi::ZT_T>(sv, W, SW, j, fused, strm);
        return;
      case 3: launch_col<3>(sv, W, SW, j, fused, strm); return;
      case 5: launch_col<5>(sv, W, SW, j, fused, strm); return;
      default: launch_col<8>(sv, W, SW, j, fused, strm); return;
    }
  }
  bool lds_ok = true;  // the row-staged pass keeps a row of halo on each side in LDS
  for (auto& d : sv.hsys) lds_ok = lds_ok && d.n2 <= 512;
  if (lds_ok)
    hipLaunchKernelGGL((rexi::k_lz_step_lds<PPT, 512>), dim3(sv.grid), dim3(TPB), 0, strm, W, SW, j);
  else
    hipLaunchKernelGGL((rexi::k_lz_step<PPT>), dim3(sv.grid), dim3(TPB), 0, strm, W, SW, j);
}

// The tiling and fused Lanczos pass of a solver (defined with the tuner);
// SWp: the shared-basis data whose column plan they set (null: the handle's).
rexi_status apply_tiling(rexi_handle* h, Solver& sv, int ppt, int grid, hipStream_t stream,
                         rexi::ShiftWork* SWp = nullptr);
void set_row_planes(rexi_handle* h, Solver& sv, int mode);
rexi_status apply_columns(rexi_handle* h, Solver& sv, int kh, int L, hipStream_t stream,
                          rexi::ShiftWork* SWp = nullptr);

// One factor sweep of a Q1 shared-basis handle (src != dst): L_a^-1, or
// L_a^-T when backward.
void fem_sweep(const rexi_handle* h, const double2* src, double2* dst, int axis, int backward, hipStream_t st) {
  const InstDesc& in = h->hinst[0];
  const int na = axis == 0 ? in.n0 : (axis == 1 ? in.n1 : in.n2);
  const int64_t threads = (int64_t)(in.n / na) * ((na + rexi::FEM_SEG - 1) / rexi::FEM_SEG);
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((threads + rexi::FEM_TPB - 1) / rexi::FEM_TPB, 16384)));
  hipLaunchKernelGGL(rexi::k_fem_sweep, g, dim3(rexi::FEM_TPB), 0, st, in, (const double*)h->chol, src, dst, axis,
                     backward, h->fem_warm[axis]);
}

// One shared-basis solver: its basis and system table, per-pole data, cached
// chunk graphs and the length of its last solve.
struct ShiftCtx {
  Solver* sv;
  rexi::ShiftWork* SW;
  std::vector<rexi_handle::ChunkGraph>* chunks;
  int* k_hint;
  int* reorth_passes;
  // poles that miss their target within the basis (the forward solver only):
  // 0 left as they are, 1 restarts on the shared basis, 2 per-pole solves
  int finish;
};

ShiftCtx fwd_ctx(rexi_handle* h) {
  return {&h->fwd, &h->SW, &h->chunks, &h->k_hint, &h->reorth_passes, h->opt.fallback};
}
ShiftCtx adj_ctx(rexi_handle* h) { return {&h->fwdA, &h->SWA, &h->chunksA, &h->k_hintA, &h->reorth_passesA, 0}; }
ShiftCtx rs_ctx(rexi_handle* h) { return {&h->fwd, &h->SWR, &h->rs_chunks, &h->rs_k_hint, &h->rs_reorth, 0}; }

// The Lanczos (or Arnoldi) process of one shared-basis solve on b, up to the
// per-pole Givens data; with host checks, sst receives the per-instance
// states at its end and its_sum their iterations.
template <typename T, int PPT>
rexi_status shifted_pass(rexi_handle* h, ShiftCtx cx, const double2* b, hipStream_t stream,
                         std::vector<SysState_t>* sst_out, int64_t* its_sum) {
  Solver& sv = *cx.sv;
  rexi::ShiftWork& SWc = *cx.SW;
  Work& W = sv.W;
  const int G = sv.grid, m = sv.m;
  const double e = sizeof(T);
  const int S = sv.S;
  double n = 0.0;  // points over all instances (byte counts assume all active)
  for (auto& d : sv.hsys) n += d.n;
  {
    Timed t(h, PC_START, n * (16.0 + e), stream);
    hipLaunchKernelGGL((rexi::k_start<T, PPT>), dim3(G), dim3(TPB), 0, stream, W, b, b);
  }
  {
    Timed t(h, PC_REDUCE, 0, stream);
    hipLaunchKernelGGL(rexi::k_start_reduce, dim3(S), dim3(TPB), 0, stream, W);
    hipLaunchKernelGGL(rexi::k_shifted_init, dim3(S), dim3(TPB), 0, stream, W, SWc);
  }
  const bool pipe = h->opt.lanczos == 1;
  const int colparts = sv.col_kh ? 1 : 0;
  // the tiled pass forms H u_j itself: the matvecs outside it store no z
  const bool zfree = sv.col_kh == 2;
  if (pipe) {
    {
      Timed t(h, PC_START, n * (zfree ? 32.0 : 48.0), stream);
      hipLaunchKernelGGL((rexi::k_lz_matvec<PPT>), dim3(G), dim3(TPB), 0, stream, W, SWc, 0, zfree ? -1 : 0, 0);
    }
    {
      Timed t(h, PC_REDUCE, 0, stream);
      hipLaunchKernelGGL(rexi::k_lz_start, dim3(S), dim3(TPB), 0, stream, W, SWc);
    }
  }
  // iterations run in chunks between host reads of the convergence counter;
  // iterations after convergence return at once (device-side state)
  const int chunk = std::max(1, h->opt.check_every);
  const bool lz = SWc.lanczos != 0;
  // second Gram-Schmidt passes are rare with the Lanczos estimate: a single
  // instance solved with host checks pauses for them (the host runs the pass
  // and resumes); otherwise they are predicated launches on a quarter grid
  // (the pipelined recurrence pauses every system of a batch at once, so
  // they stay in step: the ends of iteration j have all run when it pauses)
  const bool pause_mode = lz && !h->syncfree && (S == 1 || h->opt.lanczos == 1);
  rexi::ShiftWork SWl = SWc;
  SWl.pause_mode = pause_mode ? 1 : 0;
  const int G2 = lz ? std::max(1, G / 4) : G;
  auto second_pass = [&](int j, hipStream_t strm, int grid2) {
    if (pipe) {
      // re-orthogonalise u_{j+1}, recompute z_{j+1} = H u_{j+1}, then the Givens step
      {
        Timed t(h, PC_REORTH_A, 0, strm);
        hipLaunchKernelGGL((rexi::k_arnoldi_a<T, PPT, false>), dim3(grid2), dim3(TPB), 0, strm, W, j, 0, 0);
      }
      {
        Timed t(h, PC_REDUCE, 0, strm);
        hipLaunchKernelGGL(rexi::k_reduce_dots, dim3(S, j + 2), dim3(TPB), 0, strm, W, j, 1, 0);
      }
      {
        Timed t(h, PC_REORTH_B, 0, strm);
        hipLaunchKernelGGL((rexi::k_arnoldi_b<T, PPT>), dim3(grid2), dim3(TPB), 0, strm, W, j, 1, 0);
      }
      {
        Timed t(h, PC_REORTH_B, 0, strm);
        hipLaunchKernelGGL((rexi::k_lz_matvec<PPT>), dim3(grid2), dim3(TPB), 0, strm, W, SWc, j + 1,
                           zfree ? -1 : (j + 1) & 1, 1);
      }
      {
        Timed t(h, PC_REDUCE, 0, strm);
        hipLaunchKernelGGL(rexi::k_lz_end_second, dim3(S), dim3(TPB), 0, strm, W, SWl, j);
      }
      return;
    }
    {
      Timed t(h, PC_REORTH_A, 0, strm);
      hipLaunchKernelGGL((rexi::k_arnoldi_a<T, PPT, false>), dim3(grid2), dim3(TPB), 0, strm, W, j, 0, 0);
    }
    {
      Timed t(h, PC_REDUCE, 0, strm);
      hipLaunchKernelGGL(rexi::k_reduce_dots, dim3(S, j + 2), dim3(TPB), 0, strm, W, j, 1, 0);
    }
    {
      Timed t(h, PC_REORTH_B, 0, strm);
      hipLaunchKernelGGL((rexi::k_arnoldi_b<T, PPT>), dim3(grid2), dim3(TPB), 0, strm, W, j, 1, 0);
    }
    {
      Timed t(h, PC_REDUCE, 0, strm);
      hipLaunchKernelGGL(rexi::k_end_iter, dim3(S), dim3(TPB), 0, strm, W, SWl, j, 1, 0);
    }
  };
  // systems that pause together for second passes, with a marching pass:
  // the pass of iteration j + 1 also ends iteration j of every system (one
  // kernel per iteration, S blocks after the items); iteration(j) then
  // launches that pass, after a plain pass for the first iteration and after
  // every second Gram-Schmidt pass (which recomputes the pass that ran past
  // the pause)
  const bool fuse = pipe && pause_mode && sv.col_kh != 0;
  // algorithmic bytes per point of the pass of iteration j: reads z_j, u_j,
  // u_{j-1}, V and writes u_{j+1}, z_{j+1} (no u_{j-1} at j = 0); the tiled
  // pass forms z_j in place and stores no z
  const bool ztile = sv.col_kh == 2;
  auto lz_bytes = [&](int j) { return ztile ? (j > 0 ? 56.0 : 40.0) : (j > 0 ? 88.0 : 72.0); };
  auto plain_step = [&](int j, hipStream_t strm) {
    Timed t(h, PC_LANCZOS, n * lz_bytes(j), strm);
    launch_lz_step<PPT>(sv, W, SWl, j, strm);
  };
  auto iteration = [&](int j, hipStream_t strm) {
    if (fuse) {
      Timed t(h, PC_LANCZOS, j + 1 < m ? n * lz_bytes(j + 1) : 0.0, strm);
      launch_lz_step<PPT>(sv, W, SWl, j + 1, strm, true);
      return;
    }
    if (pipe) {
      {
        Timed t(h, PC_LANCZOS, n * lz_bytes(j), strm);
        launch_lz_step<PPT>(sv, W, SWl, j, strm);
      }
      {
        Timed t(h, PC_REDUCE, 0, strm);
        hipLaunchKernelGGL(rexi::k_lz_end, dim3(S), dim3(TPB), 0, strm, W, SWl, j, colparts);
      }
      if (!pause_mode) second_pass(j, strm, G2);
      return;
    }
    // Lanczos: project on v_{j-1}, v_j only (H is Hermitian); Arnoldi: on all
    const int i0 = lz ? std::max(0, j - 1) : 0;
    const int nproj = j + 1 - i0;
    if (h->fem_shared) {
      // Q1 elements: u_{j+1} <- Ahat u_j = L^-1 A L^-T u_j (three sweeps, the
      // element operator, three sweeps), then the first pass on it
      const InstDesc& in = h->hinst[0];
      double2* b0 = reinterpret_cast<double2*>(W.basis) + sv.hsys[0].basis;
      const double2* uj = b0 + (int64_t)j * in.n;
      double2* un = b0 + (int64_t)(j + 1) * in.n;
      const dim3 gs(std::max(1, std::min((in.n + TPB - 1) / TPB, 2048)));
      Timed t(h, PC_ARNOLDI_A, n * (12 * 32.0 + (nproj + 1) * e + 8.0), strm);
      // L^-T: u_j -> z -> y -> z; A: z -> y; L^-1: y -> z -> y -> u_{j+1}
      fem_sweep(h, uj, h->fem_z, 0, 1, strm);
      fem_sweep(h, h->fem_z, h->fem_y, 1, 1, strm);
      fem_sweep(h, h->fem_y, h->fem_z, 2, 1, strm);
      hipLaunchKernelGGL(rexi::k_fem_apply, gs, dim3(TPB), 0, strm, in, h->V64, (const double2*)h->fem_z, h->fem_y);
      fem_sweep(h, h->fem_y, h->fem_z, 0, 0, strm);
      fem_sweep(h, h->fem_z, h->fem_y, 1, 0, strm);
      fem_sweep(h, h->fem_y, un, 2, 0, strm);
      hipLaunchKernelGGL((rexi::k_arnoldi_a<T, PPT, false>), dim3(G), dim3(TPB), 0, strm, W, j, i0, 1);
    } else {
      Timed t(h, PC_ARNOLDI_A, n * ((nproj + 1) * e + 8.0), strm);
      hipLaunchKernelGGL((rexi::k_arnoldi_a<T, PPT, true>), dim3(G), dim3(TPB), 0, strm, W, j, i0, 0);
    }
    {
      Timed t(h, PC_REDUCE, 0, strm);
      hipLaunchKernelGGL(rexi::k_reduce_dots, dim3(S, j + 2), dim3(TPB), 0, strm, W, j, 0, i0);
    }
    {
      Timed t(h, PC_ARNOLDI_B, n * (nproj + 2) * e, strm);
      hipLaunchKernelGGL((rexi::k_arnoldi_b<T, PPT>), dim3(G), dim3(TPB), 0, strm, W, j, 0, i0);
    }
    {
      Timed t(h, PC_REDUCE, 0, strm);
      hipLaunchKernelGGL(rexi::k_end_iter, dim3(S), dim3(TPB), 0, strm, W, SWl, j, 0, 0);
    }
    if ((sv.reorth || lz) && !pause_mode) second_pass(j, strm, G2);
  };
  // captured schedule with the fused tiled pass: one launch per iteration
  // whose index lives on the device, so that a pause for a second pass (which
  // the host cannot see) only shifts the later launches; after every group
  // of QB launches a recovery runs the second pass of a paused iteration and
  // the pass after it (each launch predicated: nothing happens without a
  // pause). A pause costs the rest of its group; the schedule has QB launches
  // beyond m for each of the capture_pauses pauses it makes room for (more
  // pauses shorten the largest Krylov dimension a captured solve reaches).
  const bool capfuse = h->syncfree && pipe && lz && sv.col_kh == 2 && h->jdev;
  if (capfuse) {
    // a single instance: groups of 32 (a recovery is seven launches, which
    // cost about as much as the launches of a converged solve), room for one
    // pause; a batch pauses all its instances whenever one needs a pass:
    // groups of 16, room for max(2, m / 32) pauses
    const int QB = S == 1 ? 32 : 16;
    const int QR = h->opt.capture_pauses > 0 ? h->opt.capture_pauses : S == 1 ? 1 : std::max(2, m / 32);
    Work Wd = W;
    Wd.jdev = h->jdev;
    rexi::ShiftWork SWd = SWc;
    SWd.pause_mode = 1;
    hipLaunchKernelGGL(rexi::k_cap_init, dim3(1), dim3(64), 0, stream, Wd);
    {
      Timed t(h, PC_LANCZOS, n * lz_bytes(0), stream);
      launch_lz_step<PPT>(sv, Wd, SWd, 0, stream);
    }
    const int total = m + QR * QB;
    for (int L = 1; L <= total;) {
      for (int b = 0; b < QB && L <= total; ++b, ++L) {
        Timed t(h, PC_LANCZOS, 0, stream);
        launch_lz_step<PPT>(sv, Wd, SWd, rexi::JD_LAUNCH - L, stream, true);
      }
      hipLaunchKernelGGL(rexi::k_resume, dim3(S), dim3(64), 0, stream, Wd, SWd);
      {
        Timed t(h, PC_REORTH_A, 0, stream);
        hipLaunchKernelGGL((rexi::k_arnoldi_a<T, PPT, false>), dim3(G2), dim3(TPB), 0, stream, Wd, rexi::JD_REC, 0, 0);
      }
      {
        Timed t(h, PC_REDUCE, 0, stream);
        hipLaunchKernelGGL(rexi::k_reduce_dots, dim3(S, m + 1), dim3(TPB), 0, stream, Wd, rexi::JD_REC, 1, 0);
      }
      {
        Timed t(h, PC_REORTH_B, 0, stream);
        hipLaunchKernelGGL((rexi::k_arnoldi_b<T, PPT>), dim3(G2), dim3(TPB), 0, stream, Wd, rexi::JD_REC, 1, 0);
        hipLaunchKernelGGL((rexi::k_lz_matvec<PPT>), dim3(G2), dim3(TPB), 0, stream, Wd, SWc, rexi::JD_REC1, -1, 1);
      }
      {
        Timed t(h, PC_REDUCE, 0, stream);
        hipLaunchKernelGGL(rexi::k_lz_end_second, dim3(S), dim3(TPB), 0, stream, Wd, SWd, rexi::JD_REC);
      }
      {
        // (its first block also moves the later launches: launch L runs r + 2)
        rexi::ShiftWork SWr = SWd;
        SWr.cap_next = L;
        Timed t(h, PC_LANCZOS, 0, stream);
        launch_lz_step<PPT>(sv, Wd, SWr, rexi::JD_REC1, stream);
      }
    }
    HIPCHK(h, hipGetLastError());
  } else if (h->syncfree) {
    for (int j = 0; j < m; ++j) iteration(j, stream);
  } else {
    // chunks of iterations between host checks: the first spans as many
    // iterations as the previous solve needed, later ones check_every each;
    // a chunk is a cached graph (graph_chunks) or plain launches. With
    // profiling, a chunk of fused passes (Lanczos launches only) stays a
    // graph and is timed as a whole, so that the time per launch is the
    // kernels' own; other schedules are timed launch by launch
    const bool use_graphs = h->opt.graph_chunks && (!h->prof.on || fuse);
    auto launch_chunk = [&](int j0, int len) -> rexi_status {
      if (!use_graphs) {
        for (int q = j0; q < j0 + len; ++q) iteration(q, stream);
        HIPCHK(h, hipGetLastError());
        return REXI_OK;
      }
      hipGraphExec_t exec = nullptr;
      for (auto& c : (*cx.chunks))
        if (c.j0 == j0 && c.len == len) exec = c.exec;
      if (!exec) {
        if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        ++h->prof.suspend;
        for (int q = j0; q < j0 + len; ++q) iteration(q, h->cap_stream);
        --h->prof.suspend;
        hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
        if (ec != hipSuccess) return fail(h, REXI_E_HIP, "chunk capture failed: %s", hipGetErrorString(ec));
        hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(h, REXI_E_HIP, "chunk instantiation failed: %s", hipGetErrorString(ei));
        if ((*cx.chunks).size() >= 64) {
          (void)hipGraphExecDestroy((*cx.chunks).front().exec);
          (*cx.chunks).erase((*cx.chunks).begin());
        }
        (*cx.chunks).push_back({j0, len, exec});
      }
      double cbytes = 0.0;
      for (int q = j0; q < j0 + len; ++q) cbytes += q + 1 < m ? n * lz_bytes(q + 1) : 0.0;
      Timed t(h, PC_LANCZOS, cbytes, stream, len);
      HIPCHK(h, hipGraphLaunch(exec, stream));
      return REXI_OK;
    };
    // the system states travel with every convergence check, so the check
    // that ends the solve also brings them (pinned buffer of one state per
    // instance, allocated at setup)
    if (h->hst_cap < S) return fail(h, REXI_E_INVALID_ARG, "internal: %d system states, room for %d", S, h->hst_cap);
    int j = 0;
    // two iterations past the previous solve's length: the count drifts by
    // one between steps, and iterations after convergence cost a launch each
    // (finished systems skip them) where one more check costs a round trip
    int len = (*cx.k_hint) > 0 ? (*cx.k_hint) + 2 : chunk;
    int passes = 0;
    if (fuse) plain_step(0, stream);
    while (j < m) {
      len = std::max(1, std::min(len, m - j));
      rexi_status rs = launch_chunk(j, len);
      if (rs != REXI_OK) return rs;
      // [0]: systems still iterating after the chunk's last iteration; [1]: pause
      HIPCHK(h, hipMemcpyAsync(h->hpin, W.counters + (j + len - 1), sizeof(int32_t), hipMemcpyDeviceToHost,
                               stream));
      HIPCHK(h, hipMemcpyAsync(h->hpin + 1, SWc.gpause, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
      HIPCHK(h, hipMemcpyAsync(h->hst, W.st, S * sizeof(SysState_t), hipMemcpyDeviceToHost, stream));
      HIPCHK(h, hipStreamSynchronize(stream));
      const int paused_at = pause_mode ? h->hpin[1] : -1;
      if (paused_at >= 0) {
        // second Gram-Schmidt pass of iteration paused_at, then go on after it
        hipLaunchKernelGGL(rexi::k_resume, dim3(S), dim3(64), 0, stream, W, SWc);
        second_pass(paused_at, stream, G);
        if (fuse && paused_at + 1 < m) plain_step(paused_at + 1, stream);
        HIPCHK(h, hipGetLastError());
        ++passes;
        j = paused_at + 1;
        // systems still iterating after iteration paused_at (its ends, the
        // second pass's included, count them)
        HIPCHK(h, hipMemcpyAsync(h->hpin, W.counters + paused_at, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        HIPCHK(h, hipMemcpyAsync(h->hst, W.st, S * sizeof(SysState_t), hipMemcpyDeviceToHost, stream));
        HIPCHK(h, hipStreamSynchronize(stream));
        if (h->hpin[0] == 0) break;
        len = std::max(chunk, (*cx.k_hint) - j);
        continue;
      }
      j += len;
      if (h->hpin[0] == 0) break;
      len = chunk;
    }
    // the next solve starts with one chunk of this solve's length (states
    // from the last check, taken after the last iteration launched)
    std::vector<SysState_t> sst(h->hst, h->hst + S);
    int kmax = 1;
    int64_t isum = 0;
    for (auto& x : sst) {
      kmax = std::max(kmax, x.kcyc);
      isum += x.its;
    }
    (*cx.k_hint) = kmax;
    (*cx.reorth_passes) = passes;
    if (sst_out) *sst_out = sst;
    if (its_sum) *its_sum = isum;
  }
  return REXI_OK;
}

template <typename T, int PPT>
rexi_status run_restarts(rexi_handle* h, double2* out, hipStream_t stream, bool wx);

// One shared-basis solve of all poles of every instance; writes the pole sums
// to out (out = nullptr: the solve only, its per-pole coefficients y_p).
template <typename T, int PPT>
rexi_status run_shifted(rexi_handle* h, ShiftCtx cx, const double2* b, double2* out, hipStream_t stream) {
  Solver& sv = *cx.sv;
  rexi::ShiftWork& SWc = *cx.SW;
  Work& W = sv.W;
  const int G = sv.grid, m = sv.m;
  h->rs_cycles = 0;
  h->rs_its = 0;
  // the forward solve of a step forms the pole solutions when asked (info or
  // keep_solutions); their residuals need psi, which an in-place step overwrites
  const bool wx = out && h->want_x && h->X && cx.SW == &h->SW;
  const double2* bref = b;
  if (wx && (const void*)b == (const void*)out) {
    HIPCHK(h, hipMemcpyAsync(h->xb, b, (size_t)h->N * sizeof(double2), hipMemcpyDeviceToDevice, stream));
    bref = h->xb;
  }
  rexi_status ps = shifted_pass<T, PPT>(h, cx, b, stream, &h->st0, nullptr);
  if (ps != REXI_OK) return ps;
  // restarts need the Galerkin iterate of the poles that missed their target;
  // a captured schedule runs capture_cycles - 1 restart cycles (predicated on
  // the device: an instance without missed poles finishes each at once)
  const int cap_restarts = h->syncfree ? std::max(0, h->opt.capture_cycles - 1) : 0;
  const bool restart = cx.finish == 1 && h->rs_ready && out && (!h->syncfree || cap_restarts > 0);
  {
    rexi::ShiftWork SWb = SWc;
    SWb.fom = restart ? 1 : 0;
    Timed t(h, PC_REDUCE, 0, stream);
    hipLaunchKernelGGL(rexi::k_shifted_backsub, dim3((SWc.K + rexi::NWAVE - 1) / rexi::NWAVE), dim3(TPB), 0,
                       stream, W, SWb);
  }
  if (wx) {
    // x_p = V y_p (the Galerkin iterate for poles that restart; per-pole
    // solves overwrite theirs)
    rexi_status fs = form_x<PPT>(h, SWc, nullptr, nullptr, stream);
    if (fs != REXI_OK) return fs;
    h->x_valid = true;
  }
  // poles that missed their target within the basis: restarts or per-pole
  // solves finish them (host checks only)
  std::vector<int> missed;
  h->fb_poles = 0;
  h->fb_cycles = 0;
  h->fb_its = 0;
  // a system that stopped before m iterations met every pole's target
  const bool per_pole = cx.finish == 2 && h->fb.ready;
  if ((restart || per_pole) && !h->syncfree && (*cx.k_hint) >= m) {
    std::vector<int32_t> its((size_t)SWc.K);
    HIPCHK(h, hipMemcpyAsync(its.data(), SWc.its, its.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    for (int p = 0; p < SWc.K; ++p)
      if (its[p] == 0) missed.push_back(p);
  }
  if (!out) return REXI_OK;
  const bool fb = per_pole && !missed.empty();
  const double2* fb_b = b;
  if (fb && (const void*)b == (const void*)out) {
    HIPCHK(h, hipMemcpyAsync(h->fb_rhs, b, (size_t)h->N * sizeof(double2), hipMemcpyDeviceToDevice, stream));
    fb_b = h->fb_rhs;
  }
  // per-pole solves: those poles are left out of z; restarts: they enter
  // with their Galerkin iterate
  rexi::ShiftWork SWz = SWc;
  SWz.fb_skip = fb ? 1 : 0;
  {
    Timed t(h, PC_REDUCE, 0, stream);
    hipLaunchKernelGGL(rexi::k_shifted_z, dim3(sv.S), dim3(TPB), 0, stream, W, SWz);
  }
  {
    // algorithmic bytes: k_s basis vectors read and psi_out written per point
    double cb = 0.0;
    for (int i = 0; i < sv.S; ++i)
      cb += (double)sv.hsys[(size_t)i].n *
            (16.0 * (h->syncfree || (int)h->st0.size() != sv.S ? m : h->st0[(size_t)i].kcyc) + 16.0);
    Timed t(h, PC_POLESUM, cb, stream);
    hipLaunchKernelGGL((rexi::k_combine_out<T, PPT>), dim3(G), dim3(TPB), 0, stream, W, SWc, out, 0);
  }
  HIPCHK(h, hipGetLastError());
  if (fb) {
    h->fb_poles = (int)missed.size();
    rexi_status rs = run_fallback(h, missed, fb_b, out, stream);
    if (rs != REXI_OK) return rs;
  }
  if (restart && (h->syncfree || !missed.empty())) {
    h->fb_poles = (int)missed.size();
    rexi_status rs = run_restarts<T, PPT>(h, out, stream, wx);
    if (rs != REXI_OK) return rs;
  }
  if (wx && h->want_res) return explicit_residuals<PPT>(h, bref, stream);
  return REXI_OK;
}

// Restart cycles on the shared basis (single forward solver). After a cycle
// on right-hand side b, a pole that missed its target has the Galerkin
// iterate of the basis, with residual gnext_p u_k: the residuals of all such
// poles of an instance are multiples of u_k. The next cycle solves on
// b' = u_k for those poles only, pole p with weight w_p gam_p (gam_p the
// product of its gnext over the cycles) and target tol_p ||psi|| / |gam_p|,
// and adds its sums to out. Instances with no such pole have b' = 0.
template <typename T, int PPT>
rexi_status run_restarts(rexi_handle* h, double2* out, hipStream_t stream, bool wx) {
  Solver& sv = h->fwd;
  Work& W = sv.W;
  const int S = sv.S, G = sv.grid;
  const rexi::ShiftWork& R = h->SWR;
  hipLaunchKernelGGL(rexi::k_rs_begin, dim3(S), dim3(TPB), 0, stream, W, h->SW, h->rs_miss, h->rs_gam, h->rs_bn0,
                     h->rs_kbase, h->rs_hasmiss);
  hipLaunchKernelGGL(rexi::k_rs_rhs, dim3(G), dim3(TPB), 0, stream, W, h->rs_hasmiss, h->rs_rhs);
  HIPCHK(h, hipGetLastError());
  std::vector<int32_t> hm((size_t)S);
  std::vector<SysState_t> cst;
  // a captured step: a fixed number of cycles, no host reads
  const int ncyc = h->syncfree ? std::max(0, h->opt.capture_cycles - 1) : std::max(1, h->opt.max_cycles);
  for (int c = 1; c <= ncyc; ++c) {
    int64_t isum = 0;
    rexi_status ps = shifted_pass<T, PPT>(h, rs_ctx(h), h->rs_rhs, stream, &cst, &isum);
    if (ps != REXI_OK) return ps;
    h->rs_cycles = c;
    h->rs_its += isum;
    {
      Timed t(h, PC_REDUCE, 0, stream);
      hipLaunchKernelGGL(rexi::k_shifted_backsub, dim3((R.K + rexi::NWAVE - 1) / rexi::NWAVE), dim3(TPB), 0,
                         stream, W, R);
      hipLaunchKernelGGL(rexi::k_shifted_z, dim3(S), dim3(TPB), 0, stream, W, R);
    }
    {
      // k_s vectors read, psi_out read and written per point
      double cb = 0.0;
      for (int i = 0; i < S; ++i)
        cb += (double)sv.hsys[(size_t)i].n * (16.0 * ((int)cst.size() == S ? cst[(size_t)i].kcyc : sv.m) + 32.0);
      Timed t(h, PC_POLESUM, cb, stream);
      hipLaunchKernelGGL((rexi::k_combine_out<T, PPT>), dim3(G), dim3(TPB), 0, stream, W, R, out, 1);
    }
    if (wx) {
      // x_p += gam_p V' y'_p for the poles of this cycle (gam before the merge)
      rexi_status fs = form_x<PPT>(h, R, h->rs_gam, h->rs_miss, stream);
      if (fs != REXI_OK) return fs;
    }
    hipLaunchKernelGGL(rexi::k_rs_merge, dim3(S), dim3(TPB), 0, stream, W, h->SW, R, h->rs_miss, h->rs_gam,
                       h->rs_bn0, h->rs_kbase, h->rs_hasmiss);
    HIPCHK(h, hipGetLastError());
    if (h->syncfree) {
      if (c < ncyc)
        hipLaunchKernelGGL(rexi::k_rs_rhs, dim3(G), dim3(TPB), 0, stream, W, h->rs_hasmiss, h->rs_rhs);
      continue;
    }
    HIPCHK(h, hipMemcpyAsync(hm.data(), h->rs_hasmiss, S * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    bool any = false;
    for (int32_t v : hm) any = any || v != 0;
    if (!any) break;
    hipLaunchKernelGGL(rexi::k_rs_rhs, dim3(G), dim3(TPB), 0, stream, W, h->rs_hasmiss, h->rs_rhs);
    HIPCHK(h, hipGetLastError());
  }
  return REXI_OK;
}

rexi_status shifted_solve(rexi_handle* h, ShiftCtx cx, const double2* b, double2* out, hipStream_t stream) {
  switch (cx.sv->ppt) {
    case 8: return run_shifted<double2, 8>(h, cx, b, out, stream);
    case 4: return run_shifted<double2, 4>(h, cx, b, out, stream);
    case 2: return run_shifted<double2, 2>(h, cx, b, out, stream);
  }
  return fail(h, REXI_E_INVALID_ARG, "unsupported tiling");
}

rexi_status shifted_step(rexi_handle* h, const double2* b, double2* out, hipStream_t stream) {
  if (!h->fem_shared) return shifted_solve(h, fwd_ctx(h), b, out, stream);
  // Q1 elements: (A - s M)^-1 M psi = L^-T (Ahat - s)^-1 L^T psi, summed over
  // the poles on the transformed vector, then one L^-T for the whole sum
  const InstDesc& in = h->hinst[0];
  const dim3 gs(std::max(1, std::min((in.n + TPB - 1) / TPB, 2048)));
  hipLaunchKernelGGL(rexi::k_fem_lt, gs, dim3(TPB), 0, stream, in, h->chol, b, h->mrhs);
  HIPCHK(h, hipGetLastError());
  rexi_status st = shifted_solve(h, fwd_ctx(h), h->mrhs, out, stream);
  if (st != REXI_OK) return st;
  // L^-T of the sum: out -> y -> z -> out
  fem_sweep(h, out, h->fem_y, 0, 1, stream);
  fem_sweep(h, h->fem_y, h->fem_z, 1, 1, stream);
  fem_sweep(h, h->fem_z, out, 2, 1, stream);
  HIPCHK(h, hipGetLastError());
  return REXI_OK;
}

// out = sum_p w_p y_p of a finished shared-basis solve (every pole converged).
rexi_status shifted_combine(rexi_handle* h, ShiftCtx cx, double2* out, hipStream_t stream) {
  Solver& sv = *cx.sv;
  Timed t(h, PC_POLESUM, 0, stream);
  hipLaunchKernelGGL(rexi::k_shifted_z, dim3(sv.S), dim3(TPB), 0, stream, sv.W, *cx.SW);
  switch (sv.ppt) {
    case 8: hipLaunchKernelGGL((rexi::k_combine_out<double2, 8>), dim3(sv.grid), dim3(TPB), 0, stream, sv.W, *cx.SW, out, 0); break;
    case 4: hipLaunchKernelGGL((rexi::k_combine_out<double2, 4>), dim3(sv.grid), dim3(TPB), 0, stream, sv.W, *cx.SW, out, 0); break;
    default: hipLaunchKernelGGL((rexi::k_combine_out<double2, 2>), dim3(sv.grid), dim3(TPB), 0, stream, sv.W, *cx.SW, out, 0); break;
  }
  HIPCHK(h, hipGetLastError());
  return REXI_OK;
}

// Shared-basis adjoint step (single instance). REXI_E_NOT_BUILT when it does
// not apply (a pole missed its target within the basis, or no room for the
// second basis): the caller then takes the per-pole solves; nothing has been
// written then.
rexi_status shifted_adjoint(rexi_handle* h, const double2* psi_n, const double2* gbar_next, double2* gbar_n,
                            double* dV, hipStream_t st) {
  if (!h->fwdA.ready) {
    std::string keep = h->err;
    rexi_status s0 = init_shifted(h, h->fwdA, h->SWA, true, st);
    if (s0 == REXI_E_NO_MEMORY) {
      h->err = keep;
      return REXI_E_NOT_BUILT;
    }
    if (s0 != REXI_OK) return s0;
    // the forward solver's tiling and Lanczos pass
    if ((s0 = apply_tiling(h, h->fwdA, h->fwd.ppt, h->fwd.grid, st, &h->SWA)) != REXI_OK) return s0;
    if ((s0 = apply_columns(h, h->fwdA, h->fwd.col_kh, h->fwd.col_L, st, &h->SWA)) != REXI_OK) return s0;
    if (hipMalloc(&h->adj_coef, (size_t)h->fwd.m * h->fwd.m * sizeof(double2)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, REXI_E_NO_MEMORY, "adjoint coefficients");
    }
  }
  ShiftCtx cf = fwd_ctx(h);
  cf.finish = 0;
  rexi_status s1 = shifted_solve(h, cf, psi_n, nullptr, st);
  if (s1 != REXI_OK) return s1;
  s1 = shifted_solve(h, adj_ctx(h), gbar_next, nullptr, st);
  if (s1 != REXI_OK) return s1;
  const int K = h->SW.K;
  std::vector<int32_t> itf((size_t)K), ita((size_t)K);
  HIPCHK(h, hipMemcpyAsync(itf.data(), h->SW.its, K * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipMemcpyAsync(ita.data(), h->SWA.its, K * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  for (int p = 0; p < K; ++p)
    if (itf[p] == 0 || ita[p] == 0) return REXI_E_NOT_BUILT;
  if (dV) {
    const int ldc = h->fwd.m;
    Timed t(h, PC_GRAD, 0, st);
    hipLaunchKernelGGL(rexi::k_adj_coef, dim3(h->fwdA.m), dim3(TPB), 0, st, h->fwd.W, h->SW, h->fwdA.W, h->SWA,
                       h->adj_coef, ldc);
    hipLaunchKernelGGL((rexi::k_adj_grad<16>), dim3(std::min(2048, (int)((h->N + TPB - 1) / TPB))), dim3(TPB), 0,
                       st, h->fwd.W, h->fwdA.W, h->adj_coef, ldc, dV);
    HIPCHK(h, hipGetLastError());
  }
  // gbar_n = sum_p conj(w_p) y_p: the combination of the conjugate-shift solve
  return shifted_combine(h, adj_ctx(h), gbar_n, st);
}


// ---------------------------------------------------------------- autotuner
// Candidate tilings (points per thread) and grid sizes are timed on short
// real runs of the solver (start + a few iterations on a synthetic
// right-hand side) with HIP events; the fastest is kept. Results are cached
// per problem shape for the life of the process and, when REXI_TUNE_CACHE
// names a file, across processes.
struct TuneKey {
  std::string key;
  int ppt, grid;
  int kh, L;  // fused Lanczos pass: 0 row-staged, else marching slots and planes
};
// The cache is shared by every handle of the process: tune_mutex guards it
// (and the file named by REXI_TUNE_CACHE).
std::vector<TuneKey>& tune_cache() {
  static std::vector<TuneKey> c;
  return c;
}
std::mutex& tune_mutex() {
  static std::mutex mu;
  return mu;
}

std::string tune_key(const rexi_handle* h, const Solver& sv) {
  char buf[160];
  std::string k = h->shifted ? "shifted" : "perpole";
  snprintf(buf, sizeof buf, "|p%d|S%d|m%d|", sv.prec, sv.S, sv.m);
  k += buf;
  size_t cnt = 0;
  for (auto& d : sv.hsys) {
    if (cnt++ > 64) break;  // long batches: the first instances identify them
    snprintf(buf, sizeof buf, "%dx%dx%d,", d.n0, d.n1, d.n2);
    k += buf;
  }
  return k;
}

// (callers hold tune_mutex)
void tune_cache_load() {
  static bool loaded = false;
  if (loaded) return;
  loaded = true;
  const char* f = getenv("REXI_TUNE_CACHE");
  if (!f) return;
  FILE* fp = fopen(f, "r");
  if (!fp) return;
  char line[4096];
  while (fgets(line, sizeof line, fp)) {
    char key[4000];
    int ppt, grid, kh = 0, L = 0;
    if (sscanf(line, "%3999s %d %d %d %d", key, &ppt, &grid, &kh, &L) >= 3)
      tune_cache().push_back({key, ppt, grid, kh, L});
  }
  fclose(fp);
}

void tune_cache_store(const std::string& key, int ppt, int grid, int kh, int L) {
  std::lock_guard<std::mutex> lock(tune_mutex());
  tune_cache().push_back({key, ppt, grid, kh, L});
  const char* f = getenv("REXI_TUNE_CACHE");
  if (!f) return;
  FILE* fp = fopen(f, "a");
  if (!fp) return;
  fprintf(fp, "%s %d %d %d %d\n", key.c_str(), ppt, grid, kh, L);
  fclose(fp);
}

rexi_status apply_tiling(rexi_handle* h, Solver& sv, int ppt, int grid, hipStream_t stream,
                         rexi::ShiftWork* SWp) {
  sv.ppt = ppt;
  sv.tile = TPB * ppt;
  if (h->shifted) set_row_planes(h, sv, 0);  // the column plan is dropped below
  layout_systems(sv, sv.m);
  sv.grid = grid;
  sv.W.total_tiles = sv.total_tiles;
  sv.W.tile = sv.tile;
  sv.W.ilv = sv.ilv ? ilog2(sv.tile) : 0;
  HIPCHK(h, hipMemcpyAsync(sv.dsys, sv.hsys.data(), sv.S * sizeof(SysDesc), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipMemcpyAsync(sv.dtile, sv.htile.data(), (sv.S + 1) * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipStreamSynchronize(stream));
  rexi_status ts = upload_tile_sys(h, sv, stream);
  if (ts != REXI_OK) return ts;
  sv.col_kh = 0;  // a new tiling invalidates the column plan
  if (h->shifted) {
    rexi::ShiftWork& SW = SWp ? *SWp : h->SW;
    SW.col_start = nullptr;
    SW.col_sys = nullptr;
    SW.col_total = 0;
  }
  return REXI_OK;
}

// Select the fused Lanczos pass: kh = 0 the row-staged pass, else the
// marching pass with kh slots and L planes per item. REXI_OK with the
// row-staged pass when the plan does not fit.
// Geometry of the shared-basis systems: as the instance describes it (mode
// 0), or, for the marching passes, a 2D instance (1, ny, nx) relabelled with
// its rows as the planes: (ny, nx, 1) for the row-band pass (mode 1), whose
// band is then a run of a row's points, or (ny, 1, nx) for the tiled pass
// (mode 2), whose tiles are then strips of a row. The C-order layout is the
// same, so only the roles change; the stencil sums are the same, term for term.
void set_row_planes(rexi_handle* h, Solver& sv, int mode) {
  for (auto& d : sv.hsys) {
    const InstDesc& in = h->hinst[d.inst];
    const bool rp = mode != 0 && in.n0 == 1 && in.n1 > 1 && in.n2 > 1 && !in.fem;
    const bool strip = rp && mode == 2;
    d.n0 = rp ? in.n1 : in.n0;
    d.n1 = rp ? (strip ? 1 : in.n2) : in.n1;
    d.n2 = rp ? (strip ? in.n2 : 1) : in.n2;
    d.d1 = rp ? rexi::make_fastdiv((uint32_t)d.n1) : in.d1;
    d.d2 = rp ? rexi::make_fastdiv((uint32_t)d.n2) : in.d2;
    d.c0 = rp ? in.c1 : in.c0;
    d.c1 = rp ? (strip ? 0.0 : in.c2) : in.c1;
    d.c2 = rp ? (strip ? in.c2 : 0.0) : in.c2;
  }
}

// every system is a 2D instance (the tiled pass takes strips of its rows)
bool all_2d(rexi_handle* h, const Solver& sv) {
  for (auto& d : sv.hsys) {
    const InstDesc& in = h->hinst[d.inst];
    if (!(in.n0 == 1 && in.n1 > 1 && in.n2 > 1 && !in.fem)) return false;
  }
  return !sv.hsys.empty();
}

rexi_status apply_columns(rexi_handle* h, Solver& sv, int kh, int L, hipStream_t stream,
                          rexi::ShiftWork* SWp) {
  rexi::ShiftWork& SW = SWp ? *SWp : h->SW;
  sv.col_kh = 0;
  SW.col_start = nullptr;
  SW.col_sys = nullptr;
  SW.col_total = 0;
  // the tiled pass keeps a 3D instance's geometry and takes strips of a 2D
  // instance's rows; the row-band pass marches over the rows of 2D instances
  const bool strip = kh == 2 && all_2d(h, sv);
  set_row_planes(h, sv, kh == 0 ? 0 : kh == 2 ? (strip ? 2 : 0) : 1);
  if (kh == 0 || !plan_columns(sv, kh, L, strip)) {
    set_row_planes(h, sv, 0);
    HIPCHK(h, hipMemcpyAsync(sv.dsys, sv.hsys.data(), sv.S * sizeof(SysDesc), hipMemcpyHostToDevice, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    return REXI_OK;
  }
  HIPCHK(h, hipMemcpyAsync(sv.dsys, sv.hsys.data(), sv.S * sizeof(SysDesc), hipMemcpyHostToDevice, stream));
  HIPCHK(h, hipMemcpyAsync(sv.dcol, sv.hcol.data(), (sv.S + 1) * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  std::vector<int32_t> csys;
  if (sv.dcolsys && sv.col_total <= sv.colsys_cap) {
    csys.resize((size_t)sv.col_total);
    for (int q = 0; q < sv.S; ++q)
      for (int it = sv.hcol[q]; it < sv.hcol[q + 1]; ++it) csys[it] = q;
    HIPCHK(h, hipMemcpyAsync(sv.dcolsys, csys.data(), csys.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  }
  HIPCHK(h, hipStreamSynchronize(stream));
  SW.col_start = sv.dcol;
  SW.col_sys = csys.empty() ? nullptr : sv.dcolsys;
  SW.col_total = sv.col_total;
  return REXI_OK;
}

__global__ void k_tune_rhs(double2* __restrict__ v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double x = (double)(i % 9973) * 0.0137;
    v[i] = make_double2(sin(x) + 0.5, cos(1.7 * x));
  }
}

template <typename T, int PPT>
void tune_launch(rexi_handle* h, Solver& sv, const double2* b, int iters, hipStream_t st, bool fused = false) {
  Work& W = sv.W;
  const int G = sv.grid, S = sv.S;
  hipLaunchKernelGGL((rexi::k_start<T, PPT>), dim3(G), dim3(TPB), 0, st, W, b, b);
  hipLaunchKernelGGL(rexi::k_start_reduce, dim3(S), dim3(TPB), 0, st, W);
  if (h->shifted) hipLaunchKernelGGL(rexi::k_shifted_init, dim3(S), dim3(TPB), 0, st, W, h->SW);
  const bool lz = h->shifted && h->SW.lanczos;
  if (h->shifted && h->opt.lanczos == 1) {
    hipLaunchKernelGGL((rexi::k_lz_matvec<PPT>), dim3(G), dim3(TPB), 0, st, W, h->SW, 0, sv.col_kh == 2 ? -1 : 0, 0);
    hipLaunchKernelGGL(rexi::k_lz_start, dim3(S), dim3(TPB), 0, st, W, h->SW);
    if (fused && sv.col_kh) {
      // the solve's own schedule: a plain pass, then one fused launch per
      // iteration (each also ends the previous iteration)
      rexi::ShiftWork SWp = h->SW;
      SWp.pause_mode = 1;
      launch_lz_step<PPT>(sv, W, SWp, 0, st);
      for (int j = 1; j < iters && j < sv.m; ++j) launch_lz_step<PPT>(sv, W, SWp, j, st, true);
      return;
    }
    for (int j = 0; j < iters && j < sv.m; ++j) {
      launch_lz_step<PPT>(sv, W, h->SW, j, st);
      hipLaunchKernelGGL(rexi::k_lz_end, dim3(S), dim3(TPB), 0, st, W, h->SW, j, sv.col_kh ? 1 : 0);
    }
    return;
  }
  for (int j = 0; j < iters && j < sv.m; ++j) {
    const int i0 = lz ? std::max(0, j - 1) : 0;
    hipLaunchKernelGGL((rexi::k_arnoldi_a<T, PPT, true>), dim3(G), dim3(TPB), 0, st, W, j, i0, 0);
    hipLaunchKernelGGL(rexi::k_reduce_dots, dim3(S, j + 2), dim3(TPB), 0, st, W, j, 0, i0);
    hipLaunchKernelGGL((rexi::k_arnoldi_b<T, PPT>), dim3(G), dim3(TPB), 0, st, W, j, 0, i0);
    hipLaunchKernelGGL(rexi::k_end_iter, dim3(S), dim3(TPB), 0, st, W, h->shifted ? h->SW : h->noshift, j, 0, 0);
  }
}

rexi_status autotune(rexi_handle* h, Solver& sv, hipStream_t stream) {
  const std::string key = tune_key(h, sv);
  const bool march = h->shifted && h->opt.lanczos == 1 && h->opt.march_planes == 0;
  bool found = false;
  TuneKey hit{};
  {
    std::lock_guard<std::mutex> lock(tune_mutex());
    tune_cache_load();
    for (auto& c : tune_cache())
      if (c.key == key) {
        hit = c;
        found = true;
        break;
      }
  }
  if (found) {
    rexi_status st = apply_tiling(h, sv, hit.ppt, hit.grid, stream);
    if (st == REXI_OK && march) st = apply_columns(h, sv, hit.kh, hit.L, stream);
    return st;
  }
  double2* rhs = nullptr;
  if (hipMalloc(&rhs, (size_t)h->N * sizeof(double2)) != hipSuccess) {
    (void)hipGetLastError();
    return REXI_OK;  // no room to tune: keep the default tiling
  }
  hipLaunchKernelGGL(k_tune_rhs, dim3(1024), dim3(TPB), 0, stream, rhs, h->N);
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  const int iters = h->shifted ? 4 : 3;
  int best_ppt = sv.ppt, best_grid = sv.grid;
  float best = 1e30f;
  int64_t pts = 0;
  for (auto& d : sv.hsys) pts += d.n;
  for (int ppt : {8, 4, 2}) {
    const int tiles = (int)std::min<int64_t>((pts + TPB * ppt - 1) / (TPB * ppt) + sv.S, 1 << 30);
    for (int gmul : {1, 2, 4, 8}) {
      const int grid = std::max(1, std::min(tiles, 256 * gmul));
      if (gmul > 1 && grid == std::min(tiles, 256 * gmul / 2)) continue;  // same as a smaller candidate
      if (apply_tiling(h, sv, ppt, grid, stream) != REXI_OK) break;
      float tmin = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HIPCHK(h, hipEventRecord(e0, stream));
        switch (ppt * 2 + sv.prec) {
          case 16: tune_launch<double2, 8>(h, sv, rhs, iters, stream); break;
          case 17: tune_launch<float2, 8>(h, sv, rhs, iters, stream); break;
          case 8: tune_launch<double2, 4>(h, sv, rhs, iters, stream); break;
          case 9: tune_launch<float2, 4>(h, sv, rhs, iters, stream); break;
          case 4: tune_launch<double2, 2>(h, sv, rhs, iters, stream); break;
          case 5: tune_launch<float2, 2>(h, sv, rhs, iters, stream); break;
        }
        HIPCHK(h, hipEventRecord(e1, stream));
        HIPCHK(h, hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
        tmin = std::min(tmin, ms);
      }
      if (tmin < 0.97f * best) {
        best = tmin;
        best_ppt = ppt;
        best_grid = grid;
      }
    }
  }
  rexi_status st = apply_tiling(h, sv, best_ppt, best_grid, stream);
  // second stage (pipelined Lanczos): the row-staged pass against the
  // marching and tiled passes over slots x planes per item, on the chosen
  // tiling. Each candidate runs the solve's own schedule (fused launches
  // where the pass has them) for 24 iterations, five times after a warm-up
  // run; the median decides, and a later candidate must be 2% faster
  int best_kh = 0, best_L = 0;
  if (st == REXI_OK && march) {
    best = 1e30f;
    const int lz_iters = std::min(24, sv.m);
    for (int kh : {0, 3, 5, 8, 2}) {
      for (int L : {4, 8, 16}) {
        if (kh == 0 && L != 4) continue;
        if ((st = apply_columns(h, sv, kh, L, stream)) != REXI_OK) break;
        if (sv.col_kh != kh) continue;  // the plan does not fit
        std::vector<float> tr;
        for (int rep = 0; rep < 6; ++rep) {
          HIPCHK(h, hipEventRecord(e0, stream));
          switch (best_ppt) {
            case 8: tune_launch<double2, 8>(h, sv, rhs, lz_iters, stream, true); break;
            case 4: tune_launch<double2, 4>(h, sv, rhs, lz_iters, stream, true); break;
            default: tune_launch<double2, 2>(h, sv, rhs, lz_iters, stream, true); break;
          }
          HIPCHK(h, hipEventRecord(e1, stream));
          HIPCHK(h, hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) tr.push_back(ms);  // the first run warms the caches and code
        }
        std::sort(tr.begin(), tr.end());
        const float tmed = tr[tr.size() / 2];
        if (tmed < 0.98f * best) {
          best = tmed;
          best_kh = kh;
          best_L = L;
        }
      }
      if (st != REXI_OK) break;
    }
    if (st == REXI_OK) st = apply_columns(h, sv, best_kh, best_L, stream);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(rhs);
  if (st == REXI_OK) tune_cache_store(key, best_ppt, best_grid, best_kh, best_L);
  return st;
}

InstDesc make_inst(const rexi_grid& g, double hbar, double mass, int64_t off, bool fem) {
  InstDesc in{};
  int64_t n[3] = {1, 1, 1};
  double hh[3] = {1, 1, 1};
  const int nd = g.ndim;
  for (int a = 0; a < nd; ++a) {
    n[3 - nd + a] = g.n[a];
    hh[3 - nd + a] = (g.hi[a] - g.lo[a]) / (double)(g.n[a] + 1);
  }
  in.off = off;
  in.n0 = (int)n[0];
  in.n1 = (int)n[1];
  in.n2 = (int)n[2];
  in.n = (int)(n[0] * n[1] * n[2]);
  in.d2 = rexi::make_fastdiv((uint32_t)in.n2);
  in.d1 = rexi::make_fastdiv((uint32_t)in.n1);
  const double k = hbar * hbar / (2.0 * mass);
  double c[3];
  for (int a = 0; a < 3; ++a) c[a] = (3 - nd <= a) ? k / (hh[a] * hh[a]) : 0.0;
  in.c0 = c[0];
  in.c1 = c[1];
  in.c2 = c[2];
  in.diag = 2.0 * (c[0] + c[1] + c[2]);
  // Q1 elements: 1D mass (h/6) tridiag(1, 4, 1), stiffness (hbar^2/2m)(1/h)
  // tridiag(-1, 2, -1); an absent (padded) axis contributes the identity
  in.fem = fem ? 1 : 0;
  in.fvol = 1.0;
  for (int a = 0; a < 3; ++a) {
    const bool present = 3 - nd <= a;
    in.fmd[a] = present ? 4.0 * hh[a] / 6.0 : 1.0;
    in.fmo[a] = present ? hh[a] / 6.0 : 0.0;
    in.fkd[a] = present ? 2.0 * k / hh[a] : 0.0;
    in.fko[a] = present ? -k / hh[a] : 0.0;
    if (present) in.fvol *= hh[a];
  }
  return in;
}

void copy_fem(SysDesc& d, const InstDesc& in) {
  d.fem = in.fem;
  for (int a = 0; a < 3; ++a) {
    d.fmd[a] = in.fmd[a];
    d.fmo[a] = in.fmo[a];
    d.fkd[a] = in.fkd[a];
    d.fko[a] = in.fko[a];
  }
  d.fvol = in.fvol;
}

rexi_status scratch_address(rexi_handle* h, void** out);
rexi_status init_solutions(rexi_handle* h, hipStream_t stream);

rexi_status setup_common(rexi_handle** out, int count, const rexi_grid* grids, const double* V_dev,
                         const double* hbar, const double* mass, const double* dt, const int32_t* K,
                         const rexi_c128* sigma, const rexi_c128* beta, const rexi_options* opt,
                         hipStream_t stream) {
  g_setup_error.clear();
  if (!out) return fail(nullptr, REXI_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (count < 1 || !grids || !V_dev || !hbar || !mass || !dt || !K || !sigma || !beta)
    return fail(nullptr, REXI_E_INVALID_ARG, "NULL argument or count < 1");
  rexi_options o;
  rexi_default_options(&o);
  if (opt) o = *opt;
  if (o.precision != REXI_PREC_C128 && o.precision != REXI_PREC_C64_REFINE)
    return fail(nullptr, REXI_E_INVALID_ARG, "unknown precision %d", o.precision);
  if (o.solver != REXI_SOLVER_PER_POLE && o.solver != REXI_SOLVER_SHIFTED)
    return fail(nullptr, REXI_E_INVALID_ARG, "unknown solver %d", o.solver);
  if (o.solver == REXI_SOLVER_SHIFTED && o.precision != REXI_PREC_C128)
    return fail(nullptr, REXI_E_INVALID_ARG, "the shared-basis solver runs in complex128 only");
  if (o.m < 1 || o.m > 256) return fail(nullptr, REXI_E_INVALID_ARG, "m must be in [1, 256] (got %d)", o.m);
  if (!(o.reorth_eta > 0.0 && o.reorth_eta < 1.0)) return fail(nullptr, REXI_E_INVALID_ARG, "reorth_eta in (0, 1)");
  if (o.max_cycles < 1 || o.max_cycles > 1000) return fail(nullptr, REXI_E_INVALID_ARG, "max_cycles out of range");
  if (!(o.tol > 0.0) || !is_fin(o.tol)) return fail(nullptr, REXI_E_INVALID_ARG, "tol must be positive");
  if (o.tol_policy != REXI_TOL_RELRES && o.tol_policy != REXI_TOL_CERTIFIED)
    return fail(nullptr, REXI_E_INVALID_ARG, "unknown tol_policy");
  if (o.reorth < 0 || o.reorth > 2) return fail(nullptr, REXI_E_INVALID_ARG, "reorth must be 0, 1 or 2");
  if (!(o.inner_rtol >= 0.0 && o.inner_rtol < 1.0)) return fail(nullptr, REXI_E_INVALID_ARG, "inner_rtol in [0,1)");
  if (o.max_workspace_bytes < 0) return fail(nullptr, REXI_E_INVALID_ARG, "max_workspace_bytes < 0");
  if (o.grid_blocks < 0) return fail(nullptr, REXI_E_INVALID_ARG, "grid_blocks < 0");
  if (o.tile != 0 && o.tile != 512 && o.tile != 1024 && o.tile != 2048)
    return fail(nullptr, REXI_E_INVALID_ARG, "tile must be 0 (tuned), 512, 1024 or 2048 points");
  if (o.march_planes < -1 || o.march_planes > 1024)
    return fail(nullptr, REXI_E_INVALID_ARG, "march_planes must be in [-1, 1024]");
  if (o.march_slots != 0 && o.march_slots != 2 && o.march_slots != 3 && o.march_slots != 5 && o.march_slots != 8)
    return fail(nullptr, REXI_E_INVALID_ARG, "march_slots must be 0, 2, 3, 5 or 8");
  if (o.fallback < 0 || o.fallback > 2) return fail(nullptr, REXI_E_INVALID_ARG, "fallback must be 0, 1 or 2");
  if (o.fallback_m < 1 || o.fallback_m > 256)
    return fail(nullptr, REXI_E_INVALID_ARG, "fallback_m must be in [1, 256]");
  if (o.fallback_bytes < 0) return fail(nullptr, REXI_E_INVALID_ARG, "fallback_bytes < 0");
  if (!(o.stab_eps >= 0.0 && o.stab_eps < 1.0)) return fail(nullptr, REXI_E_INVALID_ARG, "stab_eps must be in [0, 1)");
  if (o.center != 0 && o.center != 1) return fail(nullptr, REXI_E_INVALID_ARG, "center must be 0 or 1");
  if (o.adjoint_shared != 0 && o.adjoint_shared != 1)
    return fail(nullptr, REXI_E_INVALID_ARG, "adjoint_shared must be 0 or 1");
  if (o.capture_cycles < 0 || o.capture_cycles > 64)
    return fail(nullptr, REXI_E_INVALID_ARG, "capture_cycles must be in [0, 64]");
  if (o.capture_pauses < 0 || o.capture_pauses > 64)
    return fail(nullptr, REXI_E_INVALID_ARG, "capture_pauses must be in [0, 64]");
  if (o.keep_solutions != 0 && o.keep_solutions != 1)
    return fail(nullptr, REXI_E_INVALID_ARG, "keep_solutions must be 0 or 1");
  if (o.discretization != REXI_DISC_FD && o.discretization != REXI_DISC_FEM_Q1)
    return fail(nullptr, REXI_E_INVALID_ARG, "unknown discretization %d", o.discretization);
  if (o.discretization == REXI_DISC_FEM_Q1 && o.solver == REXI_SOLVER_SHIFTED && count != 1)
    return fail(nullptr, REXI_E_INVALID_ARG,
                "Q1 elements with the shared-basis solver take one instance; use the per-pole solver for batches");
  if (o.discretization == REXI_DISC_FEM_Q1 && o.solver == REXI_SOLVER_SHIFTED && o.fallback == 2)
    return fail(nullptr, REXI_E_INVALID_ARG, "Q1 elements with the shared-basis solver: fallback 0 or 1");

  // ---- validate the instances (host side, before any device work)
  int64_t N = 0, Ktot = 0;
  for (int i = 0; i < count; ++i) {
    const rexi_grid& g = grids[i];
    if (g.ndim < 1 || g.ndim > 3) return fail(nullptr, REXI_E_INVALID_ARG, "instance %d: ndim %d", i, g.ndim);
    int64_t np = 1;
    for (int a = 0; a < g.ndim; ++a) {
      if (g.n[a] < 1) return fail(nullptr, REXI_E_INVALID_ARG, "instance %d: n[%d] < 1", i, a);
      if (!(g.hi[a] > g.lo[a]) || !is_fin(g.lo[a]) || !is_fin(g.hi[a]))
        return fail(nullptr, REXI_E_INVALID_ARG, "instance %d: need finite lo < hi on axis %d", i, a);
      np *= g.n[a];
      if (np > (int64_t)1 << 30) return fail(nullptr, REXI_E_INVALID_ARG, "instance %d: more than 2^30 points", i);
    }
    if (!(hbar[i] > 0.0) || !is_fin(hbar[i])) return fail(nullptr, REXI_E_INVALID_ARG, "instance %d: hbar <= 0", i);
    if (!(mass[i] > 0.0) || !is_fin(mass[i])) return fail(nullptr, REXI_E_INVALID_ARG, "instance %d: mass <= 0", i);
    if (!(dt[i] != 0.0) || !is_fin(dt[i])) return fail(nullptr, REXI_E_INVALID_ARG, "instance %d: dt must be finite and nonzero", i);
    if (K[i] < 1 || K[i] > 4096) return fail(nullptr, REXI_E_INVALID_ARG, "instance %d: K = %d", i, K[i]);
    N += np;
    Ktot += K[i];
  }
  if (N > ((int64_t)1 << 31) - 1) return fail(nullptr, REXI_E_INVALID_ARG, "more than 2^31 - 1 points in total");
  for (int64_t k = 0; k < Ktot; ++k)
    if (!is_fin(sigma[k].re) || !is_fin(sigma[k].im) || !is_fin(beta[k].re) || !is_fin(beta[k].im))
      return fail(nullptr, REXI_E_INVALID_ARG, "pole %lld: non-finite sigma or beta", (long long)k);

  // V on the host: finiteness and the range of the spectrum bound
  std::vector<double> Vh((size_t)N);
  {
    hipError_t e = hipMemcpyAsync(Vh.data(), V_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(nullptr, REXI_E_HIP, "reading V failed: %s", hipGetErrorString(e));
  }
  for (int64_t i = 0; i < N; ++i)
    if (!is_fin(Vh[(size_t)i])) return fail(nullptr, REXI_E_INVALID_ARG, "V[%lld] is not finite", (long long)i);

  rexi_handle* h = new (std::nothrow) rexi_handle();
  if (!h) return fail(nullptr, REXI_E_NO_MEMORY, "host allocation failed");
  h->opt = o;
  h->ninst = count;
  h->N = N;
  // Q1 elements on the shared basis: the two-pass Lanczos process, whose
  // matvec is the operator Ahat applied outside the pass kernels
  h->fem_shared = o.discretization == REXI_DISC_FEM_Q1 && o.solver == REXI_SOLVER_SHIFTED;
  if (h->fem_shared) h->opt.lanczos = 2;
  int64_t off = 0, kk = 0;
  int itile = 0;
  const int itile_pts = INST_TILE;
  for (int i = 0; i < count; ++i) {
    const bool fem = o.discretization == REXI_DISC_FEM_Q1;
    InstDesc in = make_inst(grids[i], hbar[i], mass[i], off, fem);
    in.sys0 = (int)kk;
    in.nsys = K[i];
    in.tile0 = itile;
    in.ntiles = (in.n + itile_pts - 1) / itile_pts;
    h->hitile.push_back(itile);
    itile += in.ntiles;
    double vmin = Vh[(size_t)off], vmax = vmin;
    for (int64_t p = off; p < off + in.n; ++p) {
      vmin = std::min(vmin, Vh[(size_t)p]);
      vmax = std::max(vmax, Vh[(size_t)p]);
    }
    // spectrum bound of H: [min V, (hbar^2/2m) sum 4/h^2 + max V]; with
    // centering the solves use H - c I, c its midpoint, and the step is
    // multiplied by exp(-i dt c / hbar): exp(-i dt H / hbar) is unchanged
    // Q1 elements: a bound of the pencil (A, M) from Rayleigh quotients: the
    // kinetic part lies in [0, sum_a (hbar^2/2m) 12/h_a^2], the potential part
    // between V_min and V_max scaled by h^d / eig(M) in [1, 3^d]
    double blo = vmin, bhi = 2.0 * in.diag + vmax;
    double mmin = 1.0;  // smallest eigenvalue of M (Euclidean errors from M-norm ones)
    if (fem) {
      const double f = std::pow(3.0, (double)grids[i].ndim);
      blo = std::min(vmin, f * vmin);
      bhi = 6.0 * in.diag + std::max(vmax, f * vmax);  // 6 diag = sum (hbar^2/2m) 12/h^2
      for (int a = 0; a < 3; ++a) mmin *= (3 - grids[i].ndim <= a) ? in.fmd[a] / 2.0 : 1.0;  // h/3 per axis
      // the shared basis solves for xhat = L^T x: its residuals and errors are
      // those of x in the M-norm, relative to ||psi||_M = ||L^T psi||
      if (h->fem_shared) mmin = 1.0;
    }
    const double c = o.center ? 0.5 * (blo + bhi) : 0.0;
    const double lo = blo - c, hi = bhi - c;
    h->lam_lo.push_back(lo);
    h->lam_hi.push_back(hi);
    // finite differences shift the diagonal (H - c I); elements shift the poles (A - (s + c) M)
    h->center.push_back(fem ? 0.0 : c);
    const cplx phase = std::exp(cplx(0.0, -dt[i] * c / hbar[i])) * (1.0 - o.stab_eps);
    for (int k = 0; k < K[i]; ++k, ++kk) {
      // s_j = i hbar sigma_j / dt, w_j = i hbar beta_j / dt (eq. rational-evaluation, B = hbar I);
      // the centering phase and the stabilisation factor (Section 3.4) scale w_j
      const cplx I(0.0, 1.0);
      const cplx sg(sigma[kk].re, sigma[kk].im), bt(beta[kk].re, beta[kk].im);
      const cplx s = I * hbar[i] * sg / dt[i];
      const cplx w = phase * (I * hbar[i] * bt / dt[i]);
      const double re = std::min(std::max(s.real(), lo), hi);
      const double dist = std::abs(cplx(re, 0.0) - s);
      const double scale = std::max({std::fabs(lo), std::fabs(hi), std::abs(s), 1e-300});
      if (!(dist > 1e-13 * scale)) {
        destroy_handle(h);
        return fail(nullptr, REXI_E_INVALID_ARG,
                    "pole %lld: shift (%g, %g) lies on the spectrum bound [%g, %g] (singular system)",
                    (long long)kk, s.real(), s.imag(), lo, hi);
      }
      // floor of an attainable FP64 relative residual for this system
      const double u = 1.1102230246251565e-16;
      const double floor_r = 8.0 * u * (1.0 + std::max(std::abs(cplx(lo) - s), std::abs(cplx(hi) - s)) / dist);
      double tol = o.tol;
      if (o.tol_policy == REXI_TOL_CERTIFIED) {
        // sum_j |w_j| rho_j / dist_j <= tol when rho_j = tol dist_j / (K |w_j|)
        tol = o.tol * dist * mmin / ((double)K[i] * std::max(std::abs(w), 1e-300));
      }
      tol = std::max(tol, floor_r);
      h->s.push_back(fem ? s + c : s);
      h->w.push_back(w);
      h->tol_sys.push_back(tol);
      // Q1: ||x - x*|| <= ||r|| / (eig_min(M) dist) (norms of M and M^-1)
      h->dist_sys.push_back(dist * mmin);
    }
    h->Kinst.push_back(K[i]);
    h->hinst.push_back(in);
    off += in.n;
  }
  h->hitile.push_back(itile);
  h->itotal = itile;
  // Q1 shared basis: bidiagonal Cholesky factors of the 1D mass matrices
  // tridiag(fmo, fmd, fmo) of each axis (d_0 = sqrt(fmd), e_i = fmo / d_{i-1},
  // d_i = sqrt(fmd - e_i^2)); an absent axis has the factor 1. Per axis:
  // d, e and 1 / d, n_a entries each
  std::vector<double> chol;
  if (h->fem_shared) {
    InstDesc& in = h->hinst[0];
    const int na[3] = {in.n0, in.n1, in.n2};
    for (int a = 0; a < 3; ++a) {
      in.loff[a] = (int64_t)chol.size();
      std::vector<double> d((size_t)na[a]), e((size_t)na[a], 0.0);
      // rho: the largest factor by which a sweep step carries an error in v,
      // |e_i / d_i| forward (L^-1) and |e_{i+1} / d_i| backward (L^-T)
      double rho = 0.0;
      for (int i = 0; i < na[a]; ++i) {
        if (i > 0) e[i] = in.fmo[a] / d[i - 1];
        d[i] = std::sqrt(in.fmd[a] - e[i] * e[i]);
        rho = std::max(rho, std::fabs(e[i] / d[i]));
        if (i > 0) rho = std::max(rho, std::fabs(e[i] / d[i - 1]));
      }
      // warm-up of a segment: rho^warm <= 2^-64 (the whole line if rho is near 1)
      h->fem_warm[a] = rho > 0.0 && rho < 0.9 ? std::min(na[a], (int)std::ceil(-64.0 * std::log(2.0) / std::log(rho)))
                                              : (rho > 0.0 ? na[a] : 0);
      chol.insert(chol.end(), d.begin(), d.end());
      chol.insert(chol.end(), e.begin(), e.end());
      for (int i = 0; i < na[a]; ++i) chol.push_back(1.0 / d[(size_t)i]);  // reciprocal pivots of the sweeps
    }
  }

#define SETUP_CHK(call)                                                                             \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) {                                                                         \
      (void)hipGetLastError();                                                                      \
      rexi_status st_ = (e_ == hipErrorOutOfMemory) ? REXI_E_NO_MEMORY : REXI_E_HIP;                \
      fail(nullptr, st_, "%s failed: %s", #call, hipGetErrorString(e_));                            \
      destroy_handle(h);                                                                            \
      return st_;                                                                                   \
    }                                                                                               \
  } while (0)
  SETUP_CHK(hipMalloc(&h->V64, (size_t)N * sizeof(double)));
  SETUP_CHK(hipMemcpyAsync(h->V64, V_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, stream));
  // FP32 V: complex64 inner solves (also those finishing missed shared-basis poles)
  if (o.precision == REXI_PREC_C64_REFINE || (o.solver == REXI_SOLVER_SHIFTED && o.fallback == 2)) {
    SETUP_CHK(hipMalloc(&h->V32, (size_t)N * sizeof(float)));
    hipLaunchKernelGGL(rexi::k_v_to_f32, dim3(1024), dim3(TPB), 0, stream, h->V64, h->V32, (int64_t)N);
    SETUP_CHK(hipGetLastError());
  }
  SETUP_CHK(hipMalloc(&h->dinst, count * sizeof(InstDesc)));
  SETUP_CHK(hipMalloc(&h->ditile, (count + 1) * sizeof(int32_t)));
  SETUP_CHK(hipMalloc(&h->dnorm, std::max(1, itile) * sizeof(double)));
  if (o.discretization == REXI_DISC_FEM_Q1) SETUP_CHK(hipMalloc(&h->mrhs, (size_t)N * sizeof(double2)));
  if (h->fem_shared) {
    SETUP_CHK(hipMalloc(&h->chol, chol.size() * sizeof(double)));
    SETUP_CHK(hipMemcpyAsync(h->chol, chol.data(), chol.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    SETUP_CHK(hipMalloc(&h->fem_y, (size_t)N * sizeof(double2)));
    SETUP_CHK(hipMalloc(&h->fem_z, (size_t)N * sizeof(double2)));
  }
  SETUP_CHK(hipMemcpyAsync(h->dinst, h->hinst.data(), count * sizeof(InstDesc), hipMemcpyHostToDevice, stream));
  SETUP_CHK(hipMemcpyAsync(h->ditile, h->hitile.data(), (count + 1) * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  SETUP_CHK(hipHostMalloc((void**)&h->hpin, 64 * sizeof(int32_t), hipHostMallocDefault));
  // a shared-basis solve has one system per instance
  SETUP_CHK(hipHostMalloc((void**)&h->hst, (size_t)std::max(1, count) * sizeof(SysState_t), hipHostMallocDefault));
  h->hst_cap = std::max(1, count);
  SETUP_CHK(hipStreamSynchronize(stream));
  h->ws_bytes = (int64_t)N * (h->V32 ? 12 : 8);
  h->shifted = o.solver == REXI_SOLVER_SHIFTED;
  rexi_status st = h->shifted ? init_shifted(h, h->fwd, h->SW, false, stream) : init_solver(h, h->fwd, 1, stream);
  if (st != REXI_OK) {
    g_setup_error = h->err;
    destroy_handle(h);
    return st;
  }
  // (the tuner times the stencil passes, which the Q1 shared basis does not use)
  if (o.autotune && o.tile == 0 && o.grid_blocks == 0 && !h->fem_shared) st = autotune(h, h->fwd, stream);
  if (st == REXI_OK && h->shifted && h->opt.lanczos == 1 && o.march_planes > 0)
    st = apply_columns(h, h->fwd, o.march_slots ? o.march_slots : 5, o.march_planes, stream);
  if (st == REXI_OK && h->shifted && o.fallback == 2) st = init_fallback(h, stream);
  if (st == REXI_OK && h->shifted && o.fallback == 1) st = init_restart(h, stream);
  if (st == REXI_OK && h->shifted && !h->mrhs && !h->fem_shared) st = init_solutions(h, stream);
  if (st != REXI_OK) {
    g_setup_error = h->err;
    destroy_handle(h);
    return st;
  }
  h->prof.on = o.profile != 0;
  // the device address of the allocation-free entry point's workspace on
  // this device (once per device); a failure is reported by that entry point
  if (scratch_address(h, &h->scratch) != REXI_OK) {
    h->scratch = nullptr;
    h->err.clear();
  }
  *out = h;
  return REXI_OK;
#undef SETUP_CHK
}

__global__ void k_norm2_inst(const InstDesc* __restrict__ inst, int ninst, const int32_t* __restrict__ itile,
                             int itotal, const double2* __restrict__ v, double* __restrict__ part, int tile) {
  __shared__ double lds[rexi::NWAVE];
  for (int item = blockIdx.x; item < itotal; item += gridDim.x) {
    const int ii = rexi::find_sys(itile, ninst, item);
    const InstDesc& in = inst[ii];
    const int t = item - in.tile0;
    double acc = 0.0;
    for (int p = t * tile + threadIdx.x; p < std::min((t + 1) * tile, in.n); p += TPB) {
      const double2 a = v[in.off + p];
      acc += a.x * a.x + a.y * a.y;
    }
    acc = rexi::block_sum(acc, lds);
    if (threadIdx.x == 0) part[item] = acc;
  }
}

// ---------------------------------------------------------------- spectrum estimate
// Lanczos on H of every instance at once (real start vector, so the basis
// stays real): the vectors are the handle's global vectors, v_i at i * N.

// Start vector: a fixed pseudo-random real pattern (the instances are
// normalised separately afterwards).
__global__ void k_ev_start(double2* __restrict__ v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    const double u = (double)((z ^ (z >> 29)) >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
    v[i] = make_double2(u - 0.5, 0.0);
  }
}

// Per item of the instance tiling: partial <v_i, w> (real parts) for i < nvec,
// at part[i * itotal + item].
__global__ void k_ev_dots(const InstDesc* __restrict__ inst, int ninst, const int32_t* __restrict__ itile,
                          int itotal, const double2* __restrict__ basis, int64_t N, const double2* __restrict__ w,
                          int nvec, double* __restrict__ part, int tile) {
  __shared__ double lds[rexi::NWAVE];
  for (int item = blockIdx.x; item < itotal; item += gridDim.x) {
    const int ii = rexi::find_sys(itile, ninst, item);
    const InstDesc& in = inst[ii];
    const int t = item - in.tile0;
    const int pend = std::min((t + 1) * tile, in.n);
    for (int i = 0; i < nvec; ++i) {
      const double2* __restrict__ v = basis + (int64_t)i * N + in.off;
      double acc = 0.0;
      for (int p = t * tile + threadIdx.x; p < pend; p += TPB) {
        const double2 a = v[p], b = w[in.off + p];
        acc += a.x * b.x + a.y * b.y;
      }
      acc = rexi::block_sum(acc, lds);
      if (threadIdx.x == 0) part[(int64_t)i * itotal + item] = acc;
    }
  }
}

// w -= sum_{i < nvec} coef[ii * ldc + i] v_i on every instance ii.
__global__ void k_ev_update(const InstDesc* __restrict__ inst, int ninst, const int32_t* __restrict__ itile,
                            int itotal, const double2* __restrict__ basis, int64_t N, double2* __restrict__ w,
                            int nvec, const double* __restrict__ coef, int ldc, int tile) {
  for (int item = blockIdx.x; item < itotal; item += gridDim.x) {
    const int ii = rexi::find_sys(itile, ninst, item);
    const InstDesc& in = inst[ii];
    const int t = item - in.tile0;
    const int pend = std::min((t + 1) * tile, in.n);
    for (int p = t * tile + threadIdx.x; p < pend; p += TPB) {
      double2 a = w[in.off + p];
      for (int i = 0; i < nvec; ++i) {
        const double c = coef[(int64_t)ii * ldc + i];
        const double2 v = basis[(int64_t)i * N + in.off + p];
        a.x -= c * v.x;
        a.y -= c * v.y;
      }
      w[in.off + p] = a;
    }
  }
}

// v = scale[ii] w on every instance ii.
__global__ void k_ev_scale(const InstDesc* __restrict__ inst, int ninst, const int32_t* __restrict__ itile,
                           int itotal, const double2* __restrict__ w, double2* __restrict__ v,
                           const double* __restrict__ scale, int tile) {
  for (int item = blockIdx.x; item < itotal; item += gridDim.x) {
    const int ii = rexi::find_sys(itile, ninst, item);
    const InstDesc& in = inst[ii];
    const int t = item - in.tile0;
    const double c = scale[ii];
    const int pend = std::min((t + 1) * tile, in.n);
    for (int p = t * tile + threadIdx.x; p < pend; p += TPB) {
      const double2 a = w[in.off + p];
      v[in.off + p] = make_double2(c * a.x, c * a.y);
    }
  }
}

// Eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm count of
// the LDL^T pivots; b[i] couples rows i and i + 1).
int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double d = 1.0;
  const double tiny = 1e-300;
  for (size_t i = 0; i < a.size(); ++i) {
    const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = a[i] - x - (i > 0 ? off / d : 0.0);
    if (d == 0.0) d = -tiny;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// The r-th smallest eigenvalue (r = 0 .. k-1) of the tridiagonal by bisection
// inside its Gershgorin interval.
double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int r) {
  const size_t k = a.size();
  double lo = 0.0, hi = 0.0;
  for (size_t i = 0; i < k; ++i) {
    const double rad = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = i == 0 ? a[i] - rad : std::min(lo, a[i] - rad);
    hi = i == 0 ? a[i] + rad : std::max(hi, a[i] + rad);
  }
  for (int it = 0; it < 200 && hi - lo > 4e-16 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, mid) > r) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

rexi_status vec_norm(rexi_handle* h, const double2* v, hipStream_t stream, double* out) {
  const int tile = INST_TILE;
  hipLaunchKernelGGL(k_norm2_inst, dim3(std::min(h->itotal, 2048)), dim3(TPB), 0, stream, h->dinst, h->ninst,
                     h->ditile, h->itotal, v, h->dnorm, tile);
  HIPCHK(h, hipGetLastError());
  std::vector<double> part((size_t)h->itotal);
  HIPCHK(h, hipMemcpyAsync(part.data(), h->dnorm, part.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(h, hipStreamSynchronize(stream));
  double s = 0.0;
  for (double p : part) s += p;
  *out = std::sqrt(s);
  return REXI_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

void rexi_default_options(rexi_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->precision = REXI_PREC_C128;
  o->solver = REXI_SOLVER_PER_POLE;
  o->m = 30;
  o->max_cycles = 40;
  o->tol = 1e-10;
  o->tol_policy = REXI_TOL_RELRES;
  o->reorth = 1;
  o->reorth_eta = 1e-2;
  o->inner_rtol = 0.1;
  o->check_every = 4;
  o->lanczos = 1;
  o->capture_cycles = 0;
  o->graph_chunks = 1;
  o->autotune = 1;
  o->capture_safe = 0;
  o->profile = 0;
  o->tile = 0;
  o->grid_blocks = 0;
  o->max_workspace_bytes = 0;
  o->march_planes = 0;
  o->march_slots = 0;
  o->fallback = 1;
  o->fallback_m = 30;
  o->fallback_bytes = 0;
  o->stab_eps = 0.0;
  o->center = 0;
  o->discretization = REXI_DISC_FD;
  o->adjoint_shared = 1;
  o->keep_solutions = 0;
  o->capture_pauses = 0;
  o->reserved_opt2_ = 0;
}

rexi_status rexi_setup(rexi_handle** out, const rexi_grid* g, const double* V_dev, double hbar, double mass,
                       double dt, int32_t K, const rexi_c128* sigma_host, const rexi_c128* beta_host,
                       const rexi_options* opt, void* stream) {
  if (!g) return fail(nullptr, REXI_E_INVALID_ARG, "grid is NULL");
  return setup_common(out, 1, g, V_dev, &hbar, &mass, &dt, &K, sigma_host, beta_host, opt, (hipStream_t)stream);
}

rexi_status rexi_setup_batch(rexi_handle** out, int32_t count, const rexi_grid* grids, const double* V_dev,
                             const double* hbar, const double* mass, const double* dt, const int32_t* K,
                             const rexi_c128* sigma_host, const rexi_c128* beta_host, const rexi_options* opt,
                             void* stream) {
  return setup_common(out, count, grids, V_dev, hbar, mass, dt, K, sigma_host, beta_host, opt,
                      (hipStream_t)stream);
}

rexi_status rexi_apply_H(rexi_handle* h, const rexi_c128* x_dev, rexi_c128* y_dev, rexi_c128 shift, void* stream) {
  if (!h) return REXI_E_INVALID_ARG;
  if (!x_dev || !y_dev) return fail(h, REXI_E_INVALID_ARG, "NULL vector");
  if ((const void*)x_dev == (const void*)y_dev) return fail(h, REXI_E_INVALID_ARG, "x and y must not alias");
  if (!is_fin(shift.re) || !is_fin(shift.im)) return fail(h, REXI_E_INVALID_ARG, "non-finite shift");
  hipStream_t st = (hipStream_t)stream;
  Timed t(h, PC_APPLY_H, (double)h->N * 40.0, st);
  hipLaunchKernelGGL(rexi::k_apply_h, dim3(std::min(h->itotal, 2048)), dim3(TPB), 0, st, h->dinst, h->ninst,
                     h->ditile, h->itotal, h->V64, (const double2*)x_dev, (double2*)y_dev, shift.re, shift.im,
                     INST_TILE);
  HIPCHK(h, hipGetLastError());
  return REXI_OK;
}

rexi_status rexi_step(rexi_handle* h, const rexi_c128* psi_in, rexi_c128* psi_out, int32_t nsteps,
                      rexi_step_info* info, void* stream) {
  if (!h) return REXI_E_INVALID_ARG;
  if (!psi_in || !psi_out) return fail(h, REXI_E_INVALID_ARG, "NULL vector");
  if (nsteps < 1) return fail(h, REXI_E_INVALID_ARG, "nsteps must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  if (h->opt.capture_safe && !info && !h->syncfree) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(h, hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusActive) {
      // the caller is capturing: enqueue the fixed, read-free schedule into it
      h->syncfree = true;
      rexi_status r = rexi_step(h, psi_in, psi_out, nsteps, nullptr, stream);
      h->syncfree = false;
      return r;
    }
    // replay (or first capture) of a graph of the whole call on the caller's stream
    for (auto& g : h->graphs)
      if (g.in == psi_in && g.out == psi_out && g.nsteps == nsteps) {
        HIPCHK(h, hipGraphLaunch(g.exec, st));
        return REXI_OK;
      }
    if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    h->syncfree = true;
    rexi_status r = rexi_step(h, psi_in, psi_out, nsteps, nullptr, h->cap_stream);
    h->syncfree = false;
    hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
    if (r != REXI_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    if (ec != hipSuccess) return fail(h, REXI_E_HIP, "stream capture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(h, REXI_E_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    if (h->graphs.size() >= 4) {
      (void)hipGraphExecDestroy(h->graphs.front().exec);
      h->graphs.erase(h->graphs.begin());
    }
    h->graphs.push_back({psi_in, psi_out, nsteps, exec});
    HIPCHK(h, hipGraphLaunch(exec, st));
    return REXI_OK;
  }
  Solver& sv = h->fwd;
  const double2* in = (const double2*)psi_in;
  double2* outp = (double2*)psi_out;
  double norm_in = 0.0, fem_norm_in = 0.0;
  int64_t its_total = 0;
  int restarts = 0;
  for (int n = 0; n < nsteps; ++n) {
    const double2* src = n == 0 ? in : outp;
    if (h->shifted) {
      // Q1 elements: ||psi|| before an in-place step overwrites it (the
      // solves see ||L^T psi||, the M-norm)
      double psi_norm = 0.0;
      if (h->fem_shared && info && n == nsteps - 1) {
        rexi_status s0n = vec_norm(h, src, st, &psi_norm);
        if (s0n != REXI_OK) return s0n;
      }
      // the last step of a call with info forms the pole solutions and their
      // explicit residuals; keep_solutions forms the solutions every step
      h->want_res = info && n == nsteps - 1;
      h->want_x = h->opt.keep_solutions || h->want_res;
      h->x_valid = false;
      h->x_res = false;
      rexi_status s1 = shifted_step(h, src, outp, st);
      h->want_x = h->want_res = false;
      if (s1 != REXI_OK) return s1;
      if (info) {
        const int K = h->SW.K;
        std::vector<double> res((size_t)K);
        std::vector<int32_t> its((size_t)K);
        HIPCHK(h, hipMemcpyAsync(res.data(), h->SW.res, K * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipMemcpyAsync(its.data(), h->SW.its, K * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipStreamSynchronize(st));
        // the states of the first cycle (restart cycles reuse the system table)
        if ((int)h->st0.size() != sv.S) {
          h->st0.resize((size_t)sv.S);
          HIPCHK(h, hipMemcpyAsync(h->st0.data(), sv.W.st, sv.S * sizeof(SysState_t), hipMemcpyDeviceToHost, st));
          HIPCHK(h, hipStreamSynchronize(st));
        }
        const std::vector<SysState_t>& sst = h->st0;
        SysState_t s0 = sst[0];
        for (auto& x : sst) {
          its_total += x.its;
          s0.its = std::max(s0.its, x.its);
          s0.bnorm = std::max(s0.bnorm, x.bnorm);
        }
        its_total += h->fb_its + h->rs_its;
        const int more = h->fb_cycles + h->rs_cycles;
        if (n == nsteps - 1) {
          // explicit FP64 residuals of the formed solutions, relative to
          // ||psi|| of the pole's instance (implicit Givens estimates when
          // the solutions are not formed: Q1 elements, or no room for them)
          std::vector<double> rex;
          if (h->x_res) {
            std::vector<double> rn((size_t)K);
            HIPCHK(h, hipMemcpyAsync(rn.data(), h->xrn, K * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(h, hipStreamSynchronize(st));
            rex.resize((size_t)K);
            int q = 0;
            for (int i = 0; i < h->ninst; ++i)
              for (int k = 0; k < h->Kinst[i]; ++k, ++q) {
                const double bn = sst[(size_t)i].bnorm;
                rex[(size_t)q] = bn > 0.0 ? rn[(size_t)q] / bn : 0.0;
              }
          }
          const std::vector<double>& rr = h->x_res ? rex : res;
          info->K = K;
          info->max_cycles_used = 1 + more;
          info->not_converged = 0;
          info->max_rel_residual = 0.0;
          info->explicit_residuals = h->x_res ? 1 : 0;
          // per instance: sum_p |w_p| rho_p / dist_p bounds the relative step
          // error; the largest over the instances is reported
          // convergence is the solver's own test (the implicit residual against
          // the pole's target; near the FP64 floor the explicit residual of
          // the computed x_p may exceed a floored target by rounding); under
          // the certified policy an instance whose explicit certified sum
          // meets its plan has converged, whatever the share of each pole:
          // the plan is tol, or the sum of |w_p| rho_p* / dist_p over its
          // floored targets where the FP64 floors exceed tol
          std::vector<double> bound((size_t)h->ninst, 0.0), plan((size_t)h->ninst, 0.0);
          std::vector<int> miss((size_t)h->ninst, 0);
          int q = 0;
          for (int i = 0; i < h->ninst; ++i)
            for (int kk = 0; kk < h->Kinst[i]; ++kk, ++q) {
              const int k = q;
              if (!(res[k] <= h->tol_sys[k])) miss[(size_t)i] += 1;
              plan[(size_t)i] += std::abs(h->w[k]) * h->tol_sys[k] / h->dist_sys[k];
              info->max_rel_residual = std::max(info->max_rel_residual, rr[k]);
              bound[(size_t)i] += std::abs(h->w[k]) * rr[k] / h->dist_sys[k];
              if (info->iterations) info->iterations[k] = its[k] > 0 ? its[k] : s0.its;
              if (info->cycles) info->cycles[k] = its[k] > s0.its ? 1 + more : 1;
              if (info->rel_residual) info->rel_residual[k] = rr[k];
              if (info->implicit_residual) info->implicit_residual[k] = res[k];
            }
          for (int i = 0; i < h->ninst; ++i)
            if (!(h->opt.tol_policy == REXI_TOL_CERTIFIED &&
                  bound[(size_t)i] <= std::max(h->opt.tol, plan[(size_t)i])))
              info->not_converged += miss[(size_t)i];
          info->certified_bound = *std::max_element(bound.begin(), bound.end());
          info->reorth_passes = h->reorth_passes;
          // ||psi|| of the whole (packed) input
          double n2 = 0.0;
          for (const auto& x : sst) n2 += x.bnorm * x.bnorm;
          info->norm_in = h->fem_shared ? psi_norm : std::sqrt(n2);
          double no = 0.0;
          rexi_status s2 = vec_norm(h, outp, st, &no);
          if (s2 != REXI_OK) return s2;
          info->norm_out = no;
        }
      }
      if (!h->syncfree) prof_collect(h, st);
      continue;
    }
    const double2* rhs = src;
    if (h->mrhs && info && n == nsteps - 1) {
      // ||psi_n|| before the step overwrites it (in place)
      rexi_status s3 = vec_norm(h, src, st, &fem_norm_in);
      if (s3 != REXI_OK) return s3;
    }
    if (h->mrhs) {
      // Q1 elements: the systems are (A - s_j M) x_j = M psi
      hipLaunchKernelGGL(rexi::k_apply_mass, dim3(std::min(h->itotal, 2048)), dim3(TPB), 0, st, h->dinst,
                         h->ninst, h->ditile, h->itotal, src, h->mrhs, INST_TILE);
      rhs = h->mrhs;
    }
    rexi_status s1 = solve(h, sv, rhs, rhs, st, &restarts);
    if (s1 != REXI_OK) return s1;
    {
      Timed t(h, PC_POLESUM, (double)h->N * 16.0 * (1.0 + (double)sv.S / h->ninst), st);
      hipLaunchKernelGGL(rexi::k_polesum, dim3(std::min(h->itotal, 2048)), dim3(TPB), 0, st, h->dinst, h->ninst,
                         h->ditile, h->itotal, sv.dsys, sv.W.x, outp, INST_TILE, 0, 0);
    }
    HIPCHK(h, hipGetLastError());
    if (info) {
      std::vector<SysState_t> hs((size_t)sv.S);
      HIPCHK(h, hipMemcpyAsync(hs.data(), sv.W.st, sv.S * sizeof(SysState_t), hipMemcpyDeviceToHost, st));
      HIPCHK(h, hipStreamSynchronize(st));
      for (auto& x : hs) its_total += x.its;
      if (n == nsteps - 1) {
        info->K = sv.S;
        info->max_cycles_used = 0;
        info->not_converged = 0;
        info->max_rel_residual = 0.0;
        info->explicit_residuals = 1;  // every cycle ends with the explicit FP64 residual
        // per instance: the absolute bound sum_j |w_j| ||r_j|| / dist_j over
        // its poles, relative to its ||psi|| (Q1 elements: the right-hand side
        // is M psi, so relative to the whole input's norm); the largest is reported
        std::vector<double> bound((size_t)h->ninst, 0.0), bni((size_t)h->ninst, 0.0);
        for (int s = 0; s < sv.S; ++s) {
          const SysState_t& x = hs[(size_t)s];
          const int i = sv.hsys[(size_t)s].inst;
          info->max_cycles_used = std::max(info->max_cycles_used, x.cycles);
          if (!(x.rho <= sv.hsys[(size_t)s].tol)) info->not_converged += 1;
          info->max_rel_residual = std::max(info->max_rel_residual, x.rho);
          bound[(size_t)i] += std::abs(h->w[(size_t)s]) * x.rho * x.bnorm / h->dist_sys[(size_t)s];
          bni[(size_t)i] = x.bnorm;
          if (info->iterations) info->iterations[s] = x.its;
          if (info->cycles) info->cycles[s] = x.cycles;
          if (info->rel_residual) info->rel_residual[s] = x.rho;
          if (info->implicit_residual) info->implicit_residual[s] = x.rho;
        }
        double n2 = 0.0;
        for (double b : bni) n2 += b * b;
        norm_in = h->mrhs ? fem_norm_in : std::sqrt(n2);
        double cb = 0.0;
        for (int i = 0; i < h->ninst; ++i) {
          const double den = h->mrhs ? norm_in : bni[(size_t)i];
          cb = std::max(cb, den > 0.0 ? bound[(size_t)i] / den : 0.0);
        }
        info->certified_bound = cb;
        info->norm_in = norm_in;
        double no = 0.0;
        rexi_status s2 = vec_norm(h, outp, st, &no);
        if (s2 != REXI_OK) return s2;
        info->norm_out = no;
      }
    }
    if (!h->syncfree) prof_collect(h, st);
  }
  h->stepped = true;
  if (info) {
    info->steps = nsteps;
    info->total_iterations = its_total;
    if (info->not_converged) return fail(h, REXI_E_NOT_CONVERGED, "%d pole solves missed their target", info->not_converged);
  }
  return REXI_OK;
}

rexi_status rexi_step_adjoint(rexi_handle* h, const rexi_c128* psi_n, const rexi_c128* gbar_next,
                              rexi_c128* gbar_n, double* dV_accum, void* stream) {
  if (!h) return REXI_E_INVALID_ARG;
  if (!psi_n || !gbar_next || !gbar_n) return fail(h, REXI_E_INVALID_ARG, "NULL vector");
  if (h->ninst != 1) return fail(h, REXI_E_INVALID_ARG, "adjoint needs a single-instance handle");
  if (h->mrhs) return fail(h, REXI_E_INVALID_ARG, "the adjoint step supports finite differences only");
  hipStream_t st = (hipStream_t)stream;
  if (h->shifted && h->opt.adjoint_shared) {
    // one shared basis per side; per-pole solves when a pole misses its target
    rexi_status sa = shifted_adjoint(h, (const double2*)psi_n, (const double2*)gbar_next, (double2*)gbar_n,
                                     dV_accum, st);
    if (sa != REXI_E_NOT_BUILT) {
      if (sa == REXI_OK) prof_collect(h, st);
      return sa;
    }
  }
  if (!h->adj.ready) {
    rexi_status s0 = init_solver(h, h->adj, 2, st);
    if (s0 != REXI_OK) return s0;
  }
  Solver& sv = h->adj;
  int restarts = 0;
  // systems [0, K): (H - s_j) x_j = psi_n ; [K, 2K): (H - conj s_j) y_j = gbar_{n+1}
  rexi_status s1 = solve(h, sv, (const double2*)psi_n, (const double2*)gbar_next, st, &restarts);
  if (s1 != REXI_OK) return s1;
  const int K = h->Kinst[0];
  if (dV_accum) {
    Timed t(h, PC_GRAD, (double)h->N * (32.0 * K + 16.0), st);
    hipLaunchKernelGGL(rexi::k_grad_v, dim3(std::min(h->itotal, 2048)), dim3(TPB), 0, st, h->dinst, h->ditile,
                       h->itotal, sv.dsys, sv.W.x, dV_accum, INST_TILE, K);
    HIPCHK(h, hipGetLastError());
  }
  {
    // gbar_n = sum_j conj(w_j) y_j (systems K..2K-1 hold y_j; their weights are w_j)
    Timed t(h, PC_POLESUM, (double)h->N * 16.0 * (1.0 + K), st);
    hipLaunchKernelGGL(rexi::k_polesum, dim3(std::min(h->itotal, 2048)), dim3(TPB), 0, st, h->dinst, h->ninst,
                       h->ditile, h->itotal, sv.dsys, sv.W.x, (double2*)gbar_n, INST_TILE, 1, K);
    HIPCHK(h, hipGetLastError());
  }
  // convergence of the 2K solves
  HIPCHK(h, hipMemcpyAsync(h->hpin, sv.W.counters + sv.max_cycles * (sv.m + 1) + 1, sizeof(int32_t),
                           hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  prof_collect(h, st);
  if (h->hpin[0] != 0) return fail(h, REXI_E_NOT_CONVERGED, "%d adjoint pole solves missed their target", h->hpin[0]);
  return REXI_OK;
}

rexi_status rexi_get_solution(rexi_handle* h, int32_t pole, rexi_c128* x_dev, void* stream) {
  if (!h) return REXI_E_INVALID_ARG;
  if (!x_dev) return fail(h, REXI_E_INVALID_ARG, "NULL output");
  if (pole < 0 || pole >= (int)h->s.size()) return fail(h, REXI_E_INVALID_ARG, "pole %d out of range", pole);
  if (!h->stepped) return fail(h, REXI_E_INVALID_ARG, "no step has run");
  hipStream_t st = (hipStream_t)stream;
  int inst = 0;
  for (int q = pole; q >= h->Kinst[inst]; ++inst) q -= h->Kinst[inst];
  const size_t bytes = (size_t)h->hinst[(size_t)inst].n * sizeof(double2);
  if (h->shifted) {
    if (!h->opt.keep_solutions || !h->x_valid)
      return fail(h, REXI_E_INVALID_ARG, "the shared-basis solver keeps its pole solutions with keep_solutions = 1");
    HIPCHK(h, hipMemcpyAsync(x_dev, h->X + h->hxoff[(size_t)pole], bytes, hipMemcpyDeviceToDevice, st));
    return REXI_OK;
  }
  const SysDesc& d = h->fwd.hsys[(size_t)pole];
  HIPCHK(h, hipMemcpyAsync(x_dev, reinterpret_cast<const double2*>(h->fwd.W.x) + d.xoff, bytes,
                           hipMemcpyDeviceToDevice, st));
  return REXI_OK;
}

rexi_status rexi_get_profile(const rexi_handle* h, rexi_profile* out) {
  if (!h || !out) return REXI_E_INVALID_ARG;
  std::memset(out, 0, sizeof *out);
  out->nclasses = PC_NCLASS;
  for (int c = 0; c < PC_NCLASS; ++c) {
    out->names[c] = kProfNames[c];
    out->launches[c] = h->prof.launches[c];
    out->ms[c] = h->prof.ms[c];
    out->bytes[c] = h->prof.bytes[c];
  }
  return REXI_OK;
}

rexi_status rexi_profile_reset(rexi_handle* h) {
  if (!h) return REXI_E_INVALID_ARG;
  for (int c = 0; c < PC_NCLASS; ++c) {
    h->prof.launches[c] = 0;
    h->prof.ms[c] = 0;
    h->prof.bytes[c] = 0;
  }
  return REXI_OK;
}

rexi_status rexi_workspace_info(const rexi_handle* h, int64_t* bytes, int32_t* m_used) {
  if (!h) return REXI_E_INVALID_ARG;
  if (bytes) *bytes = h->ws_bytes;
  if (m_used) *m_used = h->fwd.m;
  return REXI_OK;
}

}  // extern "C"

namespace {

// Device buffers of one spectrum estimate: iters + 1 basis vectors, the
// working vector, the per-item partial sums and the per-instance coefficients.
struct EvSizes {
  size_t basis, w, part, coef;
  size_t total() const { return basis + w + part + coef; }
};
size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
EvSizes ev_sizes(const rexi_handle* h, int iters) {
  EvSizes z;
  z.basis = round256((size_t)(iters + 1) * (size_t)h->N * sizeof(double2));
  z.w = round256((size_t)h->N * sizeof(double2));
  z.part = round256((size_t)(iters + 1) * std::max(1, h->itotal) * sizeof(double));
  z.coef = round256((size_t)h->ninst * (iters + 1) * sizeof(double));
  return z;
}

// Lanczos estimate of the extreme eigenvalues of H per instance. ws: the
// caller's device workspace of at least ev_sizes(h, iters).total() bytes, or
// nullptr to allocate (and free) one here. Every buffer is written before it
// is read within the call, so a reused workspace needs no clearing.
rexi_status estimate_spectrum(rexi_handle* h, int32_t iters, double* lo_host, double* hi_host, hipStream_t st,
                              void* ws) {
  if (!lo_host || !hi_host) return fail(h, REXI_E_INVALID_ARG, "NULL output");
  if (iters < 1 || iters > 256) return fail(h, REXI_E_INVALID_ARG, "iters must be in [1, 256]");
  for (const auto& in : h->hinst)
    if (in.fem) return fail(h, REXI_E_INVALID_ARG, "the spectrum estimate is for the finite-difference H");
  const int S = h->ninst, T = h->itotal, tile = INST_TILE;
  const int64_t N = h->N;
  const EvSizes zs = ev_sizes(h, iters);
  double2* basis = nullptr;
  double2* w = nullptr;
  double *part = nullptr, *dcoef = nullptr;
  auto release = [&]() {
    if (ws) return;
    if (basis) (void)hipFree(basis);
    if (w) (void)hipFree(w);
    if (part) (void)hipFree(part);
    if (dcoef) (void)hipFree(dcoef);
  };
  if (ws) {
    char* base = static_cast<char*>(ws);
    basis = reinterpret_cast<double2*>(base);
    w = reinterpret_cast<double2*>(base + zs.basis);
    part = reinterpret_cast<double*>(base + zs.basis + zs.w);
    dcoef = reinterpret_cast<double*>(base + zs.basis + zs.w + zs.part);
  } else if (hipMalloc(&basis, zs.basis) != hipSuccess || hipMalloc(&w, zs.w) != hipSuccess ||
             hipMalloc(&part, zs.part) != hipSuccess || hipMalloc(&dcoef, zs.coef) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(h, REXI_E_NO_MEMORY, "spectrum estimate workspace (%zu bytes)", zs.total());
  }
  const int G = std::max(1, std::min(T, 2048));
  // per-instance sums of the item partials of vectors [0, nvec)
  auto inst_sums = [&](int nvec, std::vector<double>& out) -> rexi_status {
    std::vector<double> pv((size_t)nvec * T);
    HIPCHK(h, hipMemcpyAsync(pv.data(), part, pv.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    out.assign((size_t)S * nvec, 0.0);
    for (int ii = 0; ii < S; ++ii)
      for (int i = 0; i < nvec; ++i) {
        double acc = 0.0;
        for (int t = h->hinst[ii].tile0; t < h->hinst[ii].tile0 + h->hinst[ii].ntiles; ++t)
          acc += pv[(size_t)i * T + t];
        out[(size_t)ii * nvec + i] = acc;
      }
    return REXI_OK;
  };
  std::vector<std::vector<double>> al((size_t)S), be((size_t)S);
  std::vector<char> live((size_t)S, 1);
  std::vector<double> sums, scale((size_t)S), coef((size_t)S * (iters + 1));
  auto lanczos = [&]() -> rexi_status {
    rexi_status rs = REXI_OK;
    // v_0 = a pseudo-random vector, normalised per instance
    hipLaunchKernelGGL(k_ev_start, dim3(1024), dim3(TPB), 0, st, w, N);
    hipLaunchKernelGGL(k_norm2_inst, dim3(G), dim3(TPB), 0, st, h->dinst, h->ninst, h->ditile, T, w, part, tile);
    HIPCHK(h, hipGetLastError());
    if ((rs = inst_sums(1, sums)) != REXI_OK) return rs;
    for (int ii = 0; ii < S; ++ii) scale[ii] = sums[ii] > 0.0 ? 1.0 / std::sqrt(sums[ii]) : 0.0;
    HIPCHK(h, hipMemcpyAsync(dcoef, scale.data(), S * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_ev_scale, dim3(G), dim3(TPB), 0, st, h->dinst, h->ninst, h->ditile, T, w, basis, dcoef,
                       tile);
    for (int j = 0; j < iters && rs == REXI_OK; ++j) {
      double2* vj = basis + (int64_t)j * N;
      hipLaunchKernelGGL(rexi::k_apply_h, dim3(std::min(T, 2048)), dim3(TPB), 0, st, h->dinst, h->ninst,
                         h->ditile, T, h->V64, (const double2*)vj, w, 0.0, 0.0, tile);
      // full re-orthogonalisation: two classical Gram-Schmidt rounds
      std::fill(coef.begin(), coef.end(), 0.0);
      for (int round = 0; round < 2; ++round) {
        hipLaunchKernelGGL(k_ev_dots, dim3(G), dim3(TPB), 0, st, h->dinst, h->ninst, h->ditile, T, basis, N, w,
                           j + 1, part, tile);
        HIPCHK(h, hipGetLastError());
        if ((rs = inst_sums(j + 1, sums)) != REXI_OK) break;
        std::vector<double> c((size_t)S * (j + 1));
        for (int ii = 0; ii < S; ++ii)
          for (int i = 0; i <= j; ++i) {
            c[(size_t)ii * (j + 1) + i] = live[ii] ? sums[(size_t)ii * (j + 1) + i] : 0.0;
            coef[(size_t)ii * (iters + 1) + i] += c[(size_t)ii * (j + 1) + i];
          }
        HIPCHK(h, hipMemcpyAsync(dcoef, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_ev_update, dim3(G), dim3(TPB), 0, st, h->dinst, h->ninst, h->ditile, T, basis, N, w,
                           j + 1, dcoef, j + 1, tile);
      }
      if (rs != REXI_OK) break;
      hipLaunchKernelGGL(k_norm2_inst, dim3(G), dim3(TPB), 0, st, h->dinst, h->ninst, h->ditile, T, w, part,
                         tile);
      HIPCHK(h, hipGetLastError());
      if ((rs = inst_sums(1, sums)) != REXI_OK) break;
      for (int ii = 0; ii < S; ++ii) {
        if (!live[ii]) {
          scale[ii] = 0.0;
          continue;
        }
        al[ii].push_back(coef[(size_t)ii * (iters + 1) + j]);
        const double bn = std::sqrt(sums[ii]);
        // an invariant subspace (the whole space of a small instance): stop there
        const double anorm = std::fabs(al[ii].back()) + (be[ii].empty() ? 0.0 : be[ii].back());
        if (!(bn > 1e-13 * std::max(anorm, 1e-300)) || (int)al[ii].size() >= h->hinst[ii].n) {
          live[ii] = 0;
          scale[ii] = 0.0;
          continue;
        }
        be[ii].push_back(bn);
        scale[ii] = 1.0 / bn;
      }
      HIPCHK(h, hipMemcpyAsync(dcoef, scale.data(), S * sizeof(double), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_ev_scale, dim3(G), dim3(TPB), 0, st, h->dinst, h->ninst, h->ditile, T, w,
                         basis + (int64_t)(j + 1) * N, dcoef, tile);
      HIPCHK(h, hipGetLastError());
    }
    if (rs != REXI_OK) return rs;
    HIPCHK(h, hipStreamSynchronize(st));
    return REXI_OK;
  };
  const rexi_status rs = lanczos();
  release();
  if (rs != REXI_OK) return rs;
  for (int ii = 0; ii < S; ++ii) {
    std::vector<double>& a = al[ii];
    std::vector<double> b(be[ii].begin(), be[ii].begin() + std::min(be[ii].size(), a.empty() ? 0 : a.size() - 1));
    if (a.empty()) {
      lo_host[ii] = hi_host[ii] = 0.0;
      continue;
    }
    lo_host[ii] = tridiag_eig(a, b, 0);
    hi_host[ii] = tridiag_eig(a, b, (int)a.size() - 1);
  }
  return REXI_OK;
}

// Workspace of the allocation-free estimate: one array per GPU (each device
// holds its own copy once the library's code is loaded on it, until the
// process ends). Host code never names it: it uses the device address that
// hipGetSymbolAddress returns for the current device (scratch_address).
constexpr size_t kScratchBytes = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// The device address of scratch on the current device, looked up once per
// device (the library's setup calls this; the entry point looks it up on a
// device the setup has not seen).
rexi_status scratch_address(rexi_handle* h, void** out) {
  int dev = -1;
  HIPCHK(h, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(h, REXI_E_INVALID_ARG, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(h, REXI_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return REXI_OK;
}

}  // namespace

extern "C" {

rexi_status rexi_estimate_spectrum(rexi_handle* h, int32_t iters, double* lo_host, double* hi_host, void* stream) {
  if (!h) return REXI_E_INVALID_ARG;
  return estimate_spectrum(h, iters, lo_host, hi_host, (hipStream_t)stream, nullptr);
}

rexi_status rexi_estimate_spectrum_noalloc(rexi_handle* h, int32_t iters, double* lo_host, double* hi_host,
                                           void* stream) {
  if (!h) return REXI_E_INVALID_ARG;
  if (iters < 1 || iters > 256) return fail(h, REXI_E_INVALID_ARG, "iters must be in [1, 256]");
  const size_t need = ev_sizes(h, iters).total();
  if (need > kScratchBytes)
    return fail(h, REXI_E_INVALID_ARG,
                "the allocation-free spectrum estimate needs %zu bytes for %d iterations on %lld points; its "
                "workspace holds %zu (use rexi_estimate_spectrum or fewer iterations)",
                need, iters, (long long)h->N, kScratchBytes);
  void* ws = h->scratch;
  if (!ws) {
    rexi_status rs = scratch_address(h, &ws);
    if (rs != REXI_OK) return rs;
    h->scratch = ws;
  }
  return estimate_spectrum(h, iters, lo_host, hi_host, (hipStream_t)stream, ws);
}

rexi_status rexi_tiling_info(const rexi_handle* h, rexi_tiling* out) {
  if (!h || !out) return REXI_E_INVALID_ARG;
  out->tile = h->fwd.tile;
  out->grid_blocks = h->fwd.grid;
  out->march_slots = h->fwd.col_kh;
  out->march_planes = h->fwd.col_kh ? h->fwd.col_L : 0;
  out->march_items = h->fwd.col_kh ? h->fwd.col_total : 0;
  out->reserved_ = 0;
  return REXI_OK;
}

rexi_status rexi_destroy(rexi_handle* h) {
  destroy_handle(h);
  return REXI_OK;
}

const char* rexi_status_string(rexi_status s) {
  switch (s) {
    case REXI_OK: return "REXI_OK";
    case REXI_E_INVALID_ARG: return "REXI_E_INVALID_ARG";
    case REXI_E_NO_MEMORY: return "REXI_E_NO_MEMORY";
    case REXI_E_HIP: return "REXI_E_HIP";
    case REXI_E_NOT_CONVERGED: return "REXI_E_NOT_CONVERGED";
    case REXI_E_NOT_BUILT: return "REXI_E_NOT_BUILT";
  }
  return "REXI_E_UNKNOWN";
}

rexi_status rexi_last_error(const rexi_handle* h, char* buf, size_t len) {
  if (!buf || len == 0) return REXI_E_INVALID_ARG;
  const std::string& e = h ? h->err : g_setup_error;
  std::snprintf(buf, len, "%s", e.c_str());
  return REXI_OK;
}

}  // extern "C"
