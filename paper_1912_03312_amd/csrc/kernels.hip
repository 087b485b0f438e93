// HIP kernels of the REXI step for gfx950 (CDNA4, wave64).
//
// The step psi <- sum_j w_j (H - s_j I)^{-1} psi (eq. rational-evaluation,
// Section 3.1) is computed by restarted GMRES on every shifted system, all
// systems advancing together. One Arnoldi iteration j of every active system
// is four launches:
//   arnoldi_a   w = c_j (H - s) u_j (stencil matvec) stored as u_{j+1};
//               partial sums of <u_i, w> (i <= j) and ||w||^2 per tile
//   reduce_dots per system: h_ij = c_i <u_i, w>, DGKS test
//   arnoldi_b   u_{j+1} -= sum_i h_ij c_i u_i; partial ||u_{j+1}||^2
//   givens      per system: h_{j+1,j} = ||u_{j+1}||, Givens QR update of the
//               Hessenberg column, implicit residual, convergence decision
// (plus arnoldi_a / reduce_dots / arnoldi_b without the matvec for a second,
// DGKS, Gram-Schmidt pass). Basis vectors are stored unnormalised, v_i =
// c_i u_i, so no pass rescales a vector. A cycle ends with
//   update_x    x += sum_i y_i c_i u_i (FP64)
//   residual    r = b - (H - s) x in FP64, u_0 = r for the next cycle
//   restart     per system: explicit relative residual, done or restart
// and the step ends with the weighted pole sum in FP64 (polesum).
//
// Work tiles: a system's n points are cut into tiles of TPB * PPT points;
// a tile is one work item. The grid-stride kernels visit every (system,
// tile) item; items of systems that are not in the state a kernel serves
// return at once, so ragged convergence needs no host decision.
//
// T is the storage type of the Krylov basis: double2 (complex128) or float2
// (complex64, with the matvec in FP32). Dots, norms, Hessenberg, solutions,
// residuals and the pole sum are FP64 for both.
#include "rexi_internal.h"

#include <type_traits>

namespace rexi {

constexpr int TPB = 256;
constexpr int NWAVE = TPB / 64;
constexpr int MAXM = 256;  // largest Krylov dimension per cycle

// ------------------------------------------------------------ complex helpers
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }
template <typename T> __device__ __forceinline__ T from_d2(double2 a);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}

// ------------------------------------------------------------ reductions
// One DPP move of a double (both 32-bit halves); rows not in ROWMASK read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave with DPP lane moves (no LDS traffic):
// quad xor 1 and 2, half-row mirror, row mirror, then the row broadcasts of
// lanes 15 and 31 leave the total in lane 63, which is read back into every
// lane. The summation order is fixed, so the result is deterministic.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1, 0xF>(v);   // quad_perm(1,0,3,2)
  v += dpp_d<0x4E, 0xF>(v);   // quad_perm(2,3,0,1)
  v += dpp_d<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_d<0x140, 0xF>(v);  // row_mirror
  v += dpp_d<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum over the block; every thread gets the result. lds: NWAVE doubles.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) s += lds[w];
  return s;
}

// Sums of four per-thread values over the block (one LDS exchange).
__device__ __forceinline__ void block_sum4(double& a, double& b, double& c, double& e, double* l4) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  e = wave_sum(e);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    l4[wid] = a;
    l4[NWAVE + wid] = b;
    l4[2 * NWAVE + wid] = c;
    l4[3 * NWAVE + wid] = e;
  }
  __syncthreads();
  a = b = c = e = 0.0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) {
    a += l4[w];
    b += l4[NWAVE + w];
    c += l4[2 * NWAVE + w];
    e += l4[3 * NWAVE + w];
  }
}

__device__ __forceinline__ double block_max(double v, double* l) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) l[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) r = fmax(r, l[w]);
  return r;
}

// Thread-strided sum of p[0..n) with eight independent loads per thread in
// flight (the partial sums of a pass are written by other compute dies, so
// every load is a round trip to memory; a load-add chain would serialise them).
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int n) {
  double acc = 0.0;
  for (int b = 0; b < n; b += 8 * TPB) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = b + u * TPB + (int)threadIdx.x;
      v[u] = t < n ? p[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  return acc;
}

__device__ __forceinline__ double2 strided_sum2(const double2* __restrict__ p, int n) {
  double ax = 0.0, ay = 0.0;
  for (int b = 0; b < n; b += 8 * TPB) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = b + u * TPB + (int)threadIdx.x;
      v[u] = t < n ? p[t] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      ax += v[u].x;
      ay += v[u].y;
    }
  }
  return make_double2(ax, ay);
}

// Locate the system of global tile `item` (tile_start is the prefix array).
__device__ __forceinline__ int find_sys(const int32_t* tile_start, int S, int item) {
  int lo = 0, hi = S;  // invariant: tile_start[lo] <= item < tile_start[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tile_start[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// System of work item `item` of W: a table lookup, else the search.
__device__ __forceinline__ int item_sys(const Work& W, int item) {
  return W.tile_sys ? W.tile_sys[item] : find_sys(W.tile_start, W.S, item);
}

template <typename T> __device__ __forceinline__ T* basis_vec(const Work& W, const SysDesc& d, int i) {
  return reinterpret_cast<T*>(W.basis) + d.basis + (int64_t)i * d.n;
}

// Per-pole bases may be stored tile-interleaved (W.ilv = log2 of the work
// tile; 0: vector after vector): the points of work tile t of all m + 1
// vectors of a system are then one contiguous region, vector i at offset
// (t (m + 1) + i) * tile. A tile item of the Arnoldi passes reads its tile of
// all j + 1 vectors; stored vector after vector those are j + 1 concurrent
// streams into memory, and the bank conflicts between them cost about half
// of the bandwidth at j ~ 16 (2.3 against 5.5 TB/s for complex64, measured).
// tile_vec: vector i within tile t (index the tile's points from 0).
template <typename T> __device__ __forceinline__ T* tile_vec(const Work& W, const SysDesc& d, int t, int i) {
  T* b = reinterpret_cast<T*>(W.basis) + d.basis;
  return W.ilv ? b + (((int64_t)t * (W.m + 1) + i) << W.ilv) : b + (int64_t)i * d.n + (int64_t)t * W.tile;
}
// Basis vectors whose loads a tile item issues together: eight, or fewer so
// that they take at most 64 registers per thread.
template <typename T, int PPT> __device__ constexpr int au_vectors() {
  return 256 / (PPT * (int)sizeof(T)) < 8 ? 256 / (PPT * (int)sizeof(T)) : 8;
}
// Slot q (0 <= q < PPT) of a thread handles point tpt<T>(q) of its work tile.
// complex64 pairs neighbouring points in a thread (slots 2k and 2k + 1 are
// adjacent), so that a lane moves 16 bytes per load, as complex128 does with
// one point: with 8-byte lanes the Arnoldi passes ran at half the bandwidth.
template <typename T> __device__ __forceinline__ int tpt(int q) {
  return sizeof(T) == 8 ? ((q >> 1) * TPB + (int)threadIdx.x) * 2 + (q & 1) : q * TPB + (int)threadIdx.x;
}
// Slots of a thread in the tile of vector u (its points p0 + tpt(q)), zero
// past n. FULL: the tile's region is allocated to its end (tile-interleaved
// bases), so a complex64 pair is loaded whole and masked. FULL is a template
// parameter: a runtime choice put every load in a branch of its own, and the
// compiler then waited for each load before issuing the next.
template <typename T, int PPT, bool FULL>
__device__ __forceinline__ void tile_load(const T* __restrict__ u, int p0, int n, T (&a)[PPT]) {
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int k = 0; k < PPT / 2; ++k) {
      const int o = tpt<T>(2 * k), p = p0 + o;
      if constexpr (FULL) {
        const float4 v = *reinterpret_cast<const float4*>(u + o);
        a[2 * k] = p < n ? T{v.x, v.y} : T{};
        a[2 * k + 1] = p + 1 < n ? T{v.z, v.w} : T{};
      } else {
        a[2 * k] = p < n ? u[o] : T{};
        a[2 * k + 1] = p + 1 < n ? u[o + 1] : T{};
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int o = tpt<T>(q);
      a[q] = p0 + o < n ? u[o] : T{};
    }
  }
}
// Store the slots of a thread to the tile of vector u (points below n only).
template <typename T, int PPT, bool FULL>
__device__ __forceinline__ void tile_store(T* __restrict__ u, int p0, int n, const T (&a)[PPT]) {
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int k = 0; k < PPT / 2; ++k) {
      const int o = tpt<T>(2 * k), p = p0 + o;
      if (FULL && p + 1 < n) {
        *reinterpret_cast<float4*>(u + o) = make_float4(a[2 * k].x, a[2 * k].y, a[2 * k + 1].x, a[2 * k + 1].y);
      } else {
        if (p < n) u[o] = a[2 * k];
        if (p + 1 < n) u[o + 1] = a[2 * k + 1];
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int o = tpt<T>(q);
      if (p0 + o < n) u[o] = a[q];
    }
  }
}
// Point q of a vector in either layout: map_vec(i)[BMap(q)] (for stencils,
// whose neighbours lie in other tiles).
struct BMap {
  int lt, vs;  // log2 of the tile (0: plain), vectors per tile
  __device__ __forceinline__ int64_t operator()(uint32_t q) const {
    return lt ? ((((int64_t)(q >> lt)) * vs) << lt) + (int64_t)(q & ((1u << lt) - 1u)) : (int64_t)q;
  }
};
__device__ __forceinline__ BMap bmap(const Work& W) { return BMap{W.ilv, W.m + 1}; }
template <typename T> __device__ __forceinline__ T* map_vec(const Work& W, const SysDesc& d, int i) {
  T* b = reinterpret_cast<T*>(W.basis) + d.basis;
  return W.ilv ? b + ((int64_t)i << W.ilv) : b + (int64_t)i * d.n;
}

// Iteration indices of captured schedules. A launch's iteration is its
// argument when that is >= 0. A captured schedule cannot read anything on the
// host, so its launches take the index from the device instead: JD_REC is
// the iteration paused for a second Gram-Schmidt pass and JD_REC1 the one
// after it (-1, nothing to do, when no pass is pending); JD_LAUNCH - L is
// launch L of the fused sequence, which runs iteration L minus the launches
// that pauses took (a paused solve skips launches until its pass has run).
constexpr int JD_REC = -1, JD_REC1 = -2, JD_LAUNCH = -16;
__device__ __forceinline__ int dev_iter(const Work& W, int j) {
  if (j >= 0) return j;
  const int rec = W.jdev[0];
  if (j == JD_REC) return rec;
  if (j == JD_REC1) return rec < 0 ? -1 : rec + 1;
  return (JD_LAUNCH - j) - W.jdev[1];
}

// The stencil's geometry and coefficients of a system held in registers (a
// SysDesc reference into global memory is re-read after every store the
// compiler cannot prove apart from it, and each re-read waits for the loads
// in flight).
struct SGeo {
  FastDiv d2, d1;
  int n0, n1, n2;
  double c0, c1, c2, diag, sre, sim;
  int64_t off;
};
__device__ __forceinline__ SGeo sgeo(const SysDesc& d) {
  return SGeo{d.d2, d.d1, d.n0, d.n1, d.n2, d.c0, d.c1, d.c2, d.diag, d.sre, d.sim, d.off};
}

// (H - s) u at point p, for storage type T, in the arithmetic of T. D is a
// SysDesc or an SGeo.
template <typename T, typename D>
__device__ __forceinline__ double2 stencil_point(const T* __restrict__ u, const D& d, double vp, uint32_t p,
                                                 BMap mp = BMap{0, 0}) {
  const uint32_t r = fdiv(p, d.d2);
  const uint32_t k = p - r * (uint32_t)d.n2;
  const uint32_t i0 = fdiv(r, d.d1);
  const uint32_t j = r - i0 * (uint32_t)d.n1;
  const uint32_t plane = (uint32_t)d.n1 * (uint32_t)d.n2;
  if constexpr (std::is_same<T, double2>::value) {
    const double2 c = u[mp(p)];
    double2 nb2 = make_double2(0.0, 0.0), nb1 = nb2, nb0 = nb2;
    // every neighbour load is issued (a missing neighbour reads p itself) and
    // a missing one is added as zero: no branch between the loads
    const bool hl = k > 0, hr = k + 1 < (uint32_t)d.n2, hd = j > 0, hu = j + 1 < (uint32_t)d.n1;
    const bool hb = i0 > 0, hf = i0 + 1 < (uint32_t)d.n0;
    const double2 tl = u[mp(hl ? p - 1 : p)], tr = u[mp(hr ? p + 1 : p)];
    const double2 td = u[mp(hd ? p - d.n2 : p)], tu = u[mp(hu ? p + d.n2 : p)];
    const double2 tb = u[mp(hb ? p - plane : p)], tf = u[mp(hf ? p + plane : p)];
    const double2 z = make_double2(0.0, 0.0);
    const double2 al = hl ? tl : z, ar = hr ? tr : z, ad = hd ? td : z, au = hu ? tu : z, ab = hb ? tb : z,
              af = hf ? tf : z;
    nb2.x += al.x; nb2.y += al.y;
    nb2.x += ar.x; nb2.y += ar.y;
    nb1.x += ad.x; nb1.y += ad.y;
    nb1.x += au.x; nb1.y += au.y;
    nb0.x += ab.x; nb0.y += ab.y;
    nb0.x += af.x; nb0.y += af.y;
    const double a = d.diag + vp - d.sre;
    double2 o;
    o.x = a * c.x + d.sim * c.y - (d.c2 * nb2.x + d.c1 * nb1.x + d.c0 * nb0.x);
    o.y = a * c.y - d.sim * c.x - (d.c2 * nb2.y + d.c1 * nb1.y + d.c0 * nb0.y);
    return o;
  } else {
    const float2 c = u[mp(p)];
    float2 nb2 = make_float2(0.f, 0.f), nb1 = nb2, nb0 = nb2;
    // every neighbour load is issued (a missing neighbour reads p itself) and
    // a missing one is added as zero: no branch between the loads
    const bool hl = k > 0, hr = k + 1 < (uint32_t)d.n2, hd = j > 0, hu = j + 1 < (uint32_t)d.n1;
    const bool hb = i0 > 0, hf = i0 + 1 < (uint32_t)d.n0;
    const float2 tl = u[mp(hl ? p - 1 : p)], tr = u[mp(hr ? p + 1 : p)];
    const float2 td = u[mp(hd ? p - d.n2 : p)], tu = u[mp(hu ? p + d.n2 : p)];
    const float2 tb = u[mp(hb ? p - plane : p)], tf = u[mp(hf ? p + plane : p)];
    const float2 z = make_float2(0.f, 0.f);
    const float2 al = hl ? tl : z, ar = hr ? tr : z, ad = hd ? td : z, au = hu ? tu : z, ab = hb ? tb : z,
              af = hf ? tf : z;
    nb2.x += al.x; nb2.y += al.y;
    nb2.x += ar.x; nb2.y += ar.y;
    nb1.x += ad.x; nb1.y += ad.y;
    nb1.x += au.x; nb1.y += au.y;
    nb0.x += ab.x; nb0.y += ab.y;
    nb0.x += af.x; nb0.y += af.y;
    const float a = (float)(d.diag - d.sre) + (float)vp;
    const float sim = (float)d.sim;
    const float c2 = (float)d.c2, c1 = (float)d.c1, c0 = (float)d.c0;
    float ox = a * c.x + sim * c.y - (c2 * nb2.x + c1 * nb1.x + c0 * nb0.x);
    float oy = a * c.y - sim * c.x - (c2 * nb2.y + c1 * nb1.y + c0 * nb0.y);
    return make_double2((double)ox, (double)oy);
  }
}

// (H - s) u at the adjacent points p and p + 1 of a complex64 vector of a
// tile-interleaved basis (p even and n2 even: both points lie in one row and
// one tile, and every pair below is one aligned 16-byte load). Each point's
// arithmetic is stencil_point<float2>'s, term by term.
__device__ __forceinline__ void stencil_pair_c64(const float2* __restrict__ u, const float* __restrict__ V,
                                                 const SGeo& d, uint32_t p, BMap mp, double2& o0,
                                                 double2& o1) {
  const uint32_t r = fdiv(p, d.d2);
  const uint32_t k = p - r * (uint32_t)d.n2;
  const uint32_t i0 = fdiv(r, d.d1);
  const uint32_t jr = r - i0 * (uint32_t)d.n1;
  const uint32_t plane = (uint32_t)d.n1 * (uint32_t)d.n2;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  auto pair = [&](uint32_t q) { return *reinterpret_cast<const float4*>(u + mp(q)); };
  const float4 c = pair(p);
  // every load is issued (a missing neighbour reads p itself) and masked:
  // no branch between the loads
  const bool hl = k > 0, hr = k + 2 < (uint32_t)d.n2;
  const bool hd = jr > 0, hu = jr + 1 < (uint32_t)d.n1, hb = i0 > 0, hf = i0 + 1 < (uint32_t)d.n0;
  const float2 l0 = u[mp(hl ? p - 1 : p)], r0 = u[mp(hr ? p + 2 : p)];
  const float4 dn0 = pair(hd ? p - d.n2 : p), up0 = pair(hu ? p + d.n2 : p);
  const float4 bk0 = pair(hb ? p - plane : p), fr0 = pair(hf ? p + plane : p);
  const float2 l = hl ? l0 : make_float2(0.f, 0.f), rr = hr ? r0 : make_float2(0.f, 0.f);
  const float4 dn = hd ? dn0 : z4, up = hu ? up0 : z4, bk = hb ? bk0 : z4, fr = hf ? fr0 : z4;
  const float2 vv = *reinterpret_cast<const float2*>(V + d.off + p);
  const float sim = (float)d.sim;
  const float c2 = (float)d.c2, c1 = (float)d.c1, c0 = (float)d.c0;
  const float a0 = (float)(d.diag - d.sre) + vv.x, a1 = (float)(d.diag - d.sre) + vv.y;
  // point p: left neighbour if any, right neighbour p + 1
  float2 nb2 = make_float2(0.f, 0.f), nb1 = nb2, nb0 = nb2;
  if (k > 0) { nb2.x += l.x; nb2.y += l.y; }
  nb2.x += c.z; nb2.y += c.w;
  if (hd) { nb1.x += dn.x; nb1.y += dn.y; }
  if (hu) { nb1.x += up.x; nb1.y += up.y; }
  if (hb) { nb0.x += bk.x; nb0.y += bk.y; }
  if (hf) { nb0.x += fr.x; nb0.y += fr.y; }
  float ox = a0 * c.x + sim * c.y - (c2 * nb2.x + c1 * nb1.x + c0 * nb0.x);
  float oy = a0 * c.y - sim * c.x - (c2 * nb2.y + c1 * nb1.y + c0 * nb0.y);
  o0 = make_double2((double)ox, (double)oy);
  // point p + 1: left neighbour p, right neighbour if any
  nb2 = make_float2(0.f, 0.f); nb1 = nb2; nb0 = nb2;
  nb2.x += c.x; nb2.y += c.y;
  if (hr) { nb2.x += rr.x; nb2.y += rr.y; }
  if (hd) { nb1.x += dn.z; nb1.y += dn.w; }
  if (hu) { nb1.x += up.z; nb1.y += up.w; }
  if (hb) { nb0.x += bk.z; nb0.y += bk.w; }
  if (hf) { nb0.x += fr.z; nb0.y += fr.w; }
  ox = a1 * c.z + sim * c.w - (c2 * nb2.x + c1 * nb1.x + c0 * nb0.x);
  oy = a1 * c.w - sim * c.z - (c2 * nb2.y + c1 * nb1.y + c0 * nb0.y);
  o1 = make_double2((double)ox, (double)oy);
}

// FP64 stencil on an FP64 vector: (H - s) x at p.
__device__ __forceinline__ double2 stencil_point_f64(const double2* __restrict__ u, int n0, int n1, int n2,
                                                     const FastDiv& d2, const FastDiv& d1, double c0, double c1,
                                                     double c2, double diag, double vp, double sre, double sim,
                                                     uint32_t p) {
  const uint32_t r = fdiv(p, d2);
  const uint32_t k = p - r * (uint32_t)n2;
  const uint32_t i0 = fdiv(r, d1);
  const uint32_t j = r - i0 * (uint32_t)n1;
  const uint32_t plane = (uint32_t)n1 * (uint32_t)n2;
  const double2 c = u[p];
  double2 nb2 = make_double2(0.0, 0.0), nb1 = nb2, nb0 = nb2;
  // every neighbour load is issued (a missing neighbour reads p itself) and a
  // missing one is added as zero: no branch between the loads
  const bool hl = k > 0, hr = k + 1 < (uint32_t)n2, hd = j > 0, hu = j + 1 < (uint32_t)n1;
  const bool hb = i0 > 0, hf = i0 + 1 < (uint32_t)n0;
  const double2 tl = u[hl ? p - 1 : p], tr = u[hr ? p + 1 : p], td = u[hd ? p - n2 : p], tu = u[hu ? p + n2 : p];
  const double2 tb = u[hb ? p - plane : p], tf = u[hf ? p + plane : p];
  const double2 z = make_double2(0.0, 0.0);
  const double2 al = hl ? tl : z, ar = hr ? tr : z, ad = hd ? td : z, au = hu ? tu : z, ab = hb ? tb : z,
                af = hf ? tf : z;
  nb2.x += al.x; nb2.y += al.y;
  nb2.x += ar.x; nb2.y += ar.y;
  nb1.x += ad.x; nb1.y += ad.y;
  nb1.x += au.x; nb1.y += au.y;
  nb0.x += ab.x; nb0.y += ab.y;
  nb0.x += af.x; nb0.y += af.y;
  const double a = diag + vp - sre;
  double2 o;
  o.x = a * c.x + sim * c.y - (c2 * nb2.x + c1 * nb1.x + c0 * nb0.x);
  o.y = a * c.y - sim * c.x - (c2 * nb2.y + c1 * nb1.y + c0 * nb0.y);
  return o;
}

// Q1 finite elements: (A - s M) u at p with A = K' + h^d diag(V) (K' the
// stiffness matrix times hbar^2/2m) and M the consistent mass matrix, both
// Kronecker structured: the entry for the neighbour offset (e0, e1, e2) in
// {-1, 0, 1}^3 is  m0(e0) m1(e1) m2(e2)  for M and
// k0(e0) m1(e1) m2(e2) + m0(e0) k1(e1) m2(e2) + m0(e0) m1(e1) k2(e2)  for K'
// (m(0) = md, m(+-1) = mo, k(0) = kd, k(+-1) = ko per axis). Arithmetic in
// the precision of T (as the finite-difference stencil).
template <typename T> struct scalar_of;
template <> struct scalar_of<double2> { using type = double; };
template <> struct scalar_of<float2> { using type = float; };

template <typename T>
__device__ __forceinline__ double2 fem_point(const T* __restrict__ u, int n0, int n1, int n2, const FastDiv& d2,
                                             const FastDiv& d1, const double* md, const double* mo,
                                             const double* kd, const double* ko, double vol, double vp,
                                             double sre, double sim, uint32_t p) {
  using R = typename scalar_of<T>::type;
  const uint32_t r = fdiv(p, d2);
  const uint32_t k = p - r * (uint32_t)n2;
  const uint32_t i0 = fdiv(r, d1);
  const uint32_t j = r - i0 * (uint32_t)n1;
  const int plane = n1 * n2;
  const int lo0 = i0 > 0 ? -1 : 0, hi0 = i0 + 1 < (uint32_t)n0 ? 1 : 0;
  const int lo1 = j > 0 ? -1 : 0, hi1 = j + 1 < (uint32_t)n1 ? 1 : 0;
  const int lo2 = k > 0 ? -1 : 0, hi2 = k + 1 < (uint32_t)n2 ? 1 : 0;
  R mx = 0, my = 0, kx = 0, ky = 0;  // M u and K' u
  for (int e0 = lo0; e0 <= hi0; ++e0) {
    const R m0 = (R)(e0 ? mo[0] : md[0]), k0 = (R)(e0 ? ko[0] : kd[0]);
    for (int e1 = lo1; e1 <= hi1; ++e1) {
      const R m1 = (R)(e1 ? mo[1] : md[1]), k1 = (R)(e1 ? ko[1] : kd[1]);
      // the three points along axis 2 at once
      R sx = 0, sy = 0, tx = 0, ty = 0;  // sum m2 u, sum k2 u
      for (int e2 = lo2; e2 <= hi2; ++e2) {
        const T v = u[(int)p + e0 * plane + e1 * n2 + e2];
        const R m2 = (R)(e2 ? mo[2] : md[2]), k2 = (R)(e2 ? ko[2] : kd[2]);
        sx += m2 * (R)v.x;
        sy += m2 * (R)v.y;
        tx += k2 * (R)v.x;
        ty += k2 * (R)v.y;
      }
      const R mm = m0 * m1;
      mx += mm * sx;
      my += mm * sy;
      const R kk = k0 * m1 + m0 * k1;
      kx += kk * sx + mm * tx;
      ky += kk * sy + mm * ty;
    }
  }
  const T c = u[p];
  const R a = (R)(vol * vp);
  const R sr = (R)sre, si = (R)sim;
  // (K' + vol V) u - s M u
  const R ox = kx + a * (R)c.x - (sr * mx - si * my);
  const R oy = ky + a * (R)c.y - (sr * my + si * mx);
  return make_double2((double)ox, (double)oy);
}

// ---------------------------------------------------------------- Q1 shared basis
// M = L L^T with L = L_0 (x) L_1 (x) L_2, L_a the bidiagonal Cholesky factor
// of the 1D mass matrix of axis a (chol + loff[a]: diagonal d[n_a], then
// subdiagonal e[n_a], e_0 = 0; an absent axis has d = 1). The solves
// (A - s M) x = M psi become (Ahat - s) xhat = L^T psi with
// Ahat = L^-1 A L^-T and x = L^-T xhat.

// y = L^T x on one instance: (L_a^T)_{i,i} = d_i, (L_a^T)_{i,i+1} = e_{i+1}.
__global__ __launch_bounds__(TPB) void k_fem_lt(InstDesc in, const double* __restrict__ chol,
                                               const double2* __restrict__ x, double2* __restrict__ y) {
  const double* d0 = chol + in.loff[0];
  const double* d1 = chol + in.loff[1];
  const double* d2 = chol + in.loff[2];
  const int64_t plane = (int64_t)in.n1 * in.n2;
  for (int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x; p < in.n; p += (int64_t)gridDim.x * TPB) {
    const uint32_t r = fdiv((uint32_t)p, in.d2);
    const int i2 = (int)(p - (int64_t)r * in.n2);
    const int i0 = (int)fdiv(r, in.d1);
    const int i1 = (int)(r - (uint32_t)i0 * (uint32_t)in.n1);
    double t0[2] = {d0[i0], i0 + 1 < in.n0 ? d0[in.n0 + i0 + 1] : 0.0};
    double t1[2] = {d1[i1], i1 + 1 < in.n1 ? d1[in.n1 + i1 + 1] : 0.0};
    double t2[2] = {d2[i2], i2 + 1 < in.n2 ? d2[in.n2 + i2 + 1] : 0.0};
    double2 acc = make_double2(0.0, 0.0);
    for (int a = 0; a < 2; ++a) {
      if (t0[a] == 0.0) continue;
      for (int b = 0; b < 2; ++b) {
        if (t1[b] == 0.0) continue;
        for (int c = 0; c < 2; ++c) {
          if (t2[c] == 0.0) continue;
          const double f = t0[a] * t1[b] * t2[c];
          const double2 v = x[in.off + p + a * plane + b * in.n2 + c];
          acc.x += f * v.x;
          acc.y += f * v.y;
        }
      }
    }
    y[in.off + p] = acc;
  }
}

// y = A x on one Q1 instance (the element operator without shift: stiffness
// (hbar^2/2m) K plus h^d V by nodal quadrature), each thread a run of FEM_R
// consecutive points along the fastest axis: per row of the 3 x 3
// neighbourhood it loads FEM_R + 2 values once for all FEM_R outputs.
constexpr int FEM_R = 4;
__global__ __launch_bounds__(TPB) void k_fem_apply(InstDesc in, const double* __restrict__ V,
                                                  const double2* __restrict__ x, double2* __restrict__ y) {
  const int n0 = in.n0, n1 = in.n1, n2 = in.n2;
  const int runs = (n2 + FEM_R - 1) / FEM_R;
  const int64_t total = (int64_t)n0 * n1 * runs;
  const int64_t plane = (int64_t)n1 * n2;
  const double2* u = x + in.off;
  for (int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x; q < total; q += (int64_t)gridDim.x * TPB) {
    const int64_t row = q / runs;
    const int i2 = (int)(q - row * runs) * FEM_R;
    const int i0 = (int)(row / n1), i1 = (int)(row - (int64_t)i0 * n1);
    double mx[FEM_R], my[FEM_R], kx[FEM_R], ky[FEM_R];
#pragma unroll
    for (int r = 0; r < FEM_R; ++r) mx[r] = my[r] = kx[r] = ky[r] = 0.0;
    for (int e0 = -1; e0 <= 1; ++e0) {
      if (i0 + e0 < 0 || i0 + e0 >= n0) continue;
      const double m0 = e0 ? in.fmo[0] : in.fmd[0], k0 = e0 ? in.fko[0] : in.fkd[0];
      for (int e1 = -1; e1 <= 1; ++e1) {
        if (i1 + e1 < 0 || i1 + e1 >= n1) continue;
        const double m1 = e1 ? in.fmo[1] : in.fmd[1], k1 = e1 ? in.fko[1] : in.fkd[1];
        const double2* ur = u + (int64_t)(i0 + e0) * plane + (int64_t)(i1 + e1) * n2;
        // the row's values at i2 - 1 .. i2 + FEM_R (zero outside the grid)
        double2 w[FEM_R + 2];
#pragma unroll
        for (int k = 0; k < FEM_R + 2; ++k) {
          const int c = i2 - 1 + k;
          w[k] = (c >= 0 && c < n2) ? ur[c] : make_double2(0.0, 0.0);
        }
        const double mm = m0 * m1, kk = k0 * m1 + m0 * k1;
#pragma unroll
        for (int r = 0; r < FEM_R; ++r) {
          const double2 a = w[r], b = w[r + 1], c = w[r + 2];
          const double sx = in.fmd[2] * b.x + in.fmo[2] * (a.x + c.x), sy = in.fmd[2] * b.y + in.fmo[2] * (a.y + c.y);
          const double tx = in.fkd[2] * b.x + in.fko[2] * (a.x + c.x), ty = in.fkd[2] * b.y + in.fko[2] * (a.y + c.y);
          mx[r] += mm * sx;
          my[r] += mm * sy;
          kx[r] += kk * sx + mm * tx;
          ky[r] += kk * sy + mm * ty;
        }
      }
    }
    const int64_t p0 = (int64_t)i0 * plane + (int64_t)i1 * n2 + i2;
#pragma unroll
    for (int r = 0; r < FEM_R; ++r) {
      if (i2 + r >= n2) break;
      const double2 c = u[p0 + r];
      const double a = in.fvol * V[in.off + p0 + r];
      y[in.off + p0 + r] = make_double2(kx[r] + a * c.x, ky[r] + a * c.y);
    }
  }
}

// One factor along axis `axis` of one instance:
// backward = 0: dst = L_a^-1 src (v_i = (x_i - e_i v_{i-1}) / d_i);
// backward = 1: dst = L_a^-T src (v_i = (x_i - e_{i+1} v_{i+1}) / d_i).
// Each thread takes one segment of FEM_SEG entries of one grid line and
// starts the recurrence `warm` entries before it (in sweep order) from
// v = 0: an error in v shrinks by |e/d| <= rho per step, so the segment
// differs from the exact sweep by at most rho^warm max|v| (the host picks
// warm with rho^warm below 2^-64; for the Q1 mass factors rho ~ 0.27). The
// segments of a line are independent, so a sweep has n / n_a * ceil(n_a /
// FEM_SEG) threads instead of n / n_a. src and dst must differ.
constexpr int FEM_SEG = 32;
constexpr int FEM_TPB = 64;
constexpr int FEM_UNR = 8;
__global__ __launch_bounds__(FEM_TPB) void k_fem_sweep(InstDesc in, const double* __restrict__ chol,
                                                      const double2* __restrict__ src, double2* __restrict__ dst,
                                                      int axis, int backward, int warm) {
  const int na = axis == 0 ? in.n0 : (axis == 1 ? in.n1 : in.n2);
  const double* dg = chol + in.loff[axis];
  const double* eg = dg + na;
  const double* rg = dg + 2 * na;  // 1 / d
  const int64_t nl = in.n / na;
  const int nseg = (na + FEM_SEG - 1) / FEM_SEG;
  const int64_t plane = (int64_t)in.n1 * in.n2;
  for (int64_t q = (int64_t)blockIdx.x * FEM_TPB + threadIdx.x; q < nl * nseg; q += (int64_t)gridDim.x * FEM_TPB) {
    // consecutive threads take consecutive lines of one segment (coalesced
    // along the fastest axis for axes 0 and 1)
    const int sg = (int)(q / nl);
    const int64_t l = q - (int64_t)sg * nl;
    int64_t base, stride;
    if (axis == 0) {
      base = l;  // (i1, i2) = (l / n2, l % n2)
      stride = plane;
    } else if (axis == 1) {
      base = (l / in.n2) * plane + l % in.n2;  // (i0, i2)
      stride = in.n2;
    } else {
      base = l * in.n2;  // row (i0, i1)
      stride = 1;
    }
    const double2* x = src + in.off + base;
    double2* v = dst + in.off + base;
    // positions k = 0 .. na-1 in sweep order; this segment writes [k0, k1).
    // The inputs of FEM_UNR positions are loaded before their steps run (the
    // last group repeats position k1 - 1 past the end, unused), so the loads
    // of a group are in flight together; the pivots' reciprocals are stored.
    const int k0 = sg * FEM_SEG, k1 = min(na, k0 + FEM_SEG);
    const int ks = max(0, k0 - warm);
    double2 prev = make_double2(0.0, 0.0);
    for (int kb = ks; kb < k1; kb += FEM_UNR) {
      double2 xv[FEM_UNR];
      double ev[FEM_UNR], rv[FEM_UNR];
#pragma unroll
      for (int u = 0; u < FEM_UNR; ++u) {
        const int k = min(kb + u, k1 - 1);
        const int i = backward ? na - 1 - k : k;
        xv[u] = x[(int64_t)i * stride];
        ev[u] = backward ? (i + 1 < na ? eg[i + 1] : 0.0) : (i > 0 ? eg[i] : 0.0);
        rv[u] = rg[i];
      }
#pragma unroll
      for (int u = 0; u < FEM_UNR; ++u) {
        const int k = kb + u;
        if (k < k1) {
          const int i = backward ? na - 1 - k : k;
          prev = make_double2((xv[u].x - ev[u] * prev.x) * rv[u], (xv[u].y - ev[u] * prev.y) * rv[u]);
          if (k >= k0) v[(int64_t)i * stride] = prev;
        }
      }
    }
  }
}

template <typename T> __device__ __forceinline__ double vpot(const Work& W, int64_t idx);
template <> __device__ __forceinline__ double vpot<double2>(const Work& W, int64_t idx) { return W.V64[idx]; }
template <> __device__ __forceinline__ double vpot<float2>(const Work& W, int64_t idx) { return (double)W.V32[idx]; }

// ------------------------------------------------------------ cycle start
// u_0 = b (cast to T) and partial ||b||^2 for every system; solutions reset.
template <typename T, int PPT>
__global__ __launch_bounds__(TPB) void k_start(Work W, const double2* __restrict__ rhs0,
                                               const double2* __restrict__ rhs1) {
  __shared__ double lds[NWAVE];
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const double2* __restrict__ b = (d.rhs_sel ? rhs1 : rhs0) + d.off;
    T* __restrict__ u0 = tile_vec<T>(W, d, t, 0);
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = t * W.tile + q * TPB + threadIdx.x;
      if (p < d.n) {
        double2 v = b[p];
        u0[q * TPB + threadIdx.x] = from_d2<T>(v);
        acc += v.x * v.x + v.y * v.y;
      }
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) W.pnorm[item] = acc;
  }
}

// Per system: ||b||, initial Givens right-hand side, state reset.
__global__ __launch_bounds__(TPB) void k_start_reduce(Work W) {
  __shared__ double lds[NWAVE];
  const int s = blockIdx.x;
  if (s >= W.S) return;
  const SysDesc& d = W.sys[s];
  if (s == 0) {
    const int nc = W.max_cycles * (W.m + 1) + 2;
    for (int i = threadIdx.x; i < nc; i += TPB) W.counters[i] = 0;
    if (W.reo_any)
      for (int i = threadIdx.x; i <= W.m; i += TPB) W.reo_any[i] = 0;
  }
  double acc = strided_sum(W.pnorm + d.tile0, d.ntiles);
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) {
    const double bn = sqrt(acc);
    SysState_t& st = W.st[s];
    st.bnorm = bn;
    st.rnorm = bn;
    st.rho = 1.0;
    st.its = 0;
    st.cycles = 0;
    st.kcyc = 0;
    st.reorth = 0;
    st.first = 1;
    double2* g = reinterpret_cast<double2*>(W.gvec) + (int64_t)s * (W.m + 1);
    for (int i = 0; i <= W.m; ++i) g[i] = make_double2(0.0, 0.0);
    g[0] = make_double2(bn, 0.0);
    W.cscale[(int64_t)s * (W.m + 1)] = bn > 0.0 ? 1.0 / bn : 0.0;
    // a zero right-hand side has the zero solution
    st.state = bn > 0.0 ? ST_ACTIVE : ST_FINISH;
  }
}

// ------------------------------------------------------------ shared basis
// All poles share one Krylov basis: with x0 = 0 every shifted system starts
// from b, and K_k(H - s I, b) = K_k(H, b). One Arnoldi (or, H being
// Hermitian, Lanczos) process on H (system 0 with shift 0) gives
// H V_k = V_{k+1} Hbar_k, hence (H - s_p) V_k = V_{k+1} (Hbar_k - s_p Itilde);
// each pole solves its own small least-squares problem
// min || ||b|| e_1 - (Hbar_k - s_p Itilde) y_p ||, and the step is
// sum_p w_p V_k y_p = V_k z with z = sum_p w_p y_p.
struct ShiftWork {
  int32_t K;          // poles over all instances (0: per-pole solver)
  const int32_t* pole0;  // [S+1] first pole of each instance (system)
  const int32_t* pinst;  // [K] instance of each pole
  const double* s;    // [K] complex shifts
  const double* w;    // [K] complex weights
  const double* tol;  // [K] target relative residuals
  // certified policy: cw[p] = |w_p| / dist(s_p, spectrum bound); an instance
  // also stops once sum_p cw[p] ||r_p|| <= tau ||b|| / 2 (null: per-pole
  // targets only)
  const double* cw;
  double tau;
  double* R;          // [K][(m+1) m] complex, rotated Hessenberg per pole
  double* g;          // [K][m+1] complex
  double* gc;         // [K][m] complex
  double* gs;         // [K][m] complex
  double* y;          // [K][m] complex
  double* z;          // [S][m] complex, combined coefficients per instance
  double* res;        // [K] implicit relative residual
  int32_t* its;       // [K] iteration at which the pole met its target (0: not yet)
  // Lanczos with partial reorthogonalisation (three-term recurrence)
  int32_t lanczos;    // 1: project only on the last two basis vectors
  double* alpha;      // [S][m] diagonal of the tridiagonal matrix
  double* beta;       // [S][m+1] off-diagonal, beta[j+1] = ||v_{j+1}||
  double* omega;      // [S][2][m+1] estimated <v_j, v_k>, <v_{j+1}, v_k> (rolling)
  int32_t* flags;     // [S][4] [0]: reorthogonalise the next vector too; [1]: passes done;
                      // [2]: iteration at which the solve paused (-1: none)
  int32_t pause_mode; // 1: pause for a second pass instead of predicated passes
  int32_t cap_next;   // captured schedules: the fused launch that follows a recovery
  int32_t* gpause;    // [1] iteration at which the solve paused (-1: none): the passes and
                      // ends of later iterations return at once, for every system
  int32_t* full;      // [S][m] 1 if column j of Hbar has entries above row j - 1
  double* zb;         // [2][sum n] complex: z_j = H u_j of the pipelined recurrence
  int64_t zstride;    // complex elements per z buffer
  const int32_t* col_start;  // [S+1] prefix of column-marching items (null: unused)
  const int32_t* col_sys;    // [col_total] system of each item (null: search col_start)
  int32_t col_total;
  int32_t fb_skip;    // 1: poles that missed their target (its = 0) are left out of z
  // Restarts on the shared basis. fom = 1: a pole that missed its target takes
  // the Galerkin iterate of the basis, whose residual is gnext_p u_k (u_k the
  // stored basis vector k): the residuals of all such poles of an instance
  // are multiples of one vector, the next cycle's right-hand side.
  int32_t fom;
  double* gnext;      // [K] complex: gnext_p = -y_{p,k-1} of the Galerkin iterate
  // restart = 1 (a restart cycle): only poles with miss[p] take part, with
  // right-hand side gam_p b (b the cycle's right-hand side); w, tol, its and
  // res above point to the cycle's own arrays, filled from these at its start
  int32_t restart;
  const int32_t* miss;  // [K]
  const double* gam;    // [K] complex
  const double* w0;     // [K] complex weights of the step
  const double* tol0;   // [K] targets relative to ||psi|| of the step
  const double* bn0;    // [S] ||psi|| per instance
};

// Grid (S, j + 2): block (s, i) with lo <= i <= j reduces the tile partials
// of <u_i, w> to h_ij = c_i <u_i, w> (lo = i0 on the first pass, 0 on the
// second); blocks i < lo zero the entry (three-term window); block j + 1
// reduces ||w||^2 (first pass). The first pass stores the Hessenberg column,
// the second (re-orthogonalisation) pass adds its correction.
__global__ __launch_bounds__(TPB) void k_reduce_dots(Work W, int j, int second, int i0) {
  __shared__ double lds[NWAVE];
  j = dev_iter(W, j);
  if (j < 0) return;
  const int s = blockIdx.x;
  const int i = blockIdx.y;
  if (s >= W.S || i > j + 1) return;
  if (second && W.reo_any && !W.reo_any[j]) return;
  SysState_t& st = W.st[s];
  if (st.state != ST_ACTIVE) return;
  if (second && !st.reorth) return;
  const SysDesc& d = W.sys[s];
  const int lo = second ? 0 : i0;
  double2* hcol = reinterpret_cast<double2*>(W.H) + (int64_t)s * (W.m + 1) * W.m + (int64_t)j * (W.m + 1);
  double2* hc = reinterpret_cast<double2*>(W.hcur) + (int64_t)s * (W.m + 1);
  if (i == j + 1) {
    if (second) return;
    double wn = strided_sum(W.pnorm + d.tile0, d.ntiles);
    wn = block_sum(wn, lds);
    if (threadIdx.x == 0) st.w2 = wn;
    return;
  }
  if (i < lo) {
    if (threadIdx.x == 0) {
      hcol[i] = make_double2(0.0, 0.0);
      hc[i] = make_double2(0.0, 0.0);
    }
    return;
  }
  const double2* part = reinterpret_cast<const double2*>(W.part) + d.pbase + (int64_t)i * d.ntiles;
  const double2 av = strided_sum2(part, d.ntiles);
  double ax = av.x, ay = av.y;
  ax = block_sum(ax, lds);
  ay = block_sum(ay, lds);
  if (threadIdx.x == 0) {
    const double c = W.cscale[(int64_t)s * (W.m + 1) + i];
    const double2 h = make_double2(c * ax, c * ay);
    hc[i] = h;
    if (second) {
      hcol[i].x += h.x;
      hcol[i].y += h.y;
    } else {
      hcol[i] = h;
    }
  }
}

// ------------------------------------------------------------ Arnoldi pass A
// MATVEC: w = c_j (H - s) u_j, written to u_{j+1}. Otherwise w = u_{j+1}
// (second Gram-Schmidt pass). Partial sums of conj(u_i) w for lo <= i <= j,
// and of ||w||^2, per tile.
// PRE (with !MATVEC): the first pass on w = c_j z already formed as z in
// u_{j+1} by an operator applied outside (the Q1 shared basis); w is scaled
// and stored back, then the same dots from i0 as the matvec pass.
template <typename T, int PPT, bool MATVEC>
__global__ __launch_bounds__(TPB) void k_arnoldi_a(Work W, int j, int i0, int pre) {
  __shared__ double2 red[NWAVE][MAXM + 1];
  j = dev_iter(W, j);
  if (j < 0) return;
  if (!MATVEC && !pre && W.reo_any && !W.reo_any[j]) return;  // no second pass at iteration j
  const bool first = MATVEC || pre;
  const int lo = first ? i0 : 0;
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysState_t& st = W.st[s];
    if (st.state != ST_ACTIVE) continue;
    if (!first && !st.reorth) continue;
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const double cj = W.cscale[(int64_t)s * (W.m + 1) + j];
    T* __restrict__ unew = tile_vec<T>(W, d, t, j + 1);
    const SGeo g = sgeo(d);
    const int dn = d.n;
    double2 w[PPT];
    double wn = 0.0;
    // complex64 in a tile-interleaved basis: point pairs with 16-byte accesses
    // (the matvec when the pairs stay in rows: n2 even, V's pairs aligned)
    bool paired = false;
    if constexpr (sizeof(T) == 8) {
      if (W.ilv && (!MATVEC || (!d.fem && (d.n2 & 1) == 0 && (d.off & 1) == 0))) {
        paired = true;
        T wv[PPT];
        if (!MATVEC) tile_load<T, PPT, true>(unew, t * W.tile, dn, wv);
#pragma unroll
        for (int k = 0; k < PPT / 2; ++k) {
          const int o = tpt<T>(2 * k);
          const int p = t * W.tile + o;
          double2 v0 = make_double2(0.0, 0.0), v1 = v0;
          if (MATVEC) {
            // (a pair past n computes point 0's stencil and is masked: no branch)
            stencil_pair_c64(reinterpret_cast<const float2*>(map_vec<T>(W, d, j)), W.V32, g,
                             (uint32_t)(p < dn ? p : 0), bmap(W), v0, v1);
            if (p >= dn) v0 = v1 = make_double2(0.0, 0.0);
          } else {
            v0 = to_d2(wv[2 * k]);
            v1 = to_d2(wv[2 * k + 1]);
          }
          if (MATVEC || pre) {
            v0.x *= cj;
            v0.y *= cj;
            v1.x *= cj;
            v1.y *= cj;
          }
          wv[2 * k] = from_d2<T>(v0);
          wv[2 * k + 1] = from_d2<T>(v1);
          // (n even here when MATVEC; otherwise the second point may be past n)
          w[2 * k] = p < dn ? to_d2(wv[2 * k]) : make_double2(0.0, 0.0);
          w[2 * k + 1] = p + 1 < dn ? to_d2(wv[2 * k + 1]) : make_double2(0.0, 0.0);
          if (p < dn) wn += w[2 * k].x * w[2 * k].x + w[2 * k].y * w[2 * k].y;
          if (p + 1 < dn) wn += w[2 * k + 1].x * w[2 * k + 1].x + w[2 * k + 1].y * w[2 * k + 1].y;
        }
        if (MATVEC || pre) tile_store<T, PPT, true>(unew, t * W.tile, dn, wv);
      }
    }
#pragma unroll
    for (int q = 0; q < PPT && !paired; ++q) {
      const int o = tpt<T>(q);  // the point within the tile
      const int p = t * W.tile + o;
      w[q] = make_double2(0.0, 0.0);
      if (p < dn) {
        if (MATVEC) {
          // (Q1 elements keep the plain layout: W.ilv = 0)
          double2 v = d.fem ? fem_point<T>(basis_vec<T>(W, d, j), d.n0, d.n1, d.n2, d.d2, d.d1, d.fmd, d.fmo,
                                           d.fkd, d.fko, d.fvol, vpot<T>(W, d.off + p), d.sre, d.sim, (uint32_t)p)
                            : stencil_point<T>(map_vec<T>(W, d, j), g, vpot<T>(W, g.off + p), (uint32_t)p, bmap(W));
          v.x *= cj;
          v.y *= cj;
          T vs = from_d2<T>(v);
          unew[o] = vs;
          w[q] = to_d2(vs);
        } else if (pre) {
          double2 v = to_d2(unew[o]);
          v.x *= cj;
          v.y *= cj;
          T vs = from_d2<T>(v);
          unew[o] = vs;
          w[q] = to_d2(vs);
        } else {
          w[q] = to_d2(unew[o]);
        }
        wn += w[q].x * w[q].x + w[q].y * w[q].y;
      }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // the projections conj(u_i) w in blocks of AU basis vectors: their loads
    // are issued together (a tall-skinny matrix-vector product), then AU
    // independent wave reductions; each dot is summed in the same order as
    // one vector at a time
    constexpr int AU = au_vectors<T, PPT>();
    auto project = [&](auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;
    int i = lo;
    for (; i + AU <= j + 1; i += AU) {
      T a[AU][PPT];
#pragma unroll
      for (int r = 0; r < AU; ++r) tile_load<T, PPT, FULL>(tile_vec<T>(W, d, t, i + r), t * W.tile, dn, a[r]);
      // (slots past n hold zeros in a and w: no guard, so the loop has no branch)
      double2 acc[AU];
#pragma unroll
      for (int r = 0; r < AU; ++r) {
        acc[r] = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const double2 c = cjmul(to_d2(a[r][q]), w[q]);
          acc[r].x += c.x;
          acc[r].y += c.y;
        }
      }
#pragma unroll
      for (int r = 0; r < AU; ++r) {
        acc[r].x = wave_sum(acc[r].x);
        acc[r].y = wave_sum(acc[r].y);
        if (lane == 0) red[wid][i + r] = acc[r];
      }
    }
    for (; i <= j; ++i) {
      T av[PPT];
      tile_load<T, PPT, FULL>(tile_vec<T>(W, d, t, i), t * W.tile, dn, av);
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        double2 a = to_d2(av[q]);
        double2 c = cjmul(a, w[q]);
        acc.x += c.x;
        acc.y += c.y;
      }
      acc.x = wave_sum(acc.x);
      acc.y = wave_sum(acc.y);
      if (lane == 0) red[wid][i] = acc;
    }
    };
    if (W.ilv) project(std::true_type{});
    else project(std::false_type{});
    wn = wave_sum(wn);
    if (lane == 0) red[wid][MAXM] = make_double2(wn, 0.0);
    __syncthreads();
    double2* part = reinterpret_cast<double2*>(W.part) + d.pbase;
    for (int i = lo + threadIdx.x; i <= j; i += TPB) {
      double2 a = make_double2(0.0, 0.0);
#pragma unroll
      for (int w2 = 0; w2 < NWAVE; ++w2) { a.x += red[w2][i].x; a.y += red[w2][i].y; }
      part[(int64_t)i * d.ntiles + t] = a;
    }
    if (threadIdx.x == 63) {
      double a = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NWAVE; ++w2) a += red[w2][MAXM].x;
      W.pnorm[item] = a;
    }
    __syncthreads();
  }
}

// Per-system Givens step (thread 0): h_{j+1,j} = beta, rotate column j,
// residual estimate |g_{j+1}|, convergence decision; at the end of the cycle
// the triangular solve R y = g.
__device__ void givens_per_pole(Work& W, int s, int j, int cycle, double beta) {
  SysState_t& st = W.st[s];
  const SysDesc& d = W.sys[s];
  const int m = W.m;
  double2* Hs = reinterpret_cast<double2*>(W.H) + (int64_t)s * (m + 1) * m;
  double2* col = Hs + (int64_t)j * (m + 1);
  double2* gcv = reinterpret_cast<double2*>(W.gc) + (int64_t)s * m;
  double2* gsv = reinterpret_cast<double2*>(W.gs) + (int64_t)s * m;
  double2* g = reinterpret_cast<double2*>(W.gvec) + (int64_t)s * (m + 1);
  double* cs = W.cscale + (int64_t)s * (m + 1);
  col[j + 1] = make_double2(beta, 0.0);
  // earlier rotations: (a, b) -> (conj(c) a + conj(s) b, -s a + c b)
  for (int i = 0; i < j; ++i) {
    const double2 c = gcv[i], sn = gsv[i];
    const double2 a = col[i], b = col[i + 1];
    const double2 t1 = cjmul(c, a), t2 = cjmul(sn, b);
    const double2 u1 = cmul(sn, a), u2 = cmul(c, b);
    col[i] = make_double2(t1.x + t2.x, t1.y + t2.y);
    col[i + 1] = make_double2(u2.x - u1.x, u2.y - u1.y);
  }
  const double2 a = col[j];
  const double den = sqrt(a.x * a.x + a.y * a.y + beta * beta);
  double2 c, sn;
  if (den > 0.0) {
    c = make_double2(a.x / den, a.y / den);
    sn = make_double2(beta / den, 0.0);
  } else {
    c = make_double2(1.0, 0.0);
    sn = make_double2(0.0, 0.0);
  }
  gcv[j] = c;
  gsv[j] = sn;
  col[j] = make_double2(den, 0.0);
  col[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = g[j];
  g[j + 1] = make_double2(-(sn.x * gj.x - sn.y * gj.y), -(sn.x * gj.y + sn.y * gj.x));
  g[j] = cjmul(c, gj);
  const double res = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
  cs[j + 1] = beta > 0.0 ? 1.0 / beta : 0.0;
  st.kcyc = j + 1;
  st.its += 1;
  // stop the cycle at the inner target (mixed path: a fixed reduction of the
  // cycle's starting residual) or at the outer target, whichever is larger
  const double target = fmax(W.inner_rtol * st.rnorm, 0.5 * d.tol * st.bnorm);
  const bool conv = res <= target || beta == 0.0 || !(res == res);
  if (conv || j + 1 == m) {
    const int k = j + 1;
    double2* y = reinterpret_cast<double2*>(W.y) + (int64_t)s * m;
    for (int r = k - 1; r >= 0; --r) {
      double2 acc = g[r];
      for (int q = r + 1; q < k; ++q) {
        const double2 tq = cmul(Hs[(int64_t)q * (m + 1) + r], y[q]);
        acc.x -= tq.x;
        acc.y -= tq.y;
      }
      const double2 dd = Hs[(int64_t)r * (m + 1) + r];
      const double dn = dd.x * dd.x + dd.y * dd.y;
      y[r] = dn > 0.0 ? make_double2((acc.x * dd.x + acc.y * dd.y) / dn, (acc.y * dd.x - acc.x * dd.y) / dn)
                      : make_double2(0.0, 0.0);
    }
    st.state = ST_FINISH;
  } else {
    atomicAdd(&W.counters[cycle * (m + 1) + j], 1);
  }
}

// Partial reorthogonalisation (shared-basis Lanczos; thread 0). The three-term
// recurrence with local orthogonalisation against v_{j-1}, v_j leaves the
// loss of orthogonality of v_{j+1} against v_k (k < j) to Simon's recurrence
//   beta_{j+1} w_{j+1,k} = beta_{k+1} w_{j,k+1} + (alpha_k - alpha_j) w_{j,k}
//                          + beta_k w_{j,k-1} - beta_j w_{j-1,k} + rounding,
// w_{j,j} = 1, w_{j+1,j} = eps1. When max_k |w_{j+1,k}| exceeds sqrt(u),
// v_{j+1} (and then v_{j+2}) get a full Gram-Schmidt pass against all earlier
// vectors, and the estimates of a reorthogonalised vector reset to eps1.
__device__ bool pro_decide(Work& W, ShiftWork& SW, int s, int j, double bj1) {
  // block-level: the estimates of row j+1 are independent across k
  __shared__ int reo_sh;
  const int m = W.m;
  const double u = 1.1102230246251565e-16;
  const double eps1 = sqrt((double)W.sys[s].n) * u;
  double* alpha = SW.alpha + (int64_t)s * m;
  double* betav = SW.beta + (int64_t)s * (m + 1);
  int32_t* flags = SW.flags + 4 * s;
  double* omega = SW.omega + (int64_t)s * 2 * (m + 1);
  double* wprev = omega + (int64_t)((j + 1) & 1) * (m + 1);  // row j-1, becomes row j+1
  double* wcur = omega + (int64_t)(j & 1) * (m + 1);         // row j
  if (threadIdx.x == 0) {
    const double2 hjj =
        reinterpret_cast<const double2*>(W.H)[(int64_t)s * (m + 1) * m + (int64_t)j * (m + 1) + j];
    alpha[j] = hjj.x;
    betav[j + 1] = bj1;
    if (j == 0) wcur[0] = 1.0;
  }
  __syncthreads();
  double an = 0.0;
  for (int k = threadIdx.x; k <= j; k += TPB) an = fmax(an, fabs(alpha[k]) + betav[k] + betav[k + 1]);
  // block max via the sum of a one-hot: reuse block_sum on squared maxima is
  // not exact, so take the max through LDS
  __shared__ double mx[NWAVE];
  for (int o = 32; o >= 1; o >>= 1) an = fmax(an, __shfl_xor(an, o, 64));
  if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = an;
  __syncthreads();
  double anorm = 0.0;
#pragma unroll
  for (int q = 0; q < NWAVE; ++q) anorm = fmax(anorm, mx[q]);
  const double bj = betav[j];
  const double aj = alpha[j];
  double worst = 0.0;
  double vals[4];
  int cnt = 0;
  for (int k = threadIdx.x; k < j; k += TPB) {
    const double wkp1 = wcur[k + 1];
    const double wk = wcur[k];
    const double wkm1 = k > 0 ? wcur[k - 1] : 0.0;
    const double wold = wprev[k];
    double v = betav[k + 1] * wkp1 + (alpha[k] - aj) * wk + (k > 0 ? betav[k] * wkm1 : 0.0) - bj * wold;
    v += copysign(2.0 * u * anorm, v);
    v = bj1 > 0.0 ? v / bj1 : 1.0;
    vals[cnt++ & 3] = v;
    worst = fmax(worst, fabs(v));
  }
  __syncthreads();  // every read of row j-1 precedes the writes of row j+1
  cnt = 0;
  for (int k = threadIdx.x; k < j; k += TPB) wprev[k] = vals[cnt++ & 3];
  for (int o = 32; o >= 1; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = worst;
  __syncthreads();
  if (threadIdx.x == 0) {
    double wmax = 0.0;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) wmax = fmax(wmax, mx[q]);
    wprev[j] = eps1;
    wprev[j + 1] = 1.0;
    const int force = flags[0];
    const bool reo = force || wmax > sqrt(u);
    if (reo) {
      flags[0] = force ? 0 : 1;  // the next vector gets a pass as well
      flags[1] += 1;
    }
    reo_sh = reo ? 1 : 0;
  }
  __syncthreads();
  const bool reo = reo_sh != 0;
  if (reo)
    for (int k = threadIdx.x; k <= j; k += TPB) wprev[k] = eps1;
  return reo;
}

// Block-level: Givens update of column j of (Hbar - s_p Itilde) for every
// pole sharing the basis; ends the Arnoldi process when every pole meets its
// target or j + 1 = m (the back substitution runs in k_shifted_backsub).
// `banded`: column j has no entries above row j - 1 (no second pass).
__device__ void givens_shifted(Work& W, ShiftWork& SW, int s, int j, double beta, bool banded) {
  __shared__ double lds[NWAVE];
  SysState_t& st = W.st[s];
  const int m = W.m;
  double* Hs = W.H + (int64_t)s * (m + 1) * m * 2;
  const double2* hcol = reinterpret_cast<const double2*>(Hs) + (int64_t)j * (m + 1);
  const double bn = st.bnorm;
  const int i_start = banded ? max(0, j - 2) : 0;
  double unconv = 0.0, wsum = 0.0;
  for (int p = SW.pole0[s] + threadIdx.x; p < SW.pole0[s + 1]; p += TPB) {
    double2* Rp = reinterpret_cast<double2*>(SW.R) + (int64_t)p * (m + 1) * m;
    double2* col = Rp + (int64_t)j * (m + 1);
    double2* gcv = reinterpret_cast<double2*>(SW.gc) + (int64_t)p * m;
    double2* gsv = reinterpret_cast<double2*>(SW.gs) + (int64_t)p * m;
    double2* g = reinterpret_cast<double2*>(SW.g) + (int64_t)p * (m + 1);
    const double2 sp = reinterpret_cast<const double2*>(SW.s)[p];
    double2 a;
    if (banded) {
      // column j holds rows j-1 and j only: the rotations j-2 and j-1 act on it,
      // in registers (rows j-2, j-1 of R receive the results)
      double2 am1 = j >= 1 ? hcol[j - 1] : make_double2(0.0, 0.0);
      double2 aj = make_double2(hcol[j].x - sp.x, hcol[j].y - sp.y);
      if (j >= 2) {
        const double2 c = gcv[j - 2], sn = gsv[j - 2];
        // (0, am1) -> (conj(s) am1, c am1)
        col[j - 2] = cjmul(sn, am1);
        am1 = cmul(c, am1);
      }
      if (j >= 1) {
        const double2 c = gcv[j - 1], sn = gsv[j - 1];
        const double2 t1 = cjmul(c, am1), t2 = cjmul(sn, aj);
        const double2 u1 = cmul(sn, am1), u2 = cmul(c, aj);
        col[j - 1] = make_double2(t1.x + t2.x, t1.y + t2.y);
        aj = make_double2(u2.x - u1.x, u2.y - u1.y);
      }
      a = aj;
    } else {
      for (int i = i_start; i <= j; ++i) col[i] = hcol[i];
      col[j].x -= sp.x;
      col[j].y -= sp.y;
      for (int i = i_start; i < j; ++i) {
        const double2 c = gcv[i], sn = gsv[i];
        const double2 aa = col[i], b = col[i + 1];
        const double2 t1 = cjmul(c, aa), t2 = cjmul(sn, b);
        const double2 u1 = cmul(sn, aa), u2 = cmul(c, b);
        col[i] = make_double2(t1.x + t2.x, t1.y + t2.y);
        col[i + 1] = make_double2(u2.x - u1.x, u2.y - u1.y);
      }
      a = col[j];
    }
    const double den = sqrt(a.x * a.x + a.y * a.y + beta * beta);
    double2 c, sn;
    if (den > 0.0) {
      c = make_double2(a.x / den, a.y / den);
      sn = make_double2(beta / den, 0.0);
    } else {
      c = make_double2(1.0, 0.0);
      sn = make_double2(0.0, 0.0);
    }
    gcv[j] = c;
    gsv[j] = sn;
    col[j] = make_double2(den, 0.0);
    const double2 gj = g[j];
    g[j + 1] = make_double2(-(sn.x * gj.x - sn.y * gj.y), -(sn.x * gj.y + sn.y * gj.x));
    g[j] = cjmul(c, gj);
    const double res = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
    SW.res[p] = bn > 0.0 ? res / bn : 0.0;
    const bool conv = res <= 0.5 * SW.tol[p] * bn || beta == 0.0 || !(res == res);
    if (conv) {
      if (SW.its[p] == 0) SW.its[p] = j + 1;
    } else {
      unconv += 1.0;
    }
    if (SW.cw) wsum += SW.cw[p] * res;
  }
  unconv = block_sum(unconv, lds);
  if (SW.cw && unconv > 0.0) {
    // the certified sum of the whole instance already meets its target: every
    // pole stops here (each one's share of the budget is not needed)
    wsum = block_sum(wsum, lds);
    if (wsum <= 0.5 * SW.tau * bn) {
      for (int p = SW.pole0[s] + threadIdx.x; p < SW.pole0[s + 1]; p += TPB)
        if (SW.its[p] == 0) SW.its[p] = j + 1;
      unconv = 0.0;
    }
  }
  if (threadIdx.x == 0) {
    const int k = j + 1;
    SW.full[(int64_t)s * m + j] = banded ? 0 : 1;
    Hs[(int64_t)j * (m + 1) * 2 + 2 * (j + 1)] = beta;  // h_{j+1,j}
    Hs[(int64_t)j * (m + 1) * 2 + 2 * (j + 1) + 1] = 0.0;
    W.cscale[(int64_t)s * (m + 1) + j + 1] = beta > 0.0 ? 1.0 / beta : 0.0;
    if (SW.lanczos) SW.beta[(int64_t)s * (m + 1) + j + 1] = beta;  // after any second pass
    st.kcyc = k;
    st.its = k;
    if (unconv == 0.0 || k == m) st.state = ST_FINISH;
    else atomicAdd(&W.counters[j], 1);
  }
}

// ------------------------------------------------------------ Arnoldi pass B
// u_{j+1} -= sum_{lo<=i<=j} hcur_i c_i u_i ; partial ||u_{j+1}||^2 per tile.
template <typename T, int PPT>
__global__ __launch_bounds__(TPB) void k_arnoldi_b(Work W, int j, int second, int i0) {
  __shared__ double lds[NWAVE];
  __shared__ double2 coef[MAXM];
  j = dev_iter(W, j);
  if (j < 0) return;
  if (second && W.reo_any && !W.reo_any[j]) return;
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysState_t& st = W.st[s];
    if (st.state != ST_ACTIVE) continue;
    if (second && !st.reorth) continue;
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const int lo = second ? 0 : i0;
    __syncthreads();
    for (int i = lo + threadIdx.x; i <= j; i += TPB) {
      const double2 h = reinterpret_cast<const double2*>(W.hcur)[(int64_t)s * (W.m + 1) + i];
      const double c = W.cscale[(int64_t)s * (W.m + 1) + i];
      coef[i] = make_double2(h.x * c, h.y * c);
    }
    __syncthreads();
    if (!second && t == 0 && threadIdx.x == 0 && W.reorth_mode <= 2) {
      // DGKS: a second pass when ||w - V h||^2 = ||w||^2 - sum |h_i|^2 (orthonormal
      // V) has dropped below eta^2 ||w||^2, i.e. when cancellation was severe
      double hs = 0.0;
      const double2* hc = reinterpret_cast<const double2*>(W.hcur) + (int64_t)s * (W.m + 1);
      hs = 0.0;
      for (int i = lo; i <= j; ++i) hs += hc[i].x * hc[i].x + hc[i].y * hc[i].y;
      const double w2 = st.w2;
      const bool reo = (W.reorth_mode == 2) || (W.reorth_mode == 1 && !(w2 - hs >= W.eta2 * w2));
      W.st[s].reorth = reo ? 1 : 0;
      if (reo && W.reo_any) W.reo_any[j] = 1;
    }
    T* __restrict__ unew = tile_vec<T>(W, d, t, j + 1);
    double wn = 0.0;
    auto update = [&](auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;
    double2 w[PPT];
    {
      T wv[PPT];
      tile_load<T, PPT, FULL>(unew, t * W.tile, d.n, wv);
#pragma unroll
      for (int q = 0; q < PPT; ++q) w[q] = to_d2(wv[q]);
    }
    // the loads of AU vectors are issued together; the updates keep the order i = lo .. j
    constexpr int AU = au_vectors<T, PPT>();
    int i = lo;
    for (; i + AU <= j + 1; i += AU) {
      T a[AU][PPT];
#pragma unroll
      for (int r = 0; r < AU; ++r) tile_load<T, PPT, FULL>(tile_vec<T>(W, d, t, i + r), t * W.tile, d.n, a[r]);
      // (slots past n hold zeros and are not stored: no guard, no branch)
#pragma unroll
      for (int r = 0; r < AU; ++r) {
        const double2 c = coef[i + r];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const double2 av = to_d2(a[r][q]);
          w[q].x -= c.x * av.x - c.y * av.y;
          w[q].y -= c.x * av.y + c.y * av.x;
        }
      }
    }
    for (; i <= j; ++i) {
      T av[PPT];
      tile_load<T, PPT, FULL>(tile_vec<T>(W, d, t, i), t * W.tile, d.n, av);
      const double2 c = coef[i];
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        double2 a = to_d2(av[q]);
        w[q].x -= c.x * a.x - c.y * a.y;
        w[q].y -= c.x * a.y + c.y * a.x;
      }
    }
    T wo[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = t * W.tile + tpt<T>(q);
      wo[q] = from_d2<T>(w[q]);
      if (p < d.n) {
        double2 vd = to_d2(wo[q]);
        wn += vd.x * vd.x + vd.y * vd.y;
      }
    }
    tile_store<T, PPT, FULL>(unew, t * W.tile, d.n, wo);
    };
    if (W.ilv) update(std::true_type{});
    else update(std::false_type{});
    wn = block_sum(wn, lds);
    if (threadIdx.x == 0) W.pnorm[item] = wn;
  }
}

// Grid S: the end of Arnoldi iteration j for system s. Reduces ||u_{j+1}||
// = h_{j+1,j}; on the first pass decides the second Gram-Schmidt pass
// (DGKS flag from pass B, or the Lanczos orthogonality estimate); when no
// second pass is due (or on the second pass), runs the Givens step: per pole,
// or for all poles of a shared basis.
__global__ __launch_bounds__(TPB) void k_end_iter(Work W, ShiftWork SW, int j, int second, int cycle) {
  __shared__ double lds[NWAVE];
  __shared__ int reo_sh;
  const int s = blockIdx.x;
  if (s >= W.S) return;
  if (second && W.reo_any && !W.reo_any[j]) return;
  SysState_t& st = W.st[s];
  if (st.state != ST_ACTIVE) return;
  if (second && !st.reorth) return;
  const SysDesc& d = W.sys[s];
  double bsq = 0.0;
  for (int tt = threadIdx.x; tt < d.ntiles; tt += TPB) bsq += W.pnorm[d.tile0 + tt];
  bsq = block_sum(bsq, lds);
  const double beta = sqrt(bsq);
  if (!second && SW.K > 0 && SW.lanczos) {
    const bool reo = pro_decide(W, SW, s, j, beta);
    if (threadIdx.x == 0) {
      st.reorth = reo ? 1 : 0;
      if (reo && W.reo_any) W.reo_any[j] = 1;
      reo_sh = reo ? 1 : 0;
      if (reo && SW.pause_mode) {
        // hand the second pass to the host: later launches of this chunk skip
        st.state = ST_PAUSED;
        SW.flags[4 * s + 2] = j;
        *SW.gpause = j;
      }
    }
  } else if (threadIdx.x == 0) {
    reo_sh = second ? 0 : st.reorth;
  }
  __syncthreads();
  if (reo_sh) return;
  if (SW.K > 0) {
    givens_shifted(W, SW, s, j, beta, SW.lanczos && !second);
  } else if (threadIdx.x == 0) {
    givens_per_pole(W, s, j, cycle, beta);
  }
}


// ------------------------------------------------------------ pipelined Lanczos
// The shared basis with H Hermitian, one streaming pass per iteration: the
// Lanczos vector u_{j+1} = H v_j - alpha_j v_j - beta_j v_{j-1} (unnormalised,
// v_i = c_i u_i) is formed point by point from z_j = H u_j, u_j and u_{j-1},
// at each point and at its stencil neighbours, and in the same pass
// z_{j+1} = H u_{j+1} is applied; the pass writes u_{j+1} and z_{j+1} and the
// partial sums of ||u_{j+1}||^2, <u_{j+1}, z_{j+1}> and <u_j, u_{j+1}>.
// alpha_{j+1} = c_{j+1}^2 <u_{j+1}, z_{j+1}> and beta_{j+1} = ||u_{j+1}|| then
// come from one per-system reduction (k_lz_end), which also runs the
// orthogonality estimate and the Givens step.

// z_i = H u_i for basis slot i (start of the solve, or after a second
// Gram-Schmidt pass), with partial <u_i, z_i> (partial slot 0) and ||u_i||^2.
template <int PPT>
__global__ __launch_bounds__(TPB) void k_lz_matvec(Work W, ShiftWork SW, int i, int zsel, int after_reorth) {
  __shared__ double lds[NWAVE];
  i = dev_iter(W, i);
  if (i < 0) return;
  if (after_reorth && W.reo_any && !W.reo_any[i - 1]) return;  // no second pass at iteration i - 1
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysState_t& st = W.st[s];
    if (st.state != ST_ACTIVE) continue;
    if (after_reorth && !st.reorth) continue;
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const double2* __restrict__ u = basis_vec<double2>(W, d, i);
    // zsel < 0: z is not stored (the tiled pass forms H u_j itself)
    double2* __restrict__ z = reinterpret_cast<double2*>(SW.zb) + (zsel < 0 ? 0 : zsel) * SW.zstride + d.xoff;
    double uzx = 0.0, uzy = 0.0, nn = 0.0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = t * W.tile + q * TPB + threadIdx.x;
      if (p < d.n) {
        const double2 c = u[p];
        const double2 hz = stencil_point<double2>(u, d, W.V64[d.off + p], (uint32_t)p);
        if (zsel >= 0) z[p] = hz;
        uzx += c.x * hz.x + c.y * hz.y;
        uzy += c.x * hz.y - c.y * hz.x;
        nn += c.x * c.x + c.y * c.y;
      }
    }
    uzx = block_sum(uzx, lds);
    uzy = block_sum(uzy, lds);
    nn = block_sum(nn, lds);
    if (threadIdx.x == 0) {
      reinterpret_cast<double2*>(W.part)[d.pbase + t] = make_double2(uzx, uzy);
      W.pnorm[item] = nn;
    }
  }
}

// Grid S: alpha_0 = c_0^2 <u_0, z_0> at the start of the solve.
__global__ __launch_bounds__(TPB) void k_lz_start(Work W, ShiftWork SW) {
  __shared__ double lds[NWAVE];
  const int s = blockIdx.x;
  if (s >= W.S) return;
  if (W.st[s].state != ST_ACTIVE) return;
  const SysDesc& d = W.sys[s];
  double ax = strided_sum2(reinterpret_cast<const double2*>(W.part) + d.pbase, d.ntiles).x;
  ax = block_sum(ax, lds);
  if (threadIdx.x == 0) {
    const double c0 = W.cscale[(int64_t)s * (W.m + 1)];
    SW.alpha[(int64_t)s * W.m] = c0 * c0 * ax;
  }
}

// True when the solve paused (for a second pass) at an iteration before j.
__device__ __forceinline__ bool paused_before(const ShiftWork& SW, int j) {
  if (!SW.pause_mode) return false;
  const int gp = *SW.gpause;
  return gp >= 0 && gp < j;
}

template <int PPT>
__global__ __launch_bounds__(TPB) void k_lz_step(Work W, ShiftWork SW, int j) {
  __shared__ double lds[NWAVE];
  const int m = W.m;
  if (paused_before(SW, j)) return;
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysState_t& st = W.st[s];
    if (st.state != ST_ACTIVE) continue;
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const double cj = W.cscale[(int64_t)s * (m + 1) + j];
    const double cjm = j > 0 ? W.cscale[(int64_t)s * (m + 1) + j - 1] : 0.0;
    const double ka = SW.alpha[(int64_t)s * m + j] * cj;
    const double kb = j > 0 ? SW.beta[(int64_t)s * (m + 1) + j] * cjm : 0.0;
    const double2* __restrict__ z = reinterpret_cast<const double2*>(SW.zb) + (j & 1) * SW.zstride + d.xoff;
    double2* __restrict__ zn = reinterpret_cast<double2*>(SW.zb) + ((j + 1) & 1) * SW.zstride + d.xoff;
    const double2* __restrict__ uj = basis_vec<double2>(W, d, j);
    const double2* __restrict__ ujm = basis_vec<double2>(W, d, j > 0 ? j - 1 : 0);
    double2* __restrict__ un = basis_vec<double2>(W, d, j + 1);
    const bool three = j > 0;
    auto U = [&](uint32_t q) -> double2 {
      const double2 a = z[q];
      const double2 b = uj[q];
      double2 r = make_double2(cj * a.x - ka * b.x, cj * a.y - ka * b.y);
      if (three) {
        const double2 c = ujm[q];
        r.x -= kb * c.x;
        r.y -= kb * c.y;
      }
      return r;
    };
    const uint32_t plane = (uint32_t)d.n1 * (uint32_t)d.n2;
    double uzx = 0.0, uzy = 0.0, oux = 0.0, ouy = 0.0, nn = 0.0;
#pragma unroll 2
    for (int q = 0; q < PPT; ++q) {
      const int pi = t * W.tile + q * TPB + threadIdx.x;
      if (pi < d.n) {
        const uint32_t p = (uint32_t)pi;
        const uint32_t r = fdiv(p, d.d2);
        const uint32_t k = p - r * (uint32_t)d.n2;
        const uint32_t i0 = fdiv(r, d.d1);
        const uint32_t jj = r - i0 * (uint32_t)d.n1;
        const double2 c = U(p);
        double2 nb2 = make_double2(0.0, 0.0), nb1 = nb2, nb0 = nb2;
        if (k > 0) { const double2 v = U(p - 1); nb2.x += v.x; nb2.y += v.y; }
        if (k + 1 < (uint32_t)d.n2) { const double2 v = U(p + 1); nb2.x += v.x; nb2.y += v.y; }
        if (jj > 0) { const double2 v = U(p - d.n2); nb1.x += v.x; nb1.y += v.y; }
        if (jj + 1 < (uint32_t)d.n1) { const double2 v = U(p + d.n2); nb1.x += v.x; nb1.y += v.y; }
        if (i0 > 0) { const double2 v = U(p - plane); nb0.x += v.x; nb0.y += v.y; }
        if (i0 + 1 < (uint32_t)d.n0) { const double2 v = U(p + plane); nb0.x += v.x; nb0.y += v.y; }
        const double a = d.diag + W.V64[d.off + p];
        double2 hz;
        hz.x = a * c.x - (d.c2 * nb2.x + d.c1 * nb1.x + d.c0 * nb0.x);
        hz.y = a * c.y - (d.c2 * nb2.y + d.c1 * nb1.y + d.c0 * nb0.y);
        un[p] = c;
        zn[p] = hz;
        const double2 u0 = uj[p];
        uzx += c.x * hz.x + c.y * hz.y;
        uzy += c.x * hz.y - c.y * hz.x;
        oux += u0.x * c.x + u0.y * c.y;
        ouy += u0.x * c.y - u0.y * c.x;
        nn += c.x * c.x + c.y * c.y;
      }
    }
    uzx = block_sum(uzx, lds);
    uzy = block_sum(uzy, lds);
    oux = block_sum(oux, lds);
    ouy = block_sum(ouy, lds);
    nn = block_sum(nn, lds);
    if (threadIdx.x == 0) {
      double2* part = reinterpret_cast<double2*>(W.part) + d.pbase;
      part[t] = make_double2(uzx, uzy);
      part[d.ntiles + t] = make_double2(oux, ouy);
      W.pnorm[item] = nn;
    }
  }
}


// k_lz_step with u_{j+1} staged in LDS for the tile and a halo of one row
// (n2 points) on each side, so the in-plane neighbours are read from LDS and
// only the neighbours in the adjacent planes are formed from global memory.
// Requires n2 <= HMAX for every system.
template <int PPT, int HMAX>
__global__ __launch_bounds__(TPB) void k_lz_step_lds(Work W, ShiftWork SW, int j) {
  __shared__ double lds[NWAVE];
  __shared__ double2 ub[TPB * PPT + 2 * HMAX];
  const int m = W.m;
  if (paused_before(SW, j)) return;
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysState_t& st = W.st[s];
    if (st.state != ST_ACTIVE) continue;
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const double cj = W.cscale[(int64_t)s * (m + 1) + j];
    const double cjm = j > 0 ? W.cscale[(int64_t)s * (m + 1) + j - 1] : 0.0;
    const double ka = SW.alpha[(int64_t)s * m + j] * cj;
    const double kb = j > 0 ? SW.beta[(int64_t)s * (m + 1) + j] * cjm : 0.0;
    const double2* __restrict__ z = reinterpret_cast<const double2*>(SW.zb) + (j & 1) * SW.zstride + d.xoff;
    double2* __restrict__ zn = reinterpret_cast<double2*>(SW.zb) + ((j + 1) & 1) * SW.zstride + d.xoff;
    const double2* __restrict__ uj = basis_vec<double2>(W, d, j);
    const double2* __restrict__ ujm = basis_vec<double2>(W, d, j > 0 ? j - 1 : 0);
    double2* __restrict__ un = basis_vec<double2>(W, d, j + 1);
    const bool three = j > 0;
    auto U = [&](uint32_t q) -> double2 {
      const double2 a = z[q];
      const double2 b = uj[q];
      double2 r = make_double2(cj * a.x - ka * b.x, cj * a.y - ka * b.y);
      if (three) {
        const double2 c = ujm[q];
        r.x -= kb * c.x;
        r.y -= kb * c.y;
      }
      return r;
    };
    const int T0 = t * W.tile;
    const int T1 = min(T0 + W.tile, d.n);
    const int L0 = max(0, T0 - d.n2);
    const int L1 = min(d.n, T1 + d.n2);
    __syncthreads();  // ub of the previous item is no longer read
    for (int q = L0 + (int)threadIdx.x; q < L1; q += TPB) ub[q - L0] = U((uint32_t)q);
    __syncthreads();
    const uint32_t plane = (uint32_t)d.n1 * (uint32_t)d.n2;
    double uzx = 0.0, uzy = 0.0, oux = 0.0, ouy = 0.0, nn = 0.0;
#pragma unroll 2
    for (int q = 0; q < PPT; ++q) {
      const int pi = T0 + q * TPB + threadIdx.x;
      if (pi < T1) {
        const uint32_t p = (uint32_t)pi;
        const uint32_t r = fdiv(p, d.d2);
        const uint32_t k = p - r * (uint32_t)d.n2;
        const uint32_t i0 = fdiv(r, d.d1);
        const uint32_t jj = r - i0 * (uint32_t)d.n1;
        const double2 c = ub[pi - L0];
        double2 nb2 = make_double2(0.0, 0.0), nb1 = nb2, nb0 = nb2;
        if (k > 0) { const double2 v = ub[pi - 1 - L0]; nb2.x += v.x; nb2.y += v.y; }
        if (k + 1 < (uint32_t)d.n2) { const double2 v = ub[pi + 1 - L0]; nb2.x += v.x; nb2.y += v.y; }
        if (jj > 0) { const double2 v = ub[pi - d.n2 - L0]; nb1.x += v.x; nb1.y += v.y; }
        if (jj + 1 < (uint32_t)d.n1) { const double2 v = ub[pi + d.n2 - L0]; nb1.x += v.x; nb1.y += v.y; }
        if (i0 > 0) { const double2 v = U(p - plane); nb0.x += v.x; nb0.y += v.y; }
        if (i0 + 1 < (uint32_t)d.n0) { const double2 v = U(p + plane); nb0.x += v.x; nb0.y += v.y; }
        const double a = d.diag + W.V64[d.off + p];
        double2 hz;
        hz.x = a * c.x - (d.c2 * nb2.x + d.c1 * nb1.x + d.c0 * nb0.x);
        hz.y = a * c.y - (d.c2 * nb2.y + d.c1 * nb1.y + d.c0 * nb0.y);
        un[p] = c;
        zn[p] = hz;
        const double2 u0 = uj[p];
        uzx += c.x * hz.x + c.y * hz.y;
        uzy += c.x * hz.y - c.y * hz.x;
        oux += u0.x * c.x + u0.y * c.y;
        ouy += u0.x * c.y - u0.y * c.x;
        nn += c.x * c.x + c.y * c.y;
      }
    }
    uzx = block_sum(uzx, lds);
    uzy = block_sum(uzy, lds);
    oux = block_sum(oux, lds);
    ouy = block_sum(ouy, lds);
    nn = block_sum(nn, lds);
    if (threadIdx.x == 0) {
      double2* part = reinterpret_cast<double2*>(W.part) + d.pbase;
      part[t] = make_double2(uzx, uzy);
      part[d.ntiles + t] = make_double2(oux, ouy);
      W.pnorm[item] = nn;
    }
  }
}

// k_lz_step marching along the slowest axis (2.5D blocking). A work item is
// a band of col_rows rows (n2 points each) of the (i1, i2) plane over col_L
// consecutive planes i0. Per plane, u_{j+1} is formed once for the band and
// one halo row on each side into LDS (two buffers: the plane being applied
// and the next one); the values of the planes before and after stay in
// registers. Each input of the item is read once, apart from the halo rows
// and the two planes bounding the range. Slots: h = threadIdx.x + q TPB over
// the (col_rows + 2) n2 points of the band with its halo rows.
// Items are ordered band-major over the plane ranges, so with col_nr a
// multiple of 8 the bands of one plane range share a compute die (blocks go
// round-robin over the 8 dies) and the halo rows they share hit its L2.
// Partial sums of the marching pass for iteration j, per item t, at parity
// j & 1: <u_{j+1}, z_{j+1}>, <u_j, u_{j+1}>, (||u_{j+1}||^2, 0) in three
// slots of col_cs entries from pbase + 3 (j & 1) col_cs (the fused pass of
// iteration j + 1 reads parity j while it writes parity j + 1).
__device__ __forceinline__ void lz_col_partials(const Work& W, int pbase, int ntiles, int np, int j, double& nn,
                                                double& uz, double& oux, double& ouy, double* l4) {
  const double2* pp = reinterpret_cast<const double2*>(W.part) + pbase + 3 * (j & 1) * ntiles;
  nn = strided_sum2(pp + 2 * ntiles, np).x;
  uz = strided_sum2(pp, np).x;
  const double2 o = strided_sum2(pp + ntiles, np);
  oux = o.x;
  ouy = o.y;
  block_sum4(nn, uz, oux, ouy, l4);
}

__device__ void lz_end_body(Work& W, ShiftWork& SW, int s, int j, int colparts);

// FUSED (systems that pause together for second passes; j >= 1): the S blocks
// after the items end iteration j - 1 of each system (lz_end_body), while every item block
// takes beta_j = ||u_j|| and alpha_j = c_j^2 <u_j, z_j> from the partial sums
// of iteration j - 1 itself (the same reduction in the same order, so the
// same values); j = m only ends iteration m - 1.
template <int KH, bool FUSED>
__global__ __launch_bounds__(TPB) void k_lz_step_col(Work W, ShiftWork SW, int j) {
  __shared__ double lds[NWAVE];
  __shared__ double l4[4 * NWAVE];
  __shared__ double2 ub[2][TPB * KH];
  const int m = W.m;
  const int nitems = FUSED ? (int)gridDim.x - W.S : (int)gridDim.x;
  if (FUSED && (int)blockIdx.x >= nitems) {
    lz_end_body(W, SW, (int)blockIdx.x - nitems, j - 1, 1);
    return;
  }
  if (FUSED && j >= m) return;
  if (paused_before(SW, j)) return;
  for (int item = blockIdx.x; item < SW.col_total; item += nitems) {
    // the system index is uniform: its descriptor is read once into scalar
    // registers (a reference would be re-read after every store, and each
    // re-read waits for the loads in flight)
    const int s = __builtin_amdgcn_readfirstlane(SW.col_sys ? SW.col_sys[item] : find_sys(SW.col_start, W.S, item));
    if (W.st[s].state != ST_ACTIVE) continue;
    const SysDesc& dref = W.sys[s];
    const int n0 = dref.n0, n1 = dref.n1, n2 = dref.n2;
    const FastDiv d2 = dref.d2;
    const double c0 = dref.c0, c1 = dref.c1, c2 = dref.c2, diag = dref.diag;
    const int cs = dref.col_cs, pbase = dref.pbase;  // partial-sum slot stride
    const int col_nr = dref.col_nr, col_rows = dref.col_rows, col_L = dref.col_L;
    const int64_t xoff = dref.xoff, voff = dref.off, bas = dref.basis;
    const int npts = dref.n;
    const int t = item - SW.col_start[s];
    const int band = t / col_nr;
    const int rng = t - band * col_nr;
    const int r0 = band * col_rows;
    const int r1 = min(n1, r0 + col_rows);
    const int ia = rng * col_L;
    const int ib = min(n0, ia + col_L);
    const int nslot = (r1 - r0 + 2) * n2;
    const uint32_t plane = (uint32_t)n1 * (uint32_t)n2;
    double cj, ka, kb;
    if (FUSED) {
      double nn, uz, ox, oy;
      lz_col_partials(W, pbase, cs, dref.col_n, j - 1, nn, uz, ox, oy, l4);
      const double bj = sqrt(nn);
      cj = bj > 0.0 ? 1.0 / bj : 0.0;
      ka = cj * cj * uz * cj;
      kb = bj * W.cscale[(int64_t)s * (m + 1) + j - 1];
    } else {
      cj = W.cscale[(int64_t)s * (m + 1) + j];
      const double cjm = j > 0 ? W.cscale[(int64_t)s * (m + 1) + j - 1] : 0.0;
      ka = SW.alpha[(int64_t)s * m + j] * cj;
      kb = j > 0 ? SW.beta[(int64_t)s * (m + 1) + j] * cjm : 0.0;
    }
    const double2* __restrict__ z = reinterpret_cast<const double2*>(SW.zb) + (j & 1) * SW.zstride + xoff;
    double2* __restrict__ zn = reinterpret_cast<double2*>(SW.zb) + ((j + 1) & 1) * SW.zstride + xoff;
    double2* const bvec = reinterpret_cast<double2*>(W.basis) + bas;
    const double2* __restrict__ uj = bvec + (int64_t)j * npts;
    const double2* __restrict__ ujm = bvec + (int64_t)(j > 0 ? j - 1 : 0) * npts;
    double2* __restrict__ un = bvec + (int64_t)(j + 1) * npts;
    const double* __restrict__ V = W.V64 + voff;
    const bool three = j > 0;
    // slot geometry: in-plane offset, row, column; valid = row inside the grid,
    // own = row inside the band
    uint32_t po[KH];
    int rw[KH], cl[KH];
    bool valid[KH], own[KH];
#pragma unroll
    for (int q = 0; q < KH; ++q) {
      const int h = (int)threadIdx.x + q * TPB;
      const int sr = (int)fdiv((uint32_t)h, d2);
      const int row = r0 - 1 + sr;
      cl[q] = h - sr * n2;
      rw[q] = row;
      valid[q] = h < nslot && row >= 0 && row < n1;
      own[q] = valid[q] && row >= r0 && row < r1;
      po[q] = valid[q] ? (uint32_t)row * (uint32_t)n2 + (uint32_t)cl[q] : 0u;
    }
    // inputs of one plane in flight (z_j, u_j, u_{j-1} at the slots, V at
    // the band), loaded one plane ahead of their use. Two buffers alternate
    // (the plane loop is unrolled by two), so loads in flight are never
    // copied between registers, which would wait for them.
    struct Raw {
      double2 z[KH], u[KH], m[KH];
      double v[KH];
    };
    auto fetch = [&](Raw& R, int i, bool halo) {
      const uint32_t base = (uint32_t)i * plane;
#pragma unroll
      for (int q = 0; q < KH; ++q) {
        R.z[q] = make_double2(0.0, 0.0);
        R.u[q] = R.z[q];
        R.m[q] = R.z[q];
        R.v[q] = 0.0;
        if (halo ? valid[q] : own[q]) {
          const uint32_t p = base + po[q];
          R.z[q] = z[p];
          R.u[q] = uj[p];
          if (three) R.m[q] = ujm[p];
          if (own[q]) R.v[q] = V[p];
        }
      }
    };
    // u_{j+1} = c_j z_j - alpha_j c_j u_j - beta_j c_{j-1} u_{j-1} from fetched inputs
    auto form = [&](const Raw& R, double2 (&dst)[KH], double2 (&ujv)[KH], double (&vv)[KH]) {
#pragma unroll
      for (int q = 0; q < KH; ++q) {
        dst[q] = make_double2(cj * R.z[q].x - ka * R.u[q].x - kb * R.m[q].x,
                              cj * R.z[q].y - ka * R.u[q].y - kb * R.m[q].y);
        ujv[q] = R.u[q];
        vv[q] = R.v[q];
      }
    };
    double2 prv[KH], cur[KH], nxt[KH], ujc[KH], ujn[KH];
    double vc[KH], vn[KH];
    Raw A, B;
    if (ia > 0) {
      fetch(A, ia - 1, false);
      form(A, prv, ujn, vn);
    } else {
#pragma unroll
      for (int q = 0; q < KH; ++q) prv[q] = make_double2(0.0, 0.0);
    }
    fetch(A, ia, true);
    __syncthreads();  // ub of the previous item is no longer read
    form(A, cur, ujc, vc);
#pragma unroll
    for (int q = 0; q < KH; ++q)
      if (valid[q]) ub[0][threadIdx.x + q * TPB] = cur[q];
    if (ia + 1 < n0) fetch(B, ia + 1, ia + 1 < ib);
    __syncthreads();
    int cb = 0;
    double uzx = 0.0, uzy = 0.0, oux = 0.0, ouy = 0.0, nn = 0.0;
    // plane i: X holds the inputs of plane i+1 (in flight), Y receives plane i+2
    auto plane_step = [&](int i, const Raw& X, Raw& Y) {
      if (i + 1 < n0) {
        // the next plane; with its halo rows when this item applies H to it
        form(X, nxt, ujn, vn);
        if (i + 1 < ib) {
#pragma unroll
          for (int q = 0; q < KH; ++q)
            if (valid[q]) ub[cb ^ 1][threadIdx.x + q * TPB] = nxt[q];
        }
        if (i + 2 < n0 && i + 2 <= ib) fetch(Y, i + 2, i + 2 < ib);
      } else {
#pragma unroll
        for (int q = 0; q < KH; ++q) nxt[q] = make_double2(0.0, 0.0);
      }
      const uint32_t base = (uint32_t)i * plane;
#pragma unroll
      for (int q = 0; q < KH; ++q) {
        if (own[q]) {
          const int h = (int)threadIdx.x + q * TPB;
          const double2 c = cur[q];
          double2 nb2 = make_double2(0.0, 0.0), nb1 = nb2;
          if (cl[q] > 0) { const double2 v = ub[cb][h - 1]; nb2.x += v.x; nb2.y += v.y; }
          if (cl[q] + 1 < n2) { const double2 v = ub[cb][h + 1]; nb2.x += v.x; nb2.y += v.y; }
          if (rw[q] > 0) { const double2 v = ub[cb][h - n2]; nb1.x += v.x; nb1.y += v.y; }
          if (rw[q] + 1 < n1) { const double2 v = ub[cb][h + n2]; nb1.x += v.x; nb1.y += v.y; }
          const double2 nb0 = make_double2(prv[q].x + nxt[q].x, prv[q].y + nxt[q].y);
          const uint32_t p = base + po[q];
          const double a = diag + vc[q];
          double2 hz;
          hz.x = a * c.x - (c2 * nb2.x + c1 * nb1.x + c0 * nb0.x);
          hz.y = a * c.y - (c2 * nb2.y + c1 * nb1.y + c0 * nb0.y);
          un[p] = c;
          zn[p] = hz;
          const double2 u0 = ujc[q];
          uzx += c.x * hz.x + c.y * hz.y;
          uzy += c.x * hz.y - c.y * hz.x;
          oux += u0.x * c.x + u0.y * c.y;
          ouy += u0.x * c.y - u0.y * c.x;
          nn += c.x * c.x + c.y * c.y;
        }
      }
      __syncthreads();  // buffer cb is read, buffer cb ^ 1 is written
#pragma unroll
      for (int q = 0; q < KH; ++q) {
        prv[q] = cur[q];
        cur[q] = nxt[q];
        ujc[q] = ujn[q];
        vc[q] = vn[q];
      }
      cb ^= 1;
    };
    for (int i = ia; i < ib; i += 2) {
      plane_step(i, B, A);
      if (i + 1 < ib) plane_step(i + 1, A, B);
    }
    uzx = block_sum(uzx, lds);
    uzy = block_sum(uzy, lds);
    oux = block_sum(oux, lds);
    ouy = block_sum(ouy, lds);
    nn = block_sum(nn, lds);
    if (threadIdx.x == 0) {
      double2* part = reinterpret_cast<double2*>(W.part) + pbase + 3 * (j & 1) * cs;
      part[t] = make_double2(uzx, uzy);
      part[cs + t] = make_double2(oux, ouy);
      part[2 * cs + t] = make_double2(nn, 0.0);
    }
  }
}

// Tiled marching pass (no stored z): the same iteration as k_lz_step_col, but
// H u_j is formed inside the pass, so z is neither read nor written (a point
// moves u_j, u_{j-1}, V and u_{j+1}: 56 B instead of 88 B). An item is a tile
// of TR x TC points of the (i1, i2) plane over col_L consecutive planes.
// Its region holds one halo row/column before the tile and two after: u_j is
// read on the whole region, u_{j+1} = c_j H u_j - alpha_j c_j u_j -
// beta_j c_{j-1} u_{j-1} is formed on the tile and one ring after it, and
// <u_{j+1}, H u_{j+1}> comes from the energy form of the Hermitian stencil,
//   <u, H u> = sum_i V_i |u_i|^2 + sum_a c_a sum_i (|u_i - u_{i+e_a}|^2
//              + [i_a = 0] |u_i|^2)   (u = 0 outside the grid),
// which needs only forward neighbours. Along the planes u_j of three planes
// and u_{j+1} of two stay in registers; in-plane neighbours come from LDS.
// Every global access is a raw buffer access: a slot outside the grid or the
// item's planes takes an offset past the buffer's end, which the hardware's
// range check turns into a zero load or a dropped store. The steps are
// therefore straight-line code, and the loads issued one step ahead are
// waited for only where they are used.
// Tile shapes: 16 x 32 points of the (i1, i2) plane for 3D grids, in blocks
// of 768 threads (12 waves, three per SIMD): the 19 x 35 region is one slot
// per thread, so a SIMD interleaves three waves' stencil arithmetic with the
// loads in flight (one block per CU at 128^3; with four waves of three slots
// each, every latency of a wave's chain was exposed). For 2D grids,
// relabelled (rows, 1, columns), strips of 253 points of a row (the region is
// the strip with one column before and two after: 256 slots, 256 threads).
constexpr int ZT_R = 16, ZT_C = 32, ZT_T = 768;
constexpr int ZS_C = 253, ZS_T = 256;
template <int TR, int TC, int NT> struct ZTile {
  static constexpr int W = TC + 3;                    // region width
  static constexpr int N = W * (TR > 1 ? TR + 3 : 1);  // region slots (TR = 1: no row halo, n1 = 1)
  static constexpr int KH = (N + NT - 1) / NT;
};
static_assert(ZTile<ZT_R, ZT_C, ZT_T>::KH == 1 && ZTile<1, ZS_C, ZS_T>::KH == 1, "one slot per thread");

// Sum over a block of NW waves; every thread gets the result. lds: NW doubles.
template <int NW>
__device__ __forceinline__ double block_sum_w(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += lds[w];
  return s;
}

constexpr uint32_t ZT_OOB = 0x80000000u;    // past the end of every buffer (records < 2^31 bytes)

typedef unsigned int zt_u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t zt_rsrc(const void* p, uint32_t bytes) {
  // raw buffer (stride 0), 32-bit data format: offsets >= bytes are out of
  // range. Base and size are uniform; reading them from the first lane puts
  // the descriptor in scalar registers whatever the compiler can prove (a
  // descriptor it takes for divergent costs a loop around every access).
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void* pu = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(pu, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
__device__ __forceinline__ double2 zt_load2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ double zt_load1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void zt_store2(__amdgpu_buffer_rsrc_t r, uint32_t off, double2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(zt_u32x4, v), r, off, 0, 0);
}

// lz_col_partials in a block of more than TPB threads, in two parts so that
// the loads of the partial sums go out before the loads of the planes (a
// wait for them then waits for nothing else). col_parts_load loads them when
// the system has at most TPB items (one per lead thread; raw buffer loads, so
// no branch: other threads read zeros); col_parts_reduce
// reduces exactly as lz_col_partials does (the same order, so the same
// values as the end-of-iteration block that reduces the same partial sums;
// one element per thread is strided_sum2's 0 + element), with every wave at
// the same two barriers.
struct ColParts {
  double2 nn, uz, o;  // elements of the three slots
};
__device__ __forceinline__ ColParts col_parts_load(const Work& W, int pbase, int ntiles, int np, int j) {
  const double2* pp = reinterpret_cast<const double2*>(W.part) + pbase + 3 * (j & 1) * ntiles;
  const __amdgpu_buffer_rsrc_t r = zt_rsrc(pp, (uint32_t)(3 * ntiles) * 16u);
  const int t = threadIdx.x;
  const bool in = np <= TPB && t < np;
  ColParts q;
  q.nn = zt_load2(r, in ? (uint32_t)(2 * ntiles + t) * 16u : ZT_OOB);
  q.uz = zt_load2(r, in ? (uint32_t)t * 16u : ZT_OOB);
  q.o = zt_load2(r, in ? (uint32_t)(ntiles + t) * 16u : ZT_OOB);
  return q;
}
__device__ __forceinline__ void col_parts_reduce(const ColParts& q, const Work& W, int pbase, int ntiles, int np,
                                                 int j, double& nn, double& uz, double& oux, double& ouy,
                                                 double* l4) {
  const bool lead = threadIdx.x < TPB;  // waves 0 .. NWAVE - 1 (wave-uniform)
  if (np <= TPB) {  // (threads past np, and every thread past TPB, hold zeros)
    nn = 0.0 + q.nn.x;
    uz = 0.0 + q.uz.x;
    oux = 0.0 + q.o.x;
    ouy = 0.0 + q.o.y;
  } else {
    const double2* pp = reinterpret_cast<const double2*>(W.part) + pbase + 3 * (j & 1) * ntiles;
    nn = lead ? strided_sum2(pp + 2 * ntiles, np).x : 0.0;
    uz = lead ? strided_sum2(pp, np).x : 0.0;
    const double2 o = lead ? strided_sum2(pp + ntiles, np) : make_double2(0.0, 0.0);
    oux = o.x;
    ouy = o.y;
  }
  oux = wave_sum(oux);
  ouy = wave_sum(ouy);
  nn = wave_sum(nn);
  uz = wave_sum(uz);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lead && lane == 0) {
    l4[wid] = nn;
    l4[NWAVE + wid] = uz;
    l4[2 * NWAVE + wid] = oux;
    l4[3 * NWAVE + wid] = ouy;
  }
  __syncthreads();
  nn = uz = oux = ouy = 0.0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) {
    nn += l4[w];
    uz += l4[NWAVE + w];
    oux += l4[2 * NWAVE + w];
    ouy += l4[3 * NWAVE + w];
  }
}

// The fields of a system's descriptor that the tiled pass reads, in registers.
struct TileSys {
  int32_t n, n0, n1, n2, col_cs, pbase, col_n, col_nr, col_L;
  int64_t off, basis;
  double c0, c1, c2, diag;
};
__device__ __forceinline__ TileSys tile_sys(const SysDesc& d) {
  return TileSys{d.n, d.n0, d.n1, d.n2, d.col_cs, d.pbase, d.col_n, d.col_nr, d.col_L,
                 d.off, d.basis, d.c0, d.c1, d.c2, d.diag};
}
// The same fields of the first system read with vector memory loads: their
// waits are counted in order with the other vector loads (a scalar load is
// waited for together with every scalar load in flight, the kernel arguments
// included), so they go out at the start of a launch with the state and the
// pause mark and are waited for where they are used: one round trip before
// the first loads of an item.
__device__ __forceinline__ uint32_t zt_ld4(const void* p) {
  return __builtin_amdgcn_raw_buffer_load_b32(zt_rsrc(p, 4u), 0, 0, 0);
}
__device__ __forceinline__ zt_u32x4 zt_ld16(const void* p) {
  return __builtin_amdgcn_raw_buffer_load_b128(zt_rsrc(p, 16u), 0, 0, 0);
}
struct SysChunks {
  zt_u32x4 a, b, c, d, e, f;  // (off, basis), (n, n0, n1, n2), (c0, c1), (c2, diag), (pbase, .., col_L, col_nr),
                              // (col_n, col_cs, ..)
};
static_assert(offsetof(SysDesc, basis) == offsetof(SysDesc, off) + 8, "SysDesc layout");
static_assert(offsetof(SysDesc, n0) == offsetof(SysDesc, n) + 4 && offsetof(SysDesc, n1) == offsetof(SysDesc, n) + 8 &&
                  offsetof(SysDesc, n2) == offsetof(SysDesc, n) + 12, "SysDesc layout");
static_assert(offsetof(SysDesc, c1) == offsetof(SysDesc, c0) + 8 && offsetof(SysDesc, diag) == offsetof(SysDesc, c2) + 8,
              "SysDesc layout");
static_assert(offsetof(SysDesc, col_L) == offsetof(SysDesc, pbase) + 8 &&
                  offsetof(SysDesc, col_nr) == offsetof(SysDesc, pbase) + 12 &&
                  offsetof(SysDesc, col_cs) == offsetof(SysDesc, col_n) + 4 &&
                  offsetof(SysDesc, col_n) + 16 <= sizeof(SysDesc),
              "SysDesc layout");
__device__ __forceinline__ SysChunks sys_chunks(const SysDesc* d) {
  const char* b = reinterpret_cast<const char*>(d);
  return SysChunks{zt_ld16(b + offsetof(SysDesc, off)), zt_ld16(b + offsetof(SysDesc, n)),
                   zt_ld16(b + offsetof(SysDesc, c0)), zt_ld16(b + offsetof(SysDesc, c2)),
                   zt_ld16(b + offsetof(SysDesc, pbase)), zt_ld16(b + offsetof(SysDesc, col_n))};
}
__device__ __forceinline__ uint32_t zt_rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t zt_rfl64(uint32_t lo, uint32_t hi) {
  return (uint64_t)zt_rfl(hi) << 32 | zt_rfl(lo);
}
__device__ __forceinline__ TileSys tile_sys(const SysChunks& c) {
  return TileSys{(int32_t)zt_rfl(c.b[0]), (int32_t)zt_rfl(c.b[1]), (int32_t)zt_rfl(c.b[2]), (int32_t)zt_rfl(c.b[3]),
                 (int32_t)zt_rfl(c.f[1]), (int32_t)zt_rfl(c.e[0]), (int32_t)zt_rfl(c.f[0]), (int32_t)zt_rfl(c.e[3]),
                 (int32_t)zt_rfl(c.e[2]), (int64_t)zt_rfl64(c.a[0], c.a[1]), (int64_t)zt_rfl64(c.a[2], c.a[3]),
                 __builtin_bit_cast(double, zt_rfl64(c.c[0], c.c[1])),
                 __builtin_bit_cast(double, zt_rfl64(c.c[2], c.c[3])),
                 __builtin_bit_cast(double, zt_rfl64(c.d[0], c.d[1])),
                 __builtin_bit_cast(double, zt_rfl64(c.d[2], c.d[3]))};
}

// At most 128 registers a lane (four waves per SIMD): a block that ends the
// previous iteration then shares a compute unit with an item (at 128^3, 257
// blocks on 256 units); with 150 registers one item waited until it had ended.
template <int TR, int TC, int NT, bool FUSED>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_lz_step_tile(Work W, ShiftWork SW, int j) {
  constexpr int KH = ZTile<TR, TC, NT>::KH;
  constexpr int ZT_W = ZTile<TR, TC, NT>::W;
  constexpr int ZT_N = ZTile<TR, TC, NT>::N;
  constexpr int NW = NT / 64;
  constexpr bool ROWS = TR > 1;  // the region has rows (TR = 1: n1 = 1)
  __shared__ double lds[NW];
  __shared__ double l4[4 * NWAVE];
  __shared__ double2 ub[2][KH * NT];
  __shared__ double2 wb[2][KH * NT];
  const int m = W.m;
  const int jarg = j;
  // one instance: its state, the pause mark and the fields of its descriptor
  // are loaded together at the start (one round trip before the item's first
  // loads; the launches of a captured schedule past convergence still return
  // after it)
  const bool S1 = W.S == 1;
  const uint32_t st0v = zt_ld4(&W.st[0].state);
  const uint32_t gpv = zt_ld4(SW.gpause);
  const SysChunks c0v = sys_chunks(W.sys);
  j = dev_iter(W, j);
  if (j < 0) return;
  if (!FUSED && jarg == JD_REC1 && blockIdx.x == 0 && threadIdx.x == 0) {
    // the pass after a captured second pass of iteration j - 1: the next fused
    // launch runs iteration j + 1 (no block of this launch reads this index)
    W.jdev[1] = SW.cap_next - (j + 1);
  }
  if (!FUSED && j >= m) return;
  // FUSED: blocks 0 .. S-1 end iteration j - 1 (one per system), the others
  // are the items. The end blocks come first so that they are dispatched
  // first: an item block fills a CU's wave slots, and an end block placed
  // after all items would wait for one of them to finish.
  const int iend = FUSED ? W.S : 0;
  const int nitems = (int)gridDim.x - iend;
  if (S1 && (int)__builtin_amdgcn_readfirstlane(st0v) != (int)ST_ACTIVE) return;  // (the end block would return too)
  if (FUSED && (int)blockIdx.x < iend) {
    // the end of iteration j - 1 takes TPB threads; the other waves leave
    // (a barrier waits only for the waves of the block that have not ended)
    if (threadIdx.x >= TPB) return;
    lz_end_body(W, SW, (int)blockIdx.x, j - 1, 1);
    return;
  }
  if (FUSED && j >= m) return;
  if (SW.pause_mode) {  // the solve paused at an earlier iteration
    const int gp = (int)__builtin_amdgcn_readfirstlane(gpv);
    if (gp >= 0 && gp < j) return;
  }
  const TileSys g0 = tile_sys(c0v);  // (scalar registers from here on)
  for (int item = (int)blockIdx.x - iend; item < SW.col_total; item += nitems) {
    int s = 0, t = item;
    TileSys g = g0;
    if (!S1) {
      s = __builtin_amdgcn_readfirstlane(SW.col_sys ? SW.col_sys[item] : find_sys(SW.col_start, W.S, item));
      if (W.st[s].state != ST_ACTIVE) continue;
      g = tile_sys(W.sys[s]);
      t = item - SW.col_start[s];
    }
    const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const double c0 = g.c0, c1 = g.c1, c2 = g.c2, diag = g.diag;
    const int cs = g.col_cs, pbase = g.pbase;
    const int np = __builtin_amdgcn_readfirstlane(g.col_n);
    ColParts cq{};
    if (FUSED && NT != TPB) cq = col_parts_load(W, pbase, cs, np, j - 1);
    const int col_nr = g.col_nr, col_L = g.col_L;
    const int64_t voff = g.off, bas = g.basis;
    const int npts = g.n;
    const int tile = t / col_nr;
    const int rng = t - tile * col_nr;
    const int ntc = (n2 + TC - 1) / TC;
    const int tr = tile / ntc;
    const int r0 = tr * TR;
    const int c0c = (tile - tr * ntc) * TC;
    const int ia = rng * col_L;
    const int ib = min(n0, ia + col_L);
    const uint32_t plane = (uint32_t)n1 * (uint32_t)n2;
    double cj = 0.0, ka = 0.0, kb = 0.0;  // set after the first loads are issued
    // u_{j-1} is read at j = 0 too (as u_0, finite), where kb = 0 removes it
    const double2* const bvec = reinterpret_cast<const double2*>(W.basis) + bas;
    const uint32_t vbytes = (uint32_t)npts * 16u;
    const __amdgpu_buffer_rsrc_t ru = zt_rsrc(bvec + (int64_t)j * npts, vbytes);
    const __amdgpu_buffer_rsrc_t rm = zt_rsrc(bvec + (int64_t)(j > 0 ? j - 1 : 0) * npts, vbytes);
    const __amdgpu_buffer_rsrc_t rn = zt_rsrc(bvec + (int64_t)(j + 1) * npts, vbytes);
    const __amdgpu_buffer_rsrc_t rv = zt_rsrc(W.V64 + voff, (uint32_t)npts * 8u);
    // slot geometry: in-plane offset; valid = inside the grid, fw = on the
    // tile or its forward ring (u_{j+1} formed), own = on the tile; eb = the
    // coefficients of the boundary edges before row 0 / column 0; hf, ho =
    // the slot, or an interior slot for slots whose neighbours are not read
    uint32_t po[KH];
    bool valid[KH], fw[KH], own[KH];
    double eb[KH];
    int hf[KH], ho[KH];
#pragma unroll
    for (int q = 0; q < KH; ++q) {
      const int h = (int)threadIdx.x + q * NT;
      const int rr = ROWS ? h / ZT_W : 1;
      const int cc = ROWS ? h - rr * ZT_W : h;
      const int row = ROWS ? r0 - 1 + rr : 0, col = c0c - 1 + cc;
      valid[q] = h < ZT_N && row >= 0 && row < n1 && col >= 0 && col < n2;
      fw[q] = valid[q] && rr >= 1 && rr <= TR + 1 && cc >= 1 && cc <= TC + 1;
      own[q] = valid[q] && rr >= 1 && rr <= TR && cc >= 1 && cc <= TC;
      po[q] = valid[q] ? (uint32_t)row * (uint32_t)n2 + (uint32_t)col : 0u;
      eb[q] = (row == 0 ? c1 : 0.0) + (col == 0 ? c2 : 0.0);
      hf[q] = fw[q] ? h : (ROWS ? ZT_W + 1 : 1);
      ho[q] = own[q] ? h : (ROWS ? ZT_W + 1 : 1);
    }
    const double2 zero = make_double2(0.0, 0.0);
    using Vec = double2[KH];
    using Sca = double[KH];
    // byte offset of plane i at the slots where sel holds (in: plane i is read)
    auto offs = [&](uint32_t (&o)[KH], int i, bool in, const bool (&sel)[KH], uint32_t esz) {
      const uint32_t base = in ? (uint32_t)i * plane : 0u;
#pragma unroll
      for (int q = 0; q < KH; ++q) o[q] = (in && sel[q]) ? (base + po[q]) * esz : ZT_OOB;
    };
    auto fetch_u = [&](Vec& U, int i, bool in) {
      uint32_t o[KH];
      offs(o, i, in && i >= 0 && i < n0, valid, 16u);
#pragma unroll
      for (int q = 0; q < KH; ++q) U[q] = zt_load2(ru, o[q]);
    };
    auto fetch_mv = [&](Vec& M, Sca& Vp, int i, bool in) {
      uint32_t o[KH], ov[KH];
      offs(o, i, in && i >= 0 && i < n0, fw, 16u);
      offs(ov, i, in && i >= 0 && i < n0, fw, 8u);
#pragma unroll
      for (int q = 0; q < KH; ++q) {
        M[q] = zt_load2(rm, o[q]);
        Vp[q] = zt_load1(rv, ov[q]);
      }
    };
    Vec Ua, Ub, Uc, Ud, Ma, Mb, Wa, Wb;
    Sca Va, Vb;
    double en = 0.0, oux = 0.0, ouy = 0.0, nn = 0.0;
    // step p: u_{j+1} of plane p + 1 (on the tile and its forward ring) and
    // the forward-difference terms of plane p. U0..U2 = u_j of planes p..p+2,
    // U3 receives plane p + 3; Mx, Vx = u_{j-1}, V of plane p + 1, My, Vy
    // receive plane p + 2; Wc = u_{j+1} of plane p, Wn receives plane p + 1.
    // Steps past the item's last plane change nothing.
    auto step = [&](int p, Vec& U0, Vec& U1, Vec& U2, Vec& U3, Vec& Mx, Vec& My, Sca& Vx, Sca& Vy, Vec& Wc,
                    Vec& Wn) {
      const int bu = (p + 1) & 1;
#pragma unroll
      for (int q = 0; q < KH; ++q) ub[bu][threadIdx.x + q * NT] = U1[q];
      fetch_u(U3, p + 3, p + 3 <= ib + 1);
      fetch_mv(My, Vy, p + 2, p + 2 <= ib);
      __syncthreads();  // ub[bu] is written; wb[p & 1] (plane p) is complete
      const bool form = p + 1 < n0 && p + 1 <= ib;
      const bool keep = p + 1 < ib;  // plane p + 1 belongs to the item
      const double ep = p + 1 == 0 ? c0 : 0.0;
      const uint32_t sbase = keep ? (uint32_t)(p + 1) * plane : 0u;
#pragma unroll
      for (int q = 0; q < KH; ++q) {
        const int h = hf[q];
        const double2 c = U1[q];
        const double2 l = ub[bu][h - 1], r = ub[bu][h + 1];
        const double2 a = ROWS ? ub[bu][h - ZT_W] : zero, b = ROWS ? ub[bu][h + ZT_W] : zero;
        const double2 nb2 = make_double2(l.x + r.x, l.y + r.y);
        const double2 nb1 = make_double2(a.x + b.x, a.y + b.y);
        const double2 nb0 = make_double2(U0[q].x + U2[q].x, U0[q].y + U2[q].y);
        const double d = diag + Vx[q];
        double2 hu;
        hu.x = d * c.x - (c2 * nb2.x + c1 * nb1.x + c0 * nb0.x);
        hu.y = d * c.y - (c2 * nb2.y + c1 * nb1.y + c0 * nb0.y);
        const bool f = form && fw[q];
        const double2 w = f ? make_double2(cj * hu.x - ka * c.x - kb * Mx[q].x, cj * hu.y - ka * c.y - kb * Mx[q].y)
                            : zero;
        const bool k = keep && own[q];
        zt_store2(rn, k ? (sbase + po[q]) * 16u : ZT_OOB, w);
        const double w2 = k ? w.x * w.x + w.y * w.y : 0.0;
        nn += w2;
        en += (Vx[q] + eb[q] + ep) * w2;
        oux += k ? c.x * w.x + c.y * w.y : 0.0;
        ouy += k ? c.x * w.y - c.y * w.x : 0.0;
        Wn[q] = w;
        wb[bu][threadIdx.x + q * NT] = w;
      }
      if (p >= ia && p < ib) {
        const int bw = p & 1;
#pragma unroll
        for (int q = 0; q < KH; ++q) {
          const int h = ho[q];
          const double2 c = Wc[q];
          const double2 r = wb[bw][h + 1], b = ROWS ? wb[bw][h + ZT_W] : zero, f = Wn[q];
          const double dx = c.x - r.x, dy = c.y - r.y;
          const double ex = c.x - b.x, ey = c.y - b.y;
          const double fx = c.x - f.x, fy = c.y - f.y;
          const double e = c2 * (dx * dx + dy * dy) + c1 * (ex * ex + ey * ey) + c0 * (fx * fx + fy * fy);
          en += own[q] ? e : 0.0;
        }
      }
    };
    __syncthreads();  // ub, wb of the previous item are no longer read
    fetch_u(Ua, ia - 1, true);
    fetch_u(Ub, ia, true);
    fetch_u(Uc, ia + 1, true);
    fetch_mv(Ma, Va, ia, true);
    // the loads of the first planes are in flight while the coefficients of
    // the iteration are reduced from the previous pass's partial sums (no
    // instruction that waits for a load moves above this point)
    __builtin_amdgcn_sched_barrier(0);
    if (FUSED) {
      double nn, uz, ox, oy;
      if (NT == TPB) lz_col_partials(W, pbase, cs, np, j - 1, nn, uz, ox, oy, l4);
      else col_parts_reduce(cq, W, pbase, cs, np, j - 1, nn, uz, ox, oy, l4);
      const double bj = sqrt(nn);
      cj = bj > 0.0 ? 1.0 / bj : 0.0;
      ka = cj * cj * uz * cj;
      kb = bj * W.cscale[(int64_t)s * (m + 1) + j - 1];
    } else {
      cj = W.cscale[(int64_t)s * (m + 1) + j];
      const double cjm = j > 0 ? W.cscale[(int64_t)s * (m + 1) + j - 1] : 0.0;
      ka = SW.alpha[(int64_t)s * m + j] * cj;
      kb = j > 0 ? SW.beta[(int64_t)s * (m + 1) + j] * cjm : 0.0;
    }
#pragma unroll
    for (int q = 0; q < KH; ++q) Wa[q] = zero;
    step(ia - 1, Ua, Ub, Uc, Ud, Ma, Mb, Va, Vb, Wa, Wb);
    // col_L further steps in groups of four (a fixed count: straight-line code)
    for (int g = 0, p = ia; g < (col_L + 3) / 4; ++g, p += 4) {
      step(p, Ub, Uc, Ud, Ua, Mb, Ma, Vb, Va, Wb, Wa);
      step(p + 1, Uc, Ud, Ua, Ub, Ma, Mb, Va, Vb, Wa, Wb);
      step(p + 2, Ud, Ua, Ub, Uc, Mb, Ma, Vb, Va, Wb, Wa);
      step(p + 3, Ua, Ub, Uc, Ud, Ma, Mb, Va, Vb, Wa, Wb);
    }
    en = block_sum_w<NW>(en, lds);
    oux = block_sum_w<NW>(oux, lds);
    ouy = block_sum_w<NW>(ouy, lds);
    nn = block_sum_w<NW>(nn, lds);
    if (threadIdx.x == 0) {
      double2* part = reinterpret_cast<double2*>(W.part) + pbase + 3 * (j & 1) * cs;
      part[t] = make_double2(en, 0.0);
      part[cs + t] = make_double2(oux, ouy);
      part[2 * cs + t] = make_double2(nn, 0.0);
    }
  }
}

// Grid S: end of pipelined iteration j (first pass). beta_{j+1} = ||u_{j+1}||,
// alpha_{j+1} = c_{j+1}^2 Re <u_{j+1}, z_{j+1}>; column j of Hbar is
// (beta_j, alpha_j, beta_{j+1}) at rows j-1, j, j+1. The orthogonality
// estimate (Simon's recurrence, as in pro_decide) and the measured local
// term c_j c_{j+1} <u_j, u_{j+1}> decide a second Gram-Schmidt pass;
// otherwise the banded Givens step of every pole runs. A single block with a
// chain of small dependent steps: every global value the block needs (tile
// partials, the alpha/beta/omega history, the poles' rotations) is loaded
// up front, so the chain costs about two memory round trips. Requires
// poles per instance <= TPB for the register path (others take a loop).
__device__ void lz_end_body(Work& W, ShiftWork& SW, int s, int j, int colparts) {
  __shared__ double l4[4 * NWAVE];
  __shared__ double hist[4][MAXM + 2];  // alpha, beta, omega row j, omega row j-1
  __shared__ int reo_sh;
  const int tid = threadIdx.x;
  const int m = W.m;
  SysState_t& st = W.st[s];
  // round trip 1: state, descriptor, pole range
  const int state = st.state;
  const SysDesc& d = W.sys[s];
  const int ntiles = d.ntiles, pbase = d.pbase, tile0 = d.tile0, np = colparts ? d.col_n : d.ntiles;
  const int npts = d.n;
  const int p0 = SW.pole0[s], p1 = SW.pole0[s + 1];
  if (state != ST_ACTIVE) return;
  if (SW.pause_mode) {
    const int gp = *SW.gpause;
    if (gp >= 0 && gp < j) return;  // the solve paused at an earlier iteration
  }
  double* alpha = SW.alpha + (int64_t)s * m;
  double* betav = SW.beta + (int64_t)s * (m + 1);
  double* omega = SW.omega + (int64_t)s * 2 * (m + 1);
  double* wprev = omega + (int64_t)((j + 1) & 1) * (m + 1);  // row j-1, becomes row j+1
  double* wcur = omega + (int64_t)(j & 1) * (m + 1);         // row j
  if (j == 0 && tid == 0) wcur[0] = 1.0;                     // omega_{0,0}
  // round trip 2: everything else (the partial sums are reduced below)
  double nn, uz, oux, ouy;
  if (!colparts) {
    const double2* part = reinterpret_cast<const double2*>(W.part) + pbase;
    nn = strided_sum(W.pnorm + tile0, np);
    uz = strided_sum2(part, np).x;
    const double2 ou = strided_sum2(part + ntiles, np);
    oux = ou.x;
    ouy = ou.y;
  }
  if (tid <= j) {
    hist[0][tid] = alpha[tid];
    hist[1][tid] = betav[tid];
    hist[2][tid] = j == 0 ? 1.0 : wcur[tid];
    hist[3][tid] = tid < j ? wprev[tid] : 0.0;
  }
  double cj = 0.0;
  int force = 0;
  if (tid == 0) {
    cj = W.cscale[(int64_t)s * (m + 1) + j];
    force = SW.flags[4 * s];
  }
  // the first TPB poles: rotations j-2, j-1 and g_j in registers
  const int p = p0 + tid;
  const bool hasp = p < p1;
  double2 cA = make_double2(1.0, 0.0), sA = make_double2(0.0, 0.0), cB = cA, sB = sA, gj = sA, sp = sA;
  double tolp = 0.0;
  int itsp = 1;
  if (hasp) {
    const double2* gcv = reinterpret_cast<const double2*>(SW.gc) + (int64_t)p * m;
    const double2* gsv = reinterpret_cast<const double2*>(SW.gs) + (int64_t)p * m;
    if (j >= 2) {
      cA = gcv[j - 2];
      sA = gsv[j - 2];
    }
    if (j >= 1) {
      cB = gcv[j - 1];
      sB = gsv[j - 1];
    }
    gj = reinterpret_cast<const double2*>(SW.g)[(int64_t)p * (m + 1) + j];
    sp = reinterpret_cast<const double2*>(SW.s)[p];
    tolp = SW.tol[p];
    itsp = SW.its[p];
  }
  // partial sums; then max_{k<j} |alpha_k| + beta_k + beta_{k+1} (the k = j
  // term needs beta_{j+1})
  if (colparts)
    lz_col_partials(W, pbase, d.col_cs, np, j, nn, uz, oux, ouy, l4);
  else
    block_sum4(nn, uz, oux, ouy, l4);
  const double beta1 = sqrt(nn);
  const double c1 = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
  const double aj = hist[0][j], bj = hist[1][j];
  double an = tid < j ? fabs(hist[0][tid]) + hist[1][tid] + hist[1][tid + 1] : 0.0;
  an = block_max(an, l4);
  const double anorm = fmax(an, fabs(aj) + bj + beta1);
  // column j of Hbar (its rows above j - 1 are zero; a second pass adds to them)
  double2* hcol = reinterpret_cast<double2*>(W.H) + (int64_t)s * (m + 1) * m + (int64_t)j * (m + 1);
  for (int i = tid; i + 1 < j; i += TPB) hcol[i] = make_double2(0.0, 0.0);
  if (tid == 0) {
    if (j > 0) hcol[j - 1] = make_double2(bj, 0.0);
    hcol[j] = make_double2(aj, 0.0);
    betav[j + 1] = beta1;
  }
  // omega row j+1 from rows j and j-1
  const double u = 1.1102230246251565e-16;
  const double eps1 = sqrt((double)npts) * u;
  double v = 0.0;
  if (tid < j) {
    const int k = tid;
    v = hist[1][k + 1] * hist[2][k + 1] + (hist[0][k] - aj) * hist[2][k] +
        (k > 0 ? hist[1][k] * hist[2][k - 1] : 0.0) - bj * hist[3][k];
    v += copysign(2.0 * u * anorm, v);
    v = beta1 > 0.0 ? v / beta1 : 1.0;
  }
  const double wmax = block_max(fabs(v), l4);
  if (tid == 0) {
    const bool est = force || wmax > sqrt(u);
    const double loc = cj * c1 * sqrt(oux * oux + ouy * ouy);  // local loss beyond sqrt(u)
    const bool reo = est || loc > 1.4901161193847656e-08;
    if (est) {
      SW.flags[4 * s] = force ? 0 : 1;  // an estimate-driven pass covers the next vector too
      SW.flags[4 * s + 1] += 1;
    }
    st.reorth = reo ? 1 : 0;
    if (reo && W.reo_any) W.reo_any[j] = 1;
    if (reo && SW.pause_mode) {
      st.state = ST_PAUSED;
      SW.flags[4 * s + 2] = j;
      *SW.gpause = j;
    }
    reo_sh = reo ? 1 : 0;
  }
  __syncthreads();
  const bool reo = reo_sh != 0;
  // a reorthogonalised vector has estimates eps1 against all earlier ones
  if (tid < j) wprev[tid] = reo ? eps1 : v;
  if (tid == 0) {
    wprev[j] = eps1;
    wprev[j + 1] = 1.0;
  }
  if (reo) return;  // the second pass follows, then k_lz_end_second
  if (tid == 0 && j + 1 < m) alpha[j + 1] = c1 * c1 * uz;
  // banded Givens step of every pole: column j holds beta_j (row j-1) and
  // alpha_j - s_p (row j); rotations j-2 and j-1 act on it, then the new
  // rotation j annihilates beta_{j+1}
  const double bn = st.bnorm;
  double unconv = 0.0, wsum = 0.0;
  for (int q = p; q < p1; q += TPB) {
    if (q != p) {  // poles beyond the first TPB: load here
      const double2* gcv = reinterpret_cast<const double2*>(SW.gc) + (int64_t)q * m;
      const double2* gsv = reinterpret_cast<const double2*>(SW.gs) + (int64_t)q * m;
      cA = j >= 2 ? gcv[j - 2] : make_double2(1.0, 0.0);
      sA = j >= 2 ? gsv[j - 2] : make_double2(0.0, 0.0);
      cB = j >= 1 ? gcv[j - 1] : make_double2(1.0, 0.0);
      sB = j >= 1 ? gsv[j - 1] : make_double2(0.0, 0.0);
      gj = reinterpret_cast<const double2*>(SW.g)[(int64_t)q * (m + 1) + j];
      sp = reinterpret_cast<const double2*>(SW.s)[q];
      tolp = SW.tol[q];
      itsp = SW.its[q];
    }
    double2* col = reinterpret_cast<double2*>(SW.R) + (int64_t)q * (m + 1) * m + (int64_t)j * (m + 1);
    double2 am1 = make_double2(j >= 1 ? bj : 0.0, 0.0);
    double2 a = make_double2(aj - sp.x, -sp.y);
    if (j >= 2) {
      col[j - 2] = cjmul(sA, am1);  // (0, am1) -> (conj(s) am1, c am1)
      am1 = cmul(cA, am1);
    }
    if (j >= 1) {
      const double2 t1 = cjmul(cB, am1), t2 = cjmul(sB, a);
      const double2 u1 = cmul(sB, am1), u2 = cmul(cB, a);
      col[j - 1] = make_double2(t1.x + t2.x, t1.y + t2.y);
      a = make_double2(u2.x - u1.x, u2.y - u1.y);
    }
    const double den = sqrt(a.x * a.x + a.y * a.y + beta1 * beta1);
    double2 c, sn;
    if (den > 0.0) {
      c = make_double2(a.x / den, a.y / den);
      sn = make_double2(beta1 / den, 0.0);
    } else {
      c = make_double2(1.0, 0.0);
      sn = make_double2(0.0, 0.0);
    }
    reinterpret_cast<double2*>(SW.gc)[(int64_t)q * m + j] = c;
    reinterpret_cast<double2*>(SW.gs)[(int64_t)q * m + j] = sn;
    col[j] = make_double2(den, 0.0);
    double2* g = reinterpret_cast<double2*>(SW.g) + (int64_t)q * (m + 1);
    const double2 gn = make_double2(-(sn.x * gj.x - sn.y * gj.y), -(sn.x * gj.y + sn.y * gj.x));
    g[j + 1] = gn;
    g[j] = cjmul(c, gj);
    const double res = sqrt(gn.x * gn.x + gn.y * gn.y);
    SW.res[q] = bn > 0.0 ? res / bn : 0.0;
    const bool conv = res <= 0.5 * tolp * bn || beta1 == 0.0 || !(res == res);
    if (conv) {
      if (itsp == 0) SW.its[q] = j + 1;
    } else {
      unconv += 1.0;
    }
    if (SW.cw) wsum += SW.cw[q] * res;
  }
  double z1 = 0.0, z2 = 0.0;
  block_sum4(unconv, wsum, z1, z2, l4);
  if (SW.cw && unconv > 0.0 && wsum <= 0.5 * SW.tau * bn) {
    // the certified sum of the whole instance already meets its target
    for (int q = p; q < p1; q += TPB)
      if (SW.its[q] == 0) SW.its[q] = j + 1;
    unconv = 0.0;
  }
  if (tid == 0) {
    const int k = j + 1;
    SW.full[(int64_t)s * m + j] = 0;
    double* Hs = W.H + (int64_t)s * (m + 1) * m * 2;
    Hs[(int64_t)j * (m + 1) * 2 + 2 * (j + 1)] = beta1;  // h_{j+1,j}
    Hs[(int64_t)j * (m + 1) * 2 + 2 * (j + 1) + 1] = 0.0;
    W.cscale[(int64_t)s * (m + 1) + j + 1] = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
    st.kcyc = k;
    st.its = k;
    if (unconv == 0.0 || k == m) st.state = ST_FINISH;
    else atomicAdd(&W.counters[j], 1);
  }
}

__global__ __launch_bounds__(TPB) void k_lz_end(Work W, ShiftWork SW, int j, int colparts) {
  if ((int)blockIdx.x >= W.S) return;
  lz_end_body(W, SW, blockIdx.x, j, colparts);
}

// Grid S: end of pipelined iteration j after a second Gram-Schmidt pass
// (z_{j+1} was recomputed): beta_{j+1}, alpha_{j+1} from the new partials,
// then the Givens step of every pole on the full column.
__global__ __launch_bounds__(TPB) void k_lz_end_second(Work W, ShiftWork SW, int j) {
  __shared__ double lds[NWAVE];
  j = dev_iter(W, j);
  if (j < 0) return;
  const int s = blockIdx.x;
  if (s >= W.S) return;
  if (W.reo_any && !W.reo_any[j]) return;
  SysState_t& st = W.st[s];
  if (st.state != ST_ACTIVE || !st.reorth) return;
  const SysDesc& d = W.sys[s];
  const int m = W.m;
  const double2* part = reinterpret_cast<const double2*>(W.part) + d.pbase;
  double nn = strided_sum(W.pnorm + d.tile0, d.ntiles);
  double uz = strided_sum2(part, d.ntiles).x;
  nn = block_sum(nn, lds);
  uz = block_sum(uz, lds);
  const double beta1 = sqrt(nn);
  const double c1 = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
  if (threadIdx.x == 0 && j + 1 < m) SW.alpha[(int64_t)s * m + j + 1] = c1 * c1 * uz;
  givens_shifted(W, SW, s, j, beta1, false);
}

// Shared basis, after the last iteration: back substitution R_p y_p = g_p per
// pole (one wave per pole, rows in sequence, the row sums across lanes).
__global__ __launch_bounds__(TPB) void k_shifted_backsub(Work W, ShiftWork SW) {
  __shared__ double2 band[NWAVE][4][MAXM];
  const int m = W.m;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int p = blockIdx.x * NWAVE + wid;
  if (p >= SW.K) return;
  const int s = SW.pinst[p];
  const int k = W.st[s].kcyc;
  const int32_t* full = SW.full + (int64_t)s * m;
  const double2* Rp = reinterpret_cast<const double2*>(SW.R) + (int64_t)p * (m + 1) * m;
  const double2* g = reinterpret_cast<const double2*>(SW.g) + (int64_t)p * (m + 1);
  double2* y = reinterpret_cast<double2*>(SW.y) + (int64_t)p * m;
  int anyfull = 0;
  for (int q = lane; q < k; q += 64) anyfull |= full[q];
  // Galerkin (FOM) iterate of a pole that missed its target: the square
  // system (H_k - s_p I) y = ||b|| e_1 has the same rotations 0..k-2 as the
  // least-squares one; its last pivot is c_{k-1} R_{k-1,k-1} and the last
  // right-hand side entry g_{k-1} / conj(c_{k-1}), so y_{k-1} is the
  // least-squares one divided by |c_{k-1}|^2 and the rest follows by the same
  // back substitution
  const bool fom = SW.fom && k > 0 && SW.its[p] == 0;
  double lastscale = 1.0;
  if (fom) {
    const double2 c = reinterpret_cast<const double2*>(SW.gc)[(int64_t)p * m + k - 1];
    lastscale = c.x * c.x + c.y * c.y;
  }
  if (!__any(anyfull)) {
    // no second pass: R has three diagonals, y_r = (g_r - R_{r,r+1} y_{r+1}
    // - R_{r,r+2} y_{r+2}) / R_rr. The wave stages the band and g in LDS,
    // then one lane runs the recurrence.
    double2(*bd)[MAXM] = band[wid];
    for (int r = lane; r < k; r += 64) {
      // the reciprocal pivot 1 / R_rr (0 for a zero pivot), formed in parallel
      double2 dd = Rp[(int64_t)r * (m + 1) + r];
      if (r == k - 1) dd = make_double2(dd.x * lastscale, dd.y * lastscale);
      const double dn = dd.x * dd.x + dd.y * dd.y;
      bd[0][r] = dn > 0.0 ? make_double2(dd.x / dn, -dd.y / dn) : make_double2(0.0, 0.0);
      bd[1][r] = r + 1 < k ? Rp[(int64_t)(r + 1) * (m + 1) + r] : make_double2(0.0, 0.0);
      bd[2][r] = r + 2 < k ? Rp[(int64_t)(r + 2) * (m + 1) + r] : make_double2(0.0, 0.0);
      bd[3][r] = g[r];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) {
      double2 y1 = make_double2(0.0, 0.0), y2 = y1;  // y_{r+1}, y_{r+2}
      for (int r = k - 1; r >= 0; --r) {
        const double2 t1 = cmul(bd[1][r], y1), t2 = cmul(bd[2][r], y2);
        const double2 acc = make_double2(bd[3][r].x - (t1.x + t2.x), bd[3][r].y - (t1.y + t2.y));
        const double2 yr = cmul(acc, bd[0][r]);
        y[r] = yr;
        if (fom && r == k - 1) reinterpret_cast<double2*>(SW.gnext)[p] = make_double2(-yr.x, -yr.y);
        y2 = y1;
        y1 = yr;
      }
    }
    return;
  }
  for (int r = k - 1; r >= 0; --r) {
    double ax = 0.0, ay = 0.0;
    for (int q = r + 1 + lane; q < k; q += 64) {
      // a banded column q holds R entries in rows q-2..q only
      if (q > r + 2 && !full[q]) continue;
      const double2 tq = cmul(Rp[(int64_t)q * (m + 1) + r], y[q]);
      ax += tq.x;
      ay += tq.y;
    }
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    if (lane == 0) {
      const double2 acc = make_double2(g[r].x - ax, g[r].y - ay);
      double2 dd = Rp[(int64_t)r * (m + 1) + r];
      if (r == k - 1) dd = make_double2(dd.x * lastscale, dd.y * lastscale);
      const double dn = dd.x * dd.x + dd.y * dd.y;
      y[r] = dn > 0.0 ? make_double2((acc.x * dd.x + acc.y * dd.y) / dn, (acc.y * dd.x - acc.x * dd.y) / dn)
                      : make_double2(0.0, 0.0);
      if (fom && r == k - 1) reinterpret_cast<double2*>(SW.gnext)[p] = make_double2(-y[r].x, -y[r].y);
    }
    __threadfence_block();
  }
}

// Grid S: z_s = sum_{p in s} w_p y_p in pole order.
// The weights are staged in LDS with a flag that leaves out a pole finished
// by a per-pole solve, so the loads of y for consecutive poles are independent.
__global__ __launch_bounds__(TPB) void k_shifted_z(Work W, ShiftWork SW) {
  __shared__ double2 wl[TPB];
  __shared__ int kl[TPB];
  const int s = blockIdx.x;
  if (s >= W.S) return;
  const int m = W.m;
  const int k = W.st[s].kcyc;
  const int q0 = SW.pole0[s], q1 = SW.pole0[s + 1];
  for (int c0 = q0; c0 < q1; c0 += TPB) {
    const int nc = min(TPB, q1 - c0);
    __syncthreads();
    if ((int)threadIdx.x < nc) {
      const int q = c0 + threadIdx.x;
      kl[threadIdx.x] = !(SW.fb_skip && SW.its[q] == 0);  // 0: finished by a per-pole solve
      wl[threadIdx.x] = reinterpret_cast<const double2*>(SW.w)[q];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += TPB) {
      double2 zi = c0 == q0 ? make_double2(0.0, 0.0) : reinterpret_cast<double2*>(SW.z)[(int64_t)s * m + i];
      const double2* yi = reinterpret_cast<const double2*>(SW.y) + (int64_t)c0 * m + i;
#pragma unroll 8
      for (int c = 0; c < nc; ++c) {
        const double2 tz = cmul(wl[c], yi[(int64_t)c * m]);
        zi.x += kl[c] ? tz.x : 0.0;
        zi.y += kl[c] ? tz.y : 0.0;
      }
      reinterpret_cast<double2*>(SW.z)[(int64_t)s * m + i] = zi;
    }
  }
}

// Grid S: a paused solve becomes active again (its second pass follows).
__global__ __launch_bounds__(64) void k_resume(Work W, ShiftWork SW) {
  const int s = blockIdx.x;
  if (s >= W.S || threadIdx.x != 0) return;
  if (W.st[s].state == ST_PAUSED) W.st[s].state = ST_ACTIVE;
  SW.flags[4 * s + 2] = -1;
  if (s == 0) {
    // a captured schedule keeps the paused iteration for its second pass
    if (W.jdev) W.jdev[0] = *SW.gpause;
    *SW.gpause = -1;
  }
}

// Captured schedules: no pass pending, no launch lost (a kernel, so that a
// graph records no memset).
__global__ __launch_bounds__(64) void k_cap_init(Work W) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    W.jdev[0] = -1;
    W.jdev[1] = 0;
  }
}

// Grid S: per-instance reset of the pole least-squares data and the
// reorthogonalisation state.
__global__ __launch_bounds__(TPB) void k_shifted_init(Work W, ShiftWork SW) {
  const int s = blockIdx.x;
  if (s >= W.S) return;
  const double bn = W.st[s].bnorm;
  if (threadIdx.x == 0) {
    SW.flags[4 * s] = 0;
    SW.flags[4 * s + 1] = 0;
    SW.flags[4 * s + 2] = -1;
    if (s == 0) *SW.gpause = -1;
    SW.beta[(int64_t)s * (W.m + 1)] = 0.0;
  }
  for (int p = SW.pole0[s] + threadIdx.x; p < SW.pole0[s + 1]; p += TPB) {
    double2* g = reinterpret_cast<double2*>(SW.g) + (int64_t)p * (W.m + 1);
    for (int i = 0; i <= W.m; ++i) g[i] = make_double2(0.0, 0.0);
    g[0] = make_double2(bn, 0.0);
    bool on = bn > 0.0;
    if (SW.restart) {
      // pole p solves (H - s_p) x = gam_p b: weight w_p gam_p; its target
      // tol_p ||psi|| / |gam_p| in the norm of b
      on = on && SW.miss[p] != 0;
      const double2 ga = reinterpret_cast<const double2*>(SW.gam)[p];
      const double2 w0 = reinterpret_cast<const double2*>(SW.w0)[p];
      const double ag = sqrt(ga.x * ga.x + ga.y * ga.y);
      reinterpret_cast<double2*>(const_cast<double*>(SW.w))[p] =
          on ? make_double2(w0.x * ga.x - w0.y * ga.y, w0.x * ga.y + w0.y * ga.x) : make_double2(0.0, 0.0);
      const_cast<double*>(SW.tol)[p] = on && ag > 0.0 ? SW.tol0[p] * SW.bn0[s] / (ag * bn) : 1.0;
    }
    SW.its[p] = on ? 0 : 1;
    SW.res[p] = on ? 1.0 : 0.0;
  }
}

// ------------------------------------------------------------ restart cycles
// Grid S, after the first cycle of a step (fom = 1): the poles that missed
// their target (residual gnext_p u_k) start the restarts with gam_p = gnext_p;
// their residual is reported as that of the Galerkin iterate. ||psi|| and
// the iterations so far are kept per instance.
__global__ __launch_bounds__(TPB) void k_rs_begin(Work W, ShiftWork SW, int32_t* __restrict__ miss,
                                                  double* __restrict__ gam, double* __restrict__ bn0,
                                                  int32_t* __restrict__ kbase, int32_t* __restrict__ hasmiss) {
  const int s = blockIdx.x;
  if (s >= W.S) return;
  const SysState_t& st = W.st[s];
  const int k = st.kcyc;
  const double bn = st.bnorm;
  const double ck = k > 0 ? W.cscale[(int64_t)s * (W.m + 1) + k] : 0.0;
  const double bk = ck > 0.0 ? 1.0 / ck : 0.0;  // ||u_k||
  int any = 0;
  for (int p = SW.pole0[s] + threadIdx.x; p < SW.pole0[s + 1]; p += TPB) {
    const bool ms = SW.its[p] == 0 && bn > 0.0 && k > 0;
    const double2 gn = ms ? reinterpret_cast<const double2*>(SW.gnext)[p] : make_double2(0.0, 0.0);
    miss[p] = ms ? 1 : 0;
    reinterpret_cast<double2*>(gam)[p] = gn;
    if (ms) SW.res[p] = sqrt(gn.x * gn.x + gn.y * gn.y) * bk / bn;
    any |= ms ? 1 : 0;
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) {
    bn0[s] = bn;
    kbase[s] = k;
    hasmiss[s] = any;
  }
}

// Grid S, after restart cycle R (the cycle's arrays) of a step whose arrays
// are SW: a pole of the cycle that met its target reports its iterations
// and residual gam_p |g| in the norm of psi; one that missed again carries
// gam_p gnext_p into the next cycle.
__global__ __launch_bounds__(TPB) void k_rs_merge(Work W, ShiftWork SW, ShiftWork R, int32_t* __restrict__ miss,
                                                  double* __restrict__ gam, const double* __restrict__ bn0,
                                                  int32_t* __restrict__ kbase, int32_t* __restrict__ hasmiss) {
  const int s = blockIdx.x;
  if (s >= W.S) return;
  const SysState_t& st = W.st[s];
  const int k = st.kcyc;
  const double bn = st.bnorm;
  const double ck = k > 0 ? W.cscale[(int64_t)s * (W.m + 1) + k] : 0.0;
  const double bk = ck > 0.0 ? 1.0 / ck : 0.0;
  const double b0 = bn0[s];
  const int kb = kbase[s];
  int any = 0;
  for (int p = SW.pole0[s] + threadIdx.x; p < SW.pole0[s + 1]; p += TPB) {
    if (!miss[p]) continue;
    double2 ga = reinterpret_cast<const double2*>(gam)[p];
    if (R.its[p] > 0) {
      SW.its[p] = kb + R.its[p];
      SW.res[p] = sqrt(ga.x * ga.x + ga.y * ga.y) * R.res[p] * bn / b0;
      miss[p] = 0;
    } else {
      const double2 gn = reinterpret_cast<const double2*>(R.gnext)[p];
      ga = make_double2(ga.x * gn.x - ga.y * gn.y, ga.x * gn.y + ga.y * gn.x);
      reinterpret_cast<double2*>(gam)[p] = ga;
      SW.res[p] = sqrt(ga.x * ga.x + ga.y * ga.y) * bk / b0;
      any = 1;
    }
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) {
    kbase[s] = kb + k;
    hasmiss[s] = any;
  }
}

// The next cycle's right-hand side: u_k of every instance that still has
// poles to finish, zero elsewhere (such instances finish at once).
__global__ __launch_bounds__(TPB) void k_rs_rhs(Work W, const int32_t* __restrict__ hasmiss,
                                                double2* __restrict__ rhs) {
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const bool on = hasmiss[s] != 0;
    const double2* __restrict__ u = basis_vec<double2>(W, d, on ? W.st[s].kcyc : 0);
    double2* __restrict__ r = rhs + d.off;
    const int pend = min((t + 1) * W.tile, d.n);
    for (int p = t * W.tile + (int)threadIdx.x; p < pend; p += TPB) r[p] = on ? u[p] : make_double2(0.0, 0.0);
  }
}

// ------------------------------------------------------------ end of cycle
// x (+)= sum_{i<k} y_i c_i u_i  (FP64), systems in ST_FINISH.
template <typename T, int PPT>
__global__ __launch_bounds__(TPB) void k_update_x(Work W) {
  __shared__ double2 coef[MAXM];
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysState_t& st = W.st[s];
    if (st.state != ST_FINISH) continue;
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const int k = st.kcyc;
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += TPB) {
      const double2 yv = reinterpret_cast<const double2*>(W.y)[(int64_t)s * W.m + i];
      const double c = W.cscale[(int64_t)s * (W.m + 1) + i];
      coef[i] = make_double2(yv.x * c, yv.y * c);
    }
    __syncthreads();
    double2* __restrict__ x = reinterpret_cast<double2*>(W.x) + d.xoff;
    double2 acc[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = t * W.tile + tpt<T>(q);
      acc[q] = (p < d.n && !st.first) ? x[p] : make_double2(0.0, 0.0);
    }
    // the loads of AU vectors are issued together; the sums keep the order i = 0 .. k - 1
    constexpr int AU = au_vectors<T, PPT>();
    auto accumulate = [&](auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;
    int i = 0;
    for (; i + AU <= k; i += AU) {
      T a[AU][PPT];
#pragma unroll
      for (int r = 0; r < AU; ++r) tile_load<T, PPT, FULL>(tile_vec<T>(W, d, t, i + r), t * W.tile, d.n, a[r]);
      // (slots past n hold zeros and are not stored: no guard, no branch)
#pragma unroll
      for (int r = 0; r < AU; ++r) {
        const double2 c = coef[i + r];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const double2 av = to_d2(a[r][q]);
          acc[q].x += c.x * av.x - c.y * av.y;
          acc[q].y += c.x * av.y + c.y * av.x;
        }
      }
    }
    for (; i < k; ++i) {
      T av[PPT];
      tile_load<T, PPT, FULL>(tile_vec<T>(W, d, t, i), t * W.tile, d.n, av);
      const double2 c = coef[i];
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        const double2 a = to_d2(av[q]);
        acc[q].x += c.x * a.x - c.y * a.y;
        acc[q].y += c.x * a.y + c.y * a.x;
      }
    }
    };
    if (W.ilv) accumulate(std::true_type{});
    else accumulate(std::false_type{});
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = t * W.tile + tpt<T>(q);
      if (p < d.n) x[p] = acc[q];
    }
  }
}

// r = b - (H - s) x in FP64; u_0 = r; partial ||r||^2. Systems in ST_FINISH.
template <typename T, int PPT>
__global__ __launch_bounds__(TPB) void k_residual(Work W, const double2* __restrict__ rhs0,
                                                  const double2* __restrict__ rhs1) {
  __shared__ double lds[NWAVE];
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysState_t& st = W.st[s];
    if (st.state != ST_FINISH) continue;
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const double2* __restrict__ b = (d.rhs_sel ? rhs1 : rhs0) + d.off;
    const double2* __restrict__ x = reinterpret_cast<const double2*>(W.x) + d.xoff;
    T* __restrict__ u0 = tile_vec<T>(W, d, t, 0);
    const SGeo g = sgeo(d);  // (in registers: d would be re-read after each store)
    const int dn = d.n, fem = d.fem;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = t * W.tile + q * TPB + threadIdx.x;
      if (p < dn) {
        const double2 hx =
            fem ? fem_point<double2>(x, d.n0, d.n1, d.n2, d.d2, d.d1, d.fmd, d.fmo, d.fkd, d.fko, d.fvol,
                                     W.V64[g.off + p], d.sre, d.sim, (uint32_t)p)
                : stencil_point_f64(x, g.n0, g.n1, g.n2, g.d2, g.d1, g.c0, g.c1, g.c2, g.diag, W.V64[g.off + p],
                                    g.sre, g.sim, (uint32_t)p);
        const double2 bp = b[p];
        const double2 r = make_double2(bp.x - hx.x, bp.y - hx.y);
        u0[q * TPB + threadIdx.x] = from_d2<T>(r);
        acc += r.x * r.x + r.y * r.y;
      }
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) W.pnorm[item] = acc;
  }
}

// Per system (ST_FINISH): explicit relative residual, done or restart.
__global__ __launch_bounds__(TPB) void k_restart(Work W, int cycle) {
  __shared__ double lds[NWAVE];
  const int s = blockIdx.x;
  if (s >= W.S) return;
  SysState_t& st = W.st[s];
  if (st.state != ST_FINISH) return;
  const SysDesc& d = W.sys[s];
  double acc = strided_sum(W.pnorm + d.tile0, d.ntiles);
  acc = block_sum(acc, lds);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(acc);
  st.cycles += 1;
  st.first = 0;
  st.rho = st.bnorm > 0.0 ? rn / st.bnorm : 0.0;
  const bool done = st.rho <= d.tol || st.cycles >= W.max_cycles || rn == 0.0 || !(rn == rn);
  if (done) {
    st.state = ST_DONE;
    if (!(st.rho <= d.tol)) atomicAdd(&W.counters[W.max_cycles * (W.m + 1) + 1], 1);
    return;
  }
  st.rnorm = rn;
  st.kcyc = 0;
  double2* g = reinterpret_cast<double2*>(W.gvec) + (int64_t)s * (W.m + 1);
  for (int i = 0; i <= W.m; ++i) g[i] = make_double2(0.0, 0.0);
  g[0] = make_double2(rn, 0.0);
  W.cscale[(int64_t)s * (W.m + 1)] = 1.0 / rn;
  st.state = ST_ACTIVE;
  atomicAdd(&W.counters[W.max_cycles * (W.m + 1)], 1);
  (void)cycle;
}


// out = sum_{i<k} z_i c_i u_i in FP64, per instance (system) of W.
template <typename T, int PPT>
__global__ __launch_bounds__(TPB) void k_combine_out(Work W, ShiftWork SW, double2* __restrict__ out, int accumulate) {
  __shared__ double2 coef[MAXM];
  int sprev = -1;
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysDesc& d = W.sys[s];
    const int k = W.st[s].kcyc;
    if (s != sprev) {
      __syncthreads();
      for (int i = threadIdx.x; i < k; i += TPB) {
        const double2 zi = reinterpret_cast<const double2*>(SW.z)[(int64_t)s * W.m + i];
        const double c = W.cscale[(int64_t)s * (W.m + 1) + i];
        coef[i] = make_double2(zi.x * c, zi.y * c);
      }
      __syncthreads();
      sprev = s;
    }
    const int t = item - d.tile0;
    const int n = d.n;
    const int64_t off = d.off;
    const T* __restrict__ u0 = basis_vec<T>(W, d, 0);
    double2 acc[PPT];
    bool in[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      acc[q] = make_double2(0.0, 0.0);
      in[q] = t * W.tile + q * TPB + (int)threadIdx.x < n;
    }
    const int p0 = t * W.tile + (int)threadIdx.x;
    // four basis vectors per step: their loads are in flight together; the
    // accumulation order per point stays i = 0, 1, ..., k - 1
    constexpr int U = 4;
    int i = 0;
    for (; i + U <= k; i += U) {
      T a[U][PPT];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const T* __restrict__ ui = u0 + (int64_t)(i + r) * n;
#pragma unroll
        for (int q = 0; q < PPT; ++q) a[r][q] = in[q] ? ui[p0 + q * TPB] : T{};
      }
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const double2 c = coef[i + r];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const double2 v = to_d2(a[r][q]);
          acc[q].x += c.x * v.x - c.y * v.y;
          acc[q].y += c.x * v.y + c.y * v.x;
        }
      }
    }
    for (; i < k; ++i) {
      const T* __restrict__ ui = u0 + (int64_t)i * n;
      const double2 c = coef[i];
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        if (in[q]) {
          const double2 v = to_d2(ui[p0 + q * TPB]);
          acc[q].x += c.x * v.x - c.y * v.y;
          acc[q].y += c.x * v.y + c.y * v.x;
        }
      }
    }
    if (accumulate) {
      // a restart cycle adds to the sums of the earlier cycles
#pragma unroll
      for (int q = 0; q < PPT; ++q)
        if (in[q]) {
          const double2 o = out[off + p0 + q * TPB];
          acc[q].x += o.x;
          acc[q].y += o.y;
        }
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q)
      if (in[q]) out[off + p0 + q * TPB] = acc[q];
  }
}

// ------------------------------------------------------------ explicit solutions
// The shared-basis solve never forms the pole solutions x_p = V_k y_p; the
// pole sum is V_k z. To certify a step by explicit FP64 residuals (the bound
// ||x_p - x_p*|| <= ||r_p|| / dist(s_p, spec H) holds for the normal matrix
// H - s_p, Section 3.1) the solutions are formed here and the residuals
// r_p = b - (H - s_p) x_p computed from them, in FP64.

// Poles per launch of k_form_x (their coefficients are staged in LDS).
constexpr int XG = 16;

// x_p (+)= sum_{i<k} a_p y_{p,i} c_i u_i in FP64 for the poles
// p = pole0[s] + g0 + g (g < XG) of every instance s, x_p at X + xoff[p].
// First cycle (gam = miss = null): a_p = 1, x_p written. Restart cycle:
// a_p = gam_p and only poles with miss[p] take part, adding to x_p (the
// cycle solved (H - s_p) d = gam_p b' for them). Dynamic LDS: XG * m complex.
template <int PPT>
__global__ __launch_bounds__(TPB) void k_form_x(Work W, ShiftWork SW, double2* __restrict__ X,
                                                const int64_t* __restrict__ xoff, int g0,
                                                const double* __restrict__ gam, const int32_t* __restrict__ miss) {
  extern __shared__ double2 xcoef[];
  int sprev = -1, np = 0, k = 0;
  uint32_t on = 0;
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysDesc& d = W.sys[s];
    const int q0 = SW.pole0[s] + g0;
    if (s != sprev) {
      k = W.st[s].kcyc;
      np = max(0, min(XG, SW.pole0[s + 1] - q0));
      on = 0;
      for (int g = 0; g < np; ++g)
        if (!miss || miss[q0 + g]) on |= 1u << g;
      __syncthreads();
      for (int e = threadIdx.x; e < np * k; e += TPB) {
        const int g = e / k, i = e - g * k;
        const int p = q0 + g;
        const double2 a = gam ? reinterpret_cast<const double2*>(gam)[p] : make_double2(1.0, 0.0);
        const double2 ay = cmul(a, reinterpret_cast<const double2*>(SW.y)[(int64_t)p * W.m + i]);
        const double c = W.cscale[(int64_t)s * (W.m + 1) + i];
        xcoef[g * W.m + i] = make_double2(ay.x * c, ay.y * c);
      }
      __syncthreads();
      sprev = s;
    }
    if (on == 0) continue;
    const int t = item - d.tile0;
    const double2* __restrict__ u0 = basis_vec<double2>(W, d, 0);
#pragma unroll 1
    for (int q = 0; q < PPT; ++q) {
      const int pt = t * W.tile + q * TPB + (int)threadIdx.x;
      if (pt >= d.n) break;
      double2 acc[XG];
#pragma unroll
      for (int g = 0; g < XG; ++g) acc[g] = make_double2(0.0, 0.0);
      // four basis vectors per step: their loads are in flight together
      constexpr int U = 4;
      int i = 0;
      for (; i + U <= k; i += U) {
        double2 a[U];
#pragma unroll
        for (int r = 0; r < U; ++r) a[r] = u0[(int64_t)(i + r) * d.n + pt];
#pragma unroll
        for (int r = 0; r < U; ++r)
#pragma unroll
          for (int g = 0; g < XG; ++g)
            if (g < np) {
              const double2 c = xcoef[g * W.m + i + r];
              acc[g].x += c.x * a[r].x - c.y * a[r].y;
              acc[g].y += c.x * a[r].y + c.y * a[r].x;
            }
      }
      for (; i < k; ++i) {
        const double2 a = u0[(int64_t)i * d.n + pt];
#pragma unroll
        for (int g = 0; g < XG; ++g)
          if (g < np) {
            const double2 c = xcoef[g * W.m + i];
            acc[g].x += c.x * a.x - c.y * a.y;
            acc[g].y += c.x * a.y + c.y * a.x;
          }
      }
#pragma unroll
      for (int g = 0; g < XG; ++g) {
        if (!((on >> g) & 1u)) continue;
        double2* __restrict__ x = X + xoff[q0 + g];
        if (miss) {
          const double2 o = x[pt];
          acc[g].x += o.x;
          acc[g].y += o.y;
        }
        x[pt] = acc[g];
      }
    }
  }
}

// Partial sums of ||b - (H - s_p) x_p||^2 over each tile, for every pole p of
// every instance, in FP64 with the solved operator (the instance's stencil,
// centering included): part[poff[p] + t] for tile t of the instance.
template <int PPT>
__global__ __launch_bounds__(TPB) void k_x_resid(Work W, ShiftWork SW, const double2* __restrict__ b,
                                                 const double2* __restrict__ X, const int64_t* __restrict__ xoff,
                                                 const int32_t* __restrict__ poff, double* __restrict__ part) {
  __shared__ double lds[NWAVE];
  for (int item = blockIdx.x; item < W.total_tiles; item += gridDim.x) {
    const int s = item_sys(W, item);
    const SysDesc& d = W.sys[s];
    const int t = item - d.tile0;
    const double2* __restrict__ bs = b + d.off;
    for (int p = SW.pole0[s]; p < SW.pole0[s + 1]; ++p) {
      const double2* __restrict__ x = X + xoff[p];
      const double sre = SW.s[2 * p], sim = SW.s[2 * p + 1];
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        const int pt = t * W.tile + q * TPB + (int)threadIdx.x;
        if (pt < d.n) {
          const double2 hx = stencil_point_f64(x, d.n0, d.n1, d.n2, d.d2, d.d1, d.c0, d.c1, d.c2, d.diag,
                                               W.V64[d.off + pt], sre, sim, (uint32_t)pt);
          const double2 bp = bs[pt];
          const double rx = bp.x - hx.x, ry = bp.y - hx.y;
          acc += rx * rx + ry * ry;
        }
      }
      acc = block_sum(acc, lds);
      if (threadIdx.x == 0) part[poff[p] + t] = acc;
    }
  }
}

// Grid K: rn[p] = ||r_p||, the square root of pole p's tile partials summed
// in tile order.
__global__ __launch_bounds__(TPB) void k_x_resid_norm(Work W, ShiftWork SW, const double* __restrict__ part,
                                                      const int32_t* __restrict__ poff, double* __restrict__ rn) {
  __shared__ double lds[NWAVE];
  const int p = blockIdx.x;
  if (p >= SW.K) return;
  const int s = SW.pinst[p];
  double acc = strided_sum(part + poff[p], W.sys[s].ntiles);
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) rn[p] = sqrt(acc);
}

// ------------------------------------------------------------ shared-basis adjoint
// One backward step from two shared bases (single instance): the forward
// solve on psi_n gives x_p = sum_b a_{p,b} c_b u_b (basis of F), the solve with
// conjugate shifts on gbar gives y_p = sum_a b_{p,a} c'_a u'_a (basis of A), and
//   dL/dV = -2 Re sum_p w_p conj(y_p) x_p
//         = -2 Re sum_{a,b} C_{ab} conj(u'_a) u_b,
//   C_{ab} = c'_a c_b sum_p w_p conj(b_{p,a}) a_{p,b}
// (a bilinear form of the two bases per grid point).

// Grid (m) blocks: row a of C (a < k_A), threads over b < k_F.
__global__ __launch_bounds__(TPB) void k_adj_coef(Work F, ShiftWork SF, Work A, ShiftWork SA, double2* __restrict__ C,
                                                  int ldc) {
  const int a = blockIdx.x;
  const int ka = A.st[0].kcyc, kf = F.st[0].kcyc;
  if (a >= ka) return;
  const double ca = A.cscale[a];
  const double2* wv = reinterpret_cast<const double2*>(SF.w);
  const double2* ya = reinterpret_cast<const double2*>(SA.y);
  const double2* yf = reinterpret_cast<const double2*>(SF.y);
  for (int b = threadIdx.x; b < kf; b += TPB) {
    double2 acc = make_double2(0.0, 0.0);
    for (int p = 0; p < SF.K; ++p) {
      const double2 t = cjmul(ya[(int64_t)p * A.m + a], yf[(int64_t)p * F.m + b]);  // conj(b) a
      const double2 u = cmul(wv[p], t);
      acc.x += u.x;
      acc.y += u.y;
    }
    const double sc = ca * F.cscale[b];
    C[(int64_t)a * ldc + b] = make_double2(acc.x * sc, acc.y * sc);
  }
}

// dV[p] += -2 Re sum_a conj(u'_a[p]) sum_b C_{ab} u_b[p], AC rows of C at a time.
template <int AC>
__global__ __launch_bounds__(TPB) void k_adj_grad(Work F, Work A, const double2* __restrict__ C, int ldc,
                                                  double* __restrict__ dV) {
  const int ka = A.st[0].kcyc, kf = F.st[0].kcyc;
  const SysDesc& df = F.sys[0];
  const SysDesc& da = A.sys[0];
  const int n = df.n;
  const double2* __restrict__ uf = basis_vec<double2>(F, df, 0);
  const double2* __restrict__ ua = basis_vec<double2>(A, da, 0);
  for (int p = blockIdx.x * TPB + threadIdx.x; p < n; p += gridDim.x * TPB) {
    double dv = 0.0;
    for (int a0 = 0; a0 < ka; a0 += AC) {
      double2 T[AC];
#pragma unroll
      for (int q = 0; q < AC; ++q) T[q] = make_double2(0.0, 0.0);
      for (int b = 0; b < kf; ++b) {
        const double2 u = uf[(int64_t)b * n + p];
#pragma unroll
        for (int q = 0; q < AC; ++q) {
          if (a0 + q < ka) {
            const double2 c = C[(int64_t)(a0 + q) * ldc + b];
            T[q].x += c.x * u.x - c.y * u.y;
            T[q].y += c.x * u.y + c.y * u.x;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < AC; ++q) {
        if (a0 + q < ka) {
          const double2 g = ua[(int64_t)(a0 + q) * n + p];
          dv += g.x * T[q].x + g.y * T[q].y;  // Re(conj(g) T)
        }
      }
    }
    dV[df.off + p] += -2.0 * dv;
  }
}

// ------------------------------------------------------------ fallback
// Poles the shared basis could not finish (its Krylov dimension is capped)
// continue as per-pole restarted solves warm-started from the shared-basis
// iterate x_p = V y_p. F is the per-pole solver of those poles, W the shared one.

// x_s = sum_{i<k} y_{p,i} c_i u_i(inst) in FP64 for every system s of F.
__global__ __launch_bounds__(TPB) void k_fb_init_x(Work F, Work W, ShiftWork SW) {
  __shared__ double2 coef[MAXM];
  int sprev = -1;
  for (int item = blockIdx.x; item < F.total_tiles; item += gridDim.x) {
    const int s = find_sys(F.tile_start, F.S, item);
    const SysDesc& d = F.sys[s];
    const int inst = d.inst;
    const SysDesc& dw = W.sys[inst];
    const int k = W.st[inst].kcyc;
    if (s != sprev) {
      __syncthreads();
      for (int i = threadIdx.x; i < k; i += TPB) {
        const double2 yi = reinterpret_cast<const double2*>(SW.y)[(int64_t)d.pole * W.m + i];
        const double c = W.cscale[(int64_t)inst * (W.m + 1) + i];
        coef[i] = make_double2(yi.x * c, yi.y * c);
      }
      __syncthreads();
      sprev = s;
    }
    const int t = item - d.tile0;
    const double2* __restrict__ u0 = basis_vec<double2>(W, dw, 0);
    double2* __restrict__ x = reinterpret_cast<double2*>(F.x) + d.xoff;
    // the whole tile of F (its own points per thread, not those of W)
    const int pend = min((t + 1) * F.tile, d.n);
    for (int p = t * F.tile + (int)threadIdx.x; p < pend; p += TPB) {
      double2 acc = make_double2(0.0, 0.0);
      for (int i = 0; i < k; ++i) {
        const double2 c = coef[i];
        const double2 a = u0[(int64_t)i * dw.n + p];
        acc.x += c.x * a.x - c.y * a.y;
        acc.y += c.x * a.y + c.y * a.x;
      }
      x[p] = acc;
    }
  }
}

// Per system of F: state of a solve whose first cycle has just ended with the
// warm-start iterate (the explicit residual and restart decision follow).
__global__ __launch_bounds__(TPB) void k_fb_state(Work F, Work W) {
  const int s = blockIdx.x;
  if (s >= F.S) return;
  if (s == 0) {
    const int nc = F.max_cycles * (F.m + 1) + 2;
    for (int i = threadIdx.x; i < nc; i += TPB) F.counters[i] = 0;
  }
  if (threadIdx.x != 0) return;
  const SysDesc& d = F.sys[s];
  SysState_t& st = F.st[s];
  st.bnorm = W.st[d.inst].bnorm;
  st.rnorm = st.bnorm;
  st.rho = 1.0;
  st.its = 0;
  st.cycles = 0;
  st.kcyc = 0;
  st.reorth = 0;
  st.first = 0;
  st.state = ST_FINISH;
}

// Per system of F: its final residual and iteration count replace the pole's.
__global__ __launch_bounds__(64) void k_fb_report(Work F, ShiftWork SW, int kshared_its) {
  const int s = blockIdx.x;
  if (s >= F.S || threadIdx.x != 0) return;
  const int p = F.sys[s].pole;
  SW.res[p] = F.st[s].rho;
  SW.its[p] = kshared_its + F.st[s].its;
}

// out[inst] += w x of one system of F (systems of one instance are added one
// launch after another, in pole order).
__global__ __launch_bounds__(TPB) void k_fb_accumulate(Work F, int s, double2* __restrict__ out) {
  const SysDesc& d = F.sys[s];
  const double2* __restrict__ x = reinterpret_cast<const double2*>(F.x) + d.xoff;
  for (int p = blockIdx.x * TPB + threadIdx.x; p < d.n; p += gridDim.x * TPB) {
    const double2 xv = x[p];
    double2 o = out[d.off + p];
    o.x += d.wre * xv.x - d.wim * xv.y;
    o.y += d.wre * xv.y + d.wim * xv.x;
    out[d.off + p] = o;
  }
}

// ------------------------------------------------------------ pole sum
// out = sum_s w_s x_s over the instance's systems in fixed order (FP64);
// conj_w selects conj(w_s) (adjoint) and sys_shift the first system used.
__global__ __launch_bounds__(TPB) void k_polesum(const InstDesc* __restrict__ inst, int ninst,
                                                 const int32_t* __restrict__ itile_start, int itotal,
                                                 const SysDesc* __restrict__ sys, const double* __restrict__ xall,
                                                 double2* __restrict__ out, int tile, int conj_w, int sys_shift) {
  for (int item = blockIdx.x; item < itotal; item += gridDim.x) {
    const int ii = find_sys(itile_start, ninst, item);
    const InstDesc& in = inst[ii];
    const int t = item - in.tile0;
    for (int p = t * tile + threadIdx.x; p < min((t + 1) * tile, in.n); p += TPB) {
      double ax = 0.0, ay = 0.0;
      for (int k = 0; k < in.nsys; ++k) {
        const SysDesc& d = sys[in.sys0 + sys_shift + k];
        const double2 xv = reinterpret_cast<const double2*>(xall)[d.xoff + p];
        const double wy = conj_w ? -d.wim : d.wim;
        ax += d.wre * xv.x - wy * xv.y;
        ay += d.wre * xv.y + wy * xv.x;
      }
      out[in.off + p] = make_double2(ax, ay);
    }
  }
}

// dV += -2 Re sum_j w_j conj(y_j) x_j, systems [0, K) hold x_j and [K, 2K) y_j.
__global__ __launch_bounds__(TPB) void k_grad_v(const InstDesc* __restrict__ inst, const int32_t* __restrict__ itile_start,
                                                int itotal, const SysDesc* __restrict__ sys,
                                                const double* __restrict__ xall, double* __restrict__ dV, int tile, int K) {
  for (int item = blockIdx.x; item < itotal; item += gridDim.x) {
    const InstDesc& in = inst[0];
    const int t = item;
    for (int p = t * tile + threadIdx.x; p < min((t + 1) * tile, in.n); p += TPB) {
      double acc = 0.0;
      for (int k = 0; k < K; ++k) {
        const SysDesc& dx = sys[k];
        const SysDesc& dy = sys[K + k];
        const double2 xv = reinterpret_cast<const double2*>(xall)[dx.xoff + p];
        const double2 yv = reinterpret_cast<const double2*>(xall)[dy.xoff + p];
        const double2 cy = cjmul(yv, xv);  // conj(y) x
        acc += dx.wre * cy.x - dx.wim * cy.y;  // Re(w conj(y) x)
      }
      dV[p] += -2.0 * acc;
    }
  }
  (void)itile_start;
}

// y = (H - shift) x in FP64 over all instances (packed).
__global__ __launch_bounds__(TPB) void k_apply_h(const InstDesc* __restrict__ inst, int ninst,
                                                 const int32_t* __restrict__ itile_start, int itotal,
                                                 const double* __restrict__ V, const double2* __restrict__ x,
                                                 double2* __restrict__ y, double sre, double sim, int tile) {
  for (int item = blockIdx.x; item < itotal; item += gridDim.x) {
    const int ii = find_sys(itile_start, ninst, item);
    const InstDesc& in = inst[ii];
    const int t = item - in.tile0;
    const double2* xi = x + in.off;
    for (int p = t * tile + threadIdx.x; p < min((t + 1) * tile, in.n); p += TPB) {
      y[in.off + p] = in.fem ? fem_point<double2>(xi, in.n0, in.n1, in.n2, in.d2, in.d1, in.fmd, in.fmo, in.fkd,
                                                  in.fko, in.fvol, V[in.off + p], sre, sim, (uint32_t)p)
                             : stencil_point_f64(xi, in.n0, in.n1, in.n2, in.d2, in.d1, in.c0, in.c1, in.c2,
                                                 in.diag, V[in.off + p], sre, sim, (uint32_t)p);
    }
  }
}

// y = M x per instance (Q1 finite elements: the right-hand side M psi of the
// shifted systems; copies x where an instance uses finite differences).
__global__ __launch_bounds__(TPB) void k_apply_mass(const InstDesc* __restrict__ inst, int ninst,
                                                    const int32_t* __restrict__ itile_start, int itotal,
                                                    const double2* __restrict__ x, double2* __restrict__ y,
                                                    int tile) {
  const double zero[3] = {0.0, 0.0, 0.0};
  for (int item = blockIdx.x; item < itotal; item += gridDim.x) {
    const int ii = find_sys(itile_start, ninst, item);
    const InstDesc& in = inst[ii];
    const int t = item - in.tile0;
    const double2* xi = x + in.off;
    for (int p = t * tile + threadIdx.x; p < min((t + 1) * tile, in.n); p += TPB) {
      // (0 + 0 V) x - (-1) M x
      y[in.off + p] = in.fem ? fem_point<double2>(xi, in.n0, in.n1, in.n2, in.d2, in.d1, in.fmd, in.fmo, zero,
                                                  zero, 0.0, 0.0, -1.0, 0.0, (uint32_t)p)
                             : xi[p];
    }
  }
}

// V64 -> V32 (the complex64 path's potential).
__global__ __launch_bounds__(TPB) void k_v_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) b[i] = (float)a[i];
}

// Flags non-finite entries of V (setup validation).
__global__ __launch_bounds__(TPB) void k_check_finite(const double* __restrict__ a, int64_t n, int32_t* flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double v = a[i];
    if (!(v == v) || v - v != 0.0) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

}  // namespace rexi
