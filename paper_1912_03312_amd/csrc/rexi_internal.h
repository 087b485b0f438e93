// Internal declarations of the REXI HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rexi {

// Unsigned division by a runtime constant d >= 1 for numerators a < 2^31:
// q = (a * mul) >> shift with mul = ceil(2^shift / d), shift = 31 + ceil(log2 d).
struct FastDiv {
  uint64_t mul;
  uint32_t shift;
  uint32_t d;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.shift = 31 + l;
  // ceil(2^shift / d); shift <= 62 so 2^shift fits in 64 bits
  unsigned __int128 num = ((unsigned __int128)1) << f.shift;
  f.mul = (uint64_t)((num + d - 1) / d);
  f.d = d;
  return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t a, const FastDiv& f) {
#if defined(__HIP_DEVICE_COMPILE__)
  // 32x64 -> high bits: a < 2^31, mul < 2^33, product < 2^64
  return (uint32_t)(((uint64_t)a * f.mul) >> f.shift);
#else
  return (uint32_t)(((unsigned __int128)a * f.mul) >> f.shift);
#endif
}

// One shifted system: (H_inst - shift I) x = b, where b is the instance's
// right-hand side (rhs_sel picks one of two packed right-hand-side vectors).
struct SysDesc {
  int64_t off;       // offset of the instance's points in packed vectors
  int64_t basis;     // element offset of the system's Krylov basis
  int64_t xoff;      // element offset of the system's FP64 solution
  int32_t n;         // points of the instance
  int32_t n0, n1, n2;  // grid dims padded to 3D, n0 slowest (1D: 1,1,n)
  FastDiv d2, d1;    // division by n2 and by n1
  double c0, c1, c2; // hbar^2 / (2 m h_a^2) per padded axis (0 if absent)
  double diag;       // 2 (c0 + c1 + c2)
  double sre, sim;   // shift s
  double wre, wim;   // weight w (pole sum)
  double tol;        // target relative residual rho*
  double dist;       // dist(shift, [lmin, lmax]) for the certificate
  int32_t inst;      // instance index
  int32_t tile0;     // first work tile of this system
  int32_t ntiles;    // work tiles of this system
  int32_t rhs_sel;   // 0 or 1
  int32_t pbase;     // offset of the system's partial-sum block
  // column-marching Lanczos pass: items of col_rows rows (n2 points each)
  // of the (i1, i2) plane over col_L consecutive planes, col_nr plane ranges
  int32_t col_rows;
  int32_t col_L;
  int32_t col_nr;
  int32_t col_n;     // items of the system (col_n = ceil(n1/col_rows) col_nr)
  int32_t col_cs;    // stride of its partial-sum slots, max(ntiles, col_n)
  int32_t pole;      // fallback solves: the pole (index into s, w) of the system
  int32_t fem;       // 1: Q1 finite elements, the system is (A - s M) x = M psi
  // Q1 elements, per padded axis: 1D mass diagonal / off-diagonal, stiffness
  // (times hbar^2/2m) diagonal / off-diagonal (1, 0, 0, 0 on an absent axis),
  // and h^d, the weight of the potential (nodal quadrature)
  double fmd[3], fmo[3], fkd[3], fko[3];
  double fvol;
};

// Instance descriptor (pole sum, apply_H).
struct InstDesc {
  int64_t off;
  int32_t n;
  int32_t n0, n1, n2;
  FastDiv d2, d1;
  double c0, c1, c2, diag;
  int32_t sys0;      // first system of the instance
  int32_t nsys;      // its poles
  int32_t tile0;     // first tile in the instance tiling
  int32_t ntiles;
  int32_t fem;       // Q1 finite elements (coefficients as in SysDesc)
  int32_t pad;
  double fmd[3], fmo[3], fkd[3], fko[3];
  double fvol;
  int64_t loff[3];   // Q1 shared basis: the Cholesky factor of axis a at chol + loff[a]
};

enum SysState : int32_t { ST_ACTIVE = 0, ST_FINISH = 1, ST_DONE = 2, ST_PAUSED = 3 };

// Per-system scalar state on the device.
struct SysState_t {
  int32_t state;
  int32_t kcyc;      // Arnoldi iterations in the current cycle
  int32_t its;       // total iterations (this solve)
  int32_t cycles;    // finished cycles (this solve)
  int32_t reorth;    // second Gram-Schmidt pass requested this iteration
  int32_t first;     // solution not yet written this solve
  double bnorm;      // ||b||
  double rnorm;      // ||r|| at the start of the current cycle
  double rho;        // last explicit relative residual
  double w2;         // ||w||^2 before projection (DGKS test)
};

// Device workspace pointers shared by the kernels.
struct Work {
  const SysDesc* sys;
  const int32_t* tile_start;   // [S+1] prefix of tiles over systems
  SysState_t* st;
  double* H;        // [S][(m+1) m] complex, column major (i + j (m+1))
  double* hcur;     // [S][m+1] complex, coefficients of the current GS pass
  double* gvec;     // [S][m+1] complex, rotated right-hand side
  double* gc;       // [S][m] complex, Givens c
  double* gs;       // [S][m] complex, Givens s
  double* cscale;   // [S][m+1] real, v_i = cscale_i * stored_i
  double* y;        // [S][m] complex, least-squares solution of the cycle
  double* part;     // complex partial sums [pbase + slot * ntiles + t]
  double* pnorm;    // real partial sums [tile]
  int32_t* counters;// [max_cycles * (m + 1) + 2]
  double* x;        // FP64 solutions [xoff + i]
  void* basis;      // Krylov bases (complex double or float)
  const double* V64;
  const float* V32;
  int32_t S;        // systems
  int32_t m;        // restart length
  int32_t total_tiles;
  int32_t reorth_mode;
  double inner_rtol;
  double eta2;      // DGKS threshold squared
  int32_t max_cycles;
  int32_t tile;     // points per tile
  int32_t ilv;      // per-pole bases stored tile-interleaved: log2(tile) (0: vector after vector)
  const int32_t* tile_sys;  // [total_tiles] system of each tile (null: search tile_start)
  int32_t* reo_any; // [m + 1] shared basis: 1 if any system takes a second pass at
                    // iteration j (null: per-system flags only)
  int32_t* jdev;    // captured schedules: [0] the iteration paused for a second pass
                    // (-1: none), [1] launches lost to pauses (null: host indices)
};

}  // namespace rexi
