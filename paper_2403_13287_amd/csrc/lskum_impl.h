// lskum_impl.h -- internals of the LSKUM library shared by its translation
// units (forward sweep and adjoint): device helpers, the plan record and host
// launch helpers.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <initializer_list>

#include <cmath>
#include <cstdint>
#include <vector>

#include "lskum.h"
#include "lskum_math.h"

namespace lskum_impl {

using lskum_math::lk_div;
using lskum_math::lk_rsqrt;

constexpr int kBlock = 256;
constexpr int kXcds = 8;
constexpr int kNormChunk = 2048;  // points per residual-norm chunk
constexpr unsigned kFlagNonPhysical = 1u;
constexpr unsigned kFlagDegenerate = 2u;

struct Geo {
  int n;
  int xcd;  // 1: blocks relabelled so that each XCD walks one contiguous range
  const double2 *xy;
  const double2 *nrm;
  const int8_t *kind;
  const int32_t *nbr;    // [k_pad][n]
  const int32_t *cnt;
  const int32_t *cloud;  // [n] cloud of each point (batched plans)
  const double *uinf;    // [n_clouds][4] free-stream state of each cloud
};

struct Flow {
  double gamma, inv_gm1, cfl, venkat_k;
  bool gamma_is_14;  // gamma == 1.4 exactly: rho from beta^(-5/2) without a log
};

// point records
struct __attribute__((aligned(32))) F4 {
  double v[4];
};
struct __attribute__((aligned(64))) F8 {
  double v[8];
};

__device__ __forceinline__ F4 ld4(const double *f, int i) {
  return reinterpret_cast<const F4 *>(f)[i];
}
__device__ __forceinline__ F8 ld8(const double *f, int i) {
  return reinterpret_cast<const F8 *>(f)[i];
}
__device__ __forceinline__ void st4(double *f, int i, const F4 &v) {
  reinterpret_cast<F4 *>(f)[i] = v;
}
__device__ __forceinline__ void st8(double *f, int i, const F8 &v) {
  reinterpret_cast<F8 *>(f)[i] = v;
}
// records addressed by a 64-bit index (edge-slot arrays)
__device__ __forceinline__ F4 ld4_at(const double *f, size_t i) {
  return reinterpret_cast<const F4 *>(f)[i];
}
__device__ __forceinline__ void st4_at(double *f, size_t i, const F4 &v) {
  reinterpret_cast<F4 *>(f)[i] = v;
}

// A tile's records in LDS as 16-byte planes: plane h holds doubles 2h and
// 2h+1 of every slot.  A wave reading 16 bytes per lane at consecutive or
// random slots then spreads over all LDS banks; whole 32- or 64-byte
// records would put its lanes on a quarter or an eighth of them.
template <int BLK>
__device__ __forceinline__ F4 pl_rd4(const double2 (*pl)[BLK], int sl) {
  const double2 a = pl[0][sl], b = pl[1][sl];
  return F4{{a.x, a.y, b.x, b.y}};
}
template <int BLK>
__device__ __forceinline__ F8 pl_rd8(const double2 (*pl)[BLK], int sl) {
  F8 r;
  for (int h = 0; h < 4; ++h) {
    const double2 a = pl[h][sl];
    r.v[2 * h] = a.x;
    r.v[2 * h + 1] = a.y;
  }
  return r;
}
template <int BLK>
__device__ __forceinline__ void pl_wr4(double2 (*pl)[BLK], int sl, const F4 &v) {
  for (int h = 0; h < 2; ++h) pl[h][sl] = make_double2(v.v[2 * h], v.v[2 * h + 1]);
}
template <int BLK>
__device__ __forceinline__ void pl_wr8(double2 (*pl)[BLK], int sl, const F8 &v) {
  for (int h = 0; h < 4; ++h) pl[h][sl] = make_double2(v.v[2 * h], v.v[2 * h + 1]);
}

// ---------------------------------------------------------------------------
// launch helpers

// Blocks are dispatched to the 8 XCDs round-robin (the default mapping).
// With xcd set, re-label them so that XCD x processes one contiguous range
// of logical blocks.  The grid is a multiple of 8; threads past n exit at
// once.
__device__ __forceinline__ int block_id(int xcd) {
  if (!xcd) return blockIdx.x;
  const int per = gridDim.x / kXcds;
  return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

template <int BLK>
__device__ __forceinline__ int point_index(int xcd) {
  return block_id(xcd) * BLK + threadIdx.x;
}

inline int grid_for(int n, int blk = kBlock) {
  int nb = (n + blk - 1) / blk;
  return (nb + kXcds - 1) / kXcds * kXcds;
}

// ds = dx*tx + dy*ty and dn = dx*nx + dy*ny with every product and sum
// rounded separately (no FMA contraction): the sign of ds/dn decides
// split-stencil membership, and this matches the oracle's uncontracted
// evaluation bit for bit.
__device__ __forceinline__ double dot_rn(double a, double b, double c, double d) {
#pragma clang fp contract(off)
  const double ab = a * b;
  const double cd = c * d;
  return ab + cd;
}

__device__ __forceinline__ void flag(unsigned *status, unsigned f) {
  if (f) __hip_atomic_fetch_or(status, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// eq. (13) and its inverse

__device__ __forceinline__ void prim_from_cons(double g, const F4 &U, double &rho, double &u,
                                               double &v, double &p) {
  rho = U.v[0];
  u = U.v[1] / rho;
  v = U.v[2] / rho;
  p = (g - 1.0) * (U.v[3] - 0.5 * rho * (u * u + v * v));
}

// eq. (13) at one point: the q-variables of the conserved state Ui;
// returns kFlagNonPhysical for rho or p <= 0 or non-finite.
__device__ __forceinline__ unsigned q_of_state(const Flow &P, const F4 &Ui, F4 &q) {
  double rho, u, v, p;
  prim_from_cons(P.gamma, Ui, rho, u, v, p);
  const unsigned f =
      (!(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p)) ? kFlagNonPhysical : 0u;
  const double beta = 0.5 * rho / p;
  q.v[0] = log(rho) + log(beta) * P.inv_gm1 - beta * (u * u + v * v);
  q.v[1] = 2.0 * beta * u;
  q.v[2] = 2.0 * beta * v;
  q.v[3] = -2.0 * beta;
  return f;
}

// Stage `stage` of the SSP Runge-Kutta (4,3) scheme at point i of kind
// `kind`, from its current state Uc, residual Ri and time step dt (U^n read
// from Un at stage 2 only), with the boundary conditions: outer points take
// their cloud's free stream, wall points drop the normal momentum.
__device__ __forceinline__ F4 ssp_stage(const Geo &G, int i, int kind, int stage,
                                        const double *__restrict__ Un, const F4 &Uc,
                                        const F4 &Ri, double dt) {
  F4 Ui;
  if (kind == 2) return ld4(G.uinf, G.cloud[i]);
  const double h = 0.5 * dt;
  if (stage == 2) {
    const F4 U0 = ld4(Un, i);
    for (int m = 0; m < 4; ++m)
      Ui.v[m] = (2.0 / 3.0) * U0.v[m] + (1.0 / 3.0) * (Uc.v[m] - h * Ri.v[m]);
  } else {
    for (int m = 0; m < 4; ++m) Ui.v[m] = Uc.v[m] - h * Ri.v[m];
  }
  if (kind == 1) {
    const double2 nv = G.nrm[i];
    const double mn = Ui.v[1] * nv.x + Ui.v[2] * nv.y;
    Ui.v[1] = Ui.v[1] - mn * nv.x;
    Ui.v[2] = Ui.v[2] - mn * nv.y;
  }
  return Ui;
}

// The stage update a flux launch may apply right after a point's residual
// (stage >= 0): U <- ssp_stage(U), and q_next <- the q-variables of the new
// state (a buffer other than the q the flux reads).  Stage 0 also stores the
// incoming U, the step's U^n, in Un for the third stage.
struct StageArgs {
  int stage;
  double *Un;
  const double *dt;
  double *U;
  double *q_next;
};

// ---------------------------------------------------------------------------
// block tiles
//
// A block owns BLK consecutive points (one Hilbert tile).  Kernels that
// gather neighbour records first stage the tile's own records in LDS, so the
// gathers of in-tile neighbours become LDS reads and only the remote ones go
// through the vector memory path.  On the 1M-point airfoil cloud 79 % of the
// neighbours fall inside their own 256-point tile, 72 % inside a 128-point
// one and 62 % inside the 64-point tiles of the flux kernel's
// one-wavefront blocks.

template <int BLK>
__device__ __forceinline__ int tile_lo(int xcd) {
  return block_id(xcd) * BLK;
}

// lj = j - lo; true when j belongs to the tile starting at lo
template <int BLK>
__device__ __forceinline__ bool in_tile(int j, int lo, int &lj) {
  lj = j - lo;
  return (unsigned)lj < (unsigned)BLK;
}

// Reader of point i's neighbour row (column-major connectivity).  Slots at
// or past the row's count read the last real slot and return i itself, so
// prefetching ahead never leaves the row: gather loops fetch the index two
// neighbours ahead and the neighbour's records one ahead, which keeps two
// dependent memory round trips off each iteration.
struct Row {
  const int32_t *col;  // &nbr[i], stride n
  int n, c, i;
  __device__ __forceinline__ int operator()(int k) const {
    const int kk = k < c ? k : c - 1;
    const int j = col[(size_t)kk * n];
    return k < c ? j : i;
  }
};

// Venkatakrishnan-limited increment phi*delta of one q component at one end
// of an edge: D is the room to the stencil max (delta > 0) or min (delta < 0),
// phi = min(1, (D^2 + eps2 + 2 delta D)/(D^2 + 2 delta^2 + delta D + eps2)),
// phi = 1 for delta = 0.
__device__ __forceinline__ double limited(double delta, double room_max, double room_min,
                                          double eps2) {
  const double D = delta > 0.0 ? room_max : room_min;
  const double num = D * D + eps2 + 2.0 * delta * D;
  const double den = D * D + 2.0 * delta * delta + delta * D + eps2;
  const double phi = delta == 0.0 ? 1.0 : fmin(1.0, lskum_math::lk_div1(num, den));
  return phi * delta;
}

// Min-max-limited increment: phi = min(1, D/delta) with D the room on
// delta's side, so the reconstructed value stays within the stencil bounds.
__device__ __forceinline__ double limited_minmax(double delta, double room_max,
                                                 double room_min) {
  const double D = delta > 0.0 ? room_max : room_min;
  const double phi = delta == 0.0 ? 1.0 : fmin(1.0, lk_div(D, delta));
  return phi * delta;
}

// Limiter constant of an edge: eps^2 = (K |d|)^3.
__device__ __forceinline__ double edge_eps2(double K, double dx, double dy) {
  const double d2 = dx * dx + dy * dy;
  const double kd = K * (d2 > 0.0 ? d2 * lk_rsqrt(d2) : 0.0);
  return kd * kd * kd;
}

// Increment of the modified q of eq. (14) at one end of edge d:
// -(d . grad q)/2.
__device__ __forceinline__ double half_step(double dx, double dy, double gx, double gy) {
  return -0.5 * (dx * gx + dy * gy);
}

// State at one end of an edge, recovered from the limited modified q.
struct EndState {
  double rho, us, un, p, E;
  double sqb;    // sqrt(beta)
  double bcoef;  // 1 / (2 sqrt(pi beta))
};

// Inverse of eq. (13): beta = -q4/2, (u, v) = (q2, q3)/(2 beta),
// rho = exp(q1 + beta (u^2+v^2)) beta^(-1/(gamma-1)), p = rho/(2 beta).
// For gamma = 1.4 the power is beta^(-5/2) = rsqrt(beta) / beta^2, so one
// rsqrt gives sqrt(beta), 1/beta and the power without a log or a divide.
// Intermediates of end_state kept for the adjoint.
struct EndExtra {
  double beta, ib, u, v, uu;  // ib = 1/beta
};

// G14: 1 when gamma = 1.4 is known at compile time, 0 for a general gamma,
// -1 to decide from P.gamma_is_14 at run time.  A kernel compiled for one
// case carries neither the other's code nor its constants in registers.
template <bool KEEP, int G14 = -1>
__device__ __forceinline__ unsigned end_state_t(const double qt[4], const Flow &P, double tx,
                                                double ty, double nx, double ny, EndState &s,
                                                EndExtra *x) {
  constexpr double kHalfRsqrtPi = 0.28209479177387814347;  // 1 / (2 sqrt(pi))
  const double beta = -0.5 * qt[3];
  const double rsb = lk_rsqrt(beta);
  const double ib = rsb * rsb;
  const double inv2b = 0.5 * ib;
  const double u = qt[1] * inv2b;
  const double v = qt[2] * inv2b;
  const double uu = u * u + v * v;
  double rho;
  if (G14 == 1 || (G14 < 0 && P.gamma_is_14))
    rho = lskum_math::lk_exp(qt[0] + beta * uu) * (rsb * ib * ib);
  else
    rho = lskum_math::lk_exp(qt[0] + beta * uu - log(beta) * P.inv_gm1);
  const double p = rho * inv2b;
  s.rho = rho;
  s.p = p;
  s.us = u * tx + v * ty;
  s.un = u * nx + v * ny;
  s.E = p * P.inv_gm1 + 0.5 * rho * uu;
  s.sqb = beta * rsb;
  s.bcoef = kHalfRsqrtPi * rsb;
  if (KEEP) *x = EndExtra{beta, ib, u, v, uu};
  return (!(beta > 0.0) || !(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p))
             ? kFlagNonPhysical
             : 0u;
}

template <int G14 = -1>
__device__ __forceinline__ unsigned end_state(const double qt[4], const Flow &P, double tx,
                                              double ty, double nx, double ny, EndState &s) {
  return end_state_t<false, G14>(qt, P, tx, ty, nx, ny, s, nullptr);
}

// Kinetic split flux along direction d with sign sg (+1 or -1): half-range
// moments of the Maxwellian of eq. (2) under the CIR split of eq. (3).
// ud: velocity along d, uo: the other component.  Output (mass, d-momentum,
// o-momentum, energy).
__device__ __forceinline__ void split_flux(double sg, const EndState &s, double ud, double uo,
                                           double G[4]) {
  const double S = ud * s.sqb;
  const double A = 0.5 * (1.0 + sg * lskum_math::lk_erf(S));
  const double B = lskum_math::lk_exp(-(S * S)) * s.bcoef;
  const double F = ud * A + sg * B;
  G[0] = s.rho * F;
  G[1] = (s.p + s.rho * ud * ud) * A + sg * s.rho * ud * B;
  G[2] = s.rho * uo * F;
  G[3] = (s.E + s.p) * ud * A + sg * (s.E + 0.5 * s.p) * B;
}

// Least-squares weights of one half-plane stencil: for an s-split the
// derivative is sum_i (Snn ds_i - Ssn dn_i)/det * dG_i, for an n-split
// sum_i (Sss dn_i - Ssn ds_i)/det * dG_i (eq. (11) in the (s, n) frame).
struct SplitW {
  double a, b;  // weight of edge i = a*ds_i + b*dn_i
};

__device__ __forceinline__ SplitW split_weights(bool s_dir, int count, double sss, double ssn,
                                                double snn, unsigned &f) {
  const double det = sss * snn - ssn * ssn;
  if (count < 2 || !(det > 1e-12 * sss * snn)) {
    f |= kFlagDegenerate;
    return SplitW{0.0, 0.0};
  }
  const double inv = 1.0 / det;
  return s_dir ? SplitW{snn * inv, -ssn * inv} : SplitW{-ssn * inv, sss * inv};
}

// Sum over the block (blockDim.x a power of two), fixed order.
__device__ __forceinline__ double block_sum(double v, double *lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  return lds[0];
}

// in-edge entries of the adjoint: slot in the source row, source point
constexpr int kSlotShift = 25;
constexpr int32_t kPointMask = (1 << kSlotShift) - 1;

// LDS tables of one tile size: block b stages the points of its tile (at
// most BLK consecutive points) and their out-of-tile neighbours (the tile's
// halo) in LDS, and its rows are stored as slots of that table, so the
// gather loop reads LDS only.
struct TileMap {
  int blk = 0;                // largest tile (the block size); 0 = not built
  int hmax = 0;               // table slots past blk, rounded up to a multiple of 4
  int groups = 0;             // groups of 8 row entries: k_pad rounded up to 8, over 8
  int ntiles = 0;
  int32_t *tlo = nullptr;     // [ntiles + 1] tile t holds points tlo[t] .. tlo[t+1]-1
  uint16_t *lcol = nullptr;   // [groups][n][8] table slot of every row entry (pads: own slot)
  int32_t *hoff = nullptr;    // [ntiles + 1] halo of tile t is hids[hoff[t] .. hoff[t+1])
  int32_t *hids = nullptr;    // halo point ids, ascending within a tile
};

// Tile tables of the in-edge rows (the rows that list each point), for the
// adjoint's transposed gathers: lent [k_in][n] holds, per in-edge entry,
// the source's LDS slot (low 16 bits) and the slot at which the source's
// row lists the point (bits 16 and up).
struct InTileMap {
  int blk = 0;
  int hmax = 0;
  int ntiles = 0;
  int32_t *tlo = nullptr;  // [ntiles + 1] tile bounds
  uint32_t *lent = nullptr;
  int32_t *hoff = nullptr;
  int32_t *hids = nullptr;
};

// kernel view of a TileMap
struct Tiles {
  const uint16_t *lcol;
  const int32_t *hoff;
  const int32_t *hids;
  int hmax;
  int groups;          // 8-entry groups of lcol
  const int32_t *tlo;  // tile bounds (tables of capped tiles)
  int ntiles;
};

}  // namespace lskum_impl

// ---------------------------------------------------------------------------
// plan

struct lskum_plan_s {
  int device = 0;
  int32_t n = 0, k_pad = 0, n_clouds = 0, n_wall = 0, n_chunks = 0;
  int block = 512, xcd = 0;
  int flux_block = 64;  // points per block of the flux kernel
  lskum_impl::TileMap maps[3];       // tile sizes 128, 256, 512 (built on demand)
  std::vector<lskum_params> params;  // one per cloud
  std::vector<int32_t> offset;       // first point of each cloud (+ total)
  double2 *xy = nullptr, *nrm = nullptr;
  int8_t *kind = nullptr;
  int32_t *nbr = nullptr, *cnt = nullptr, *cloud = nullptr;
  int32_t *wall = nullptr, *woff = nullptr;  // concatenated wall loops, offsets [n_clouds+1]
  double *uinf = nullptr;                    // [n_clouds][4]
  double *mach = nullptr, *aoa = nullptr;    // [n_clouds]
  int2 *chunks = nullptr;                    // residual-norm chunks
  int32_t *chunk_first = nullptr;            // first chunk of each cloud [n_clouds+1]
  double *partial = nullptr;                 // [n_chunks]
  double *norm_scratch = nullptr;            // [n_clouds]
  int32_t *counter = nullptr;                // graph-replay iteration counter
  unsigned *status = nullptr;
  // adjoint data, built by the first VJP call on the plan
  bool adj_ready = false;
  int32_t k_in = 0;               // padded in-edge row width (largest in-degree)
  int32_t *in_cnt = nullptr;      // [n] in-edges of each point
  int32_t *in_ent = nullptr;      // [k_in][n] (slot << kSlotShift) | source point
  lskum_impl::InTileMap in_map;   // tile tables of the in-edge rows (plan's tile size)
  double *spw = nullptr;          // [n][8] half-plane least-squares weights (with the plan)
  double *lsg = nullptr;          // [n][8] least-squares geometry of each point
  int32_t *outer = nullptr;       // outer points, grouped by cloud
  int32_t *ooff = nullptr;        // [n_clouds+1] offsets into outer
};

namespace lskum_impl {

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline Geo geo(const lskum_plan_s *p) {
  return Geo{p->n, p->xcd, p->xy, p->nrm, p->kind, p->nbr, p->cnt, p->cloud, p->uinf};
}

inline Flow flow(const lskum_plan_s *p) {
  Flow f;
  const lskum_params &q = p->params[0];  // shared settings (validated equal)
  f.gamma = q.gamma;
  f.inv_gm1 = 1.0 / (q.gamma - 1.0);
  f.cfl = q.cfl;
  f.venkat_k = q.venkat_k;
  f.gamma_is_14 = q.gamma == 1.4;
  return f;
}

// scheme variant of the flux kernel: 0 default, 1 first-order flux, 2 min-max limiter
inline int flux_variant(const lskum_plan_s *p) {
  const int o = p->params[0].options;
  return (o & LSKUM_FIRST_ORDER) ? 1 : ((o & LSKUM_MINMAX) ? 2 : 0);
}

inline int launched() { return hipGetLastError() == hipSuccess ? LSKUM_OK : LSKUM_ERR_HIP; }

// 4-double records need 32-byte, 8-double records 64-byte alignment.
inline bool a32(const void *p) { return p && ((uintptr_t)p % 32) == 0; }
inline bool a64(const void *p) { return p && ((uintptr_t)p % 64) == 0; }

// A byte range of a caller's buffer, for the aliasing checks of the entry
// points: a buffer that a launch writes must not share a byte with any other
// buffer the launch reads or writes.
struct Span {
  const void *p;
  size_t bytes;
};
inline bool overlap(const Span &a, const Span &b) {
  const uintptr_t a0 = (uintptr_t)a.p, b0 = (uintptr_t)b.p;
  return a.bytes && b.bytes && a0 < b0 + b.bytes && b0 < a0 + a.bytes;
}
// every written span disjoint from every other span (written or read)
inline bool writes_disjoint(std::initializer_list<Span> written, std::initializer_list<Span> read) {
  for (auto w = written.begin(); w != written.end(); ++w) {
    for (auto v = w + 1; v != written.end(); ++v)
      if (overlap(*w, *v)) return false;
    for (const Span &r : read)
      if (overlap(*w, r)) return false;
  }
  return true;
}

template <class T>
int upload(T **dst, const void *src, size_t count) {
  if (hipMalloc((void **)dst, count * sizeof(T) + (count == 0 ? sizeof(T) : 0)) != hipSuccess)
    return LSKUM_ERR_NO_MEMORY;
  if (count && hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return LSKUM_ERR_HIP;
  return LSKUM_OK;
}

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// kernel launches with the plan's tile size
#define LSKUM_TILED(kern, p, stream, ...)                                                    \
  do {                                                                                       \
    const int g_ = grid_for((p)->n, (p)->block);                                             \
    switch ((p)->block) {                                                                    \
      case 128: kern<128><<<g_, 128, 0, S(stream)>>>(__VA_ARGS__); break;                    \
      case 512: kern<512><<<g_, 512, 0, S(stream)>>>(__VA_ARGS__); break;                    \
      default: kern<256><<<g_, 256, 0, S(stream)>>>(__VA_ARGS__); break;                     \
    }                                                                                        \
  } while (0)

// Point i's whole row of table slots in registers, loaded before the
// staging barrier so that these loads overlap the staging and the gather
// loop reads LDS only (rows of at most KMAX entries).  Entries past the
// count hold the point's own slot; their loads re-read entry 0.
template <int KMAX, class E = uint16_t>
struct SlotRegs {
  int s[KMAX];
  __device__ __forceinline__ void load(const E *col, int n, int c, int own) {
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int sl = col[(size_t)(k < c ? k : 0) * n];
      s[k] = k < c ? sl : own;
    }
  }
  // The same from a table of `rows` rows, with no load waiting for the
  // count: entries past it are loaded but never read.
  __device__ __forceinline__ void load_rows(const E *col, int n, int rows) {
#pragma unroll
    for (int k = 0; k < KMAX; ++k) s[k] = col[(size_t)(k < rows ? k : rows - 1) * n];
  }
};

// Point i's whole row of table slots in registers, from a table laid out
// as [groups][n][8] (16 bytes per point and group: one load per 8 entries),
// two slots to a register; no load waits for the row's count (entries past
// it are loaded but never read).  Rows of at most KMAX entries.
template <int KMAX>
struct SlotGroups {
  static_assert(KMAX % 8 == 0, "whole groups");
  uint32_t w[KMAX / 2];
  __device__ __forceinline__ void load(const uint16_t *lcol, int n, int i, int groups) {
    const uint4 *g4 = reinterpret_cast<const uint4 *>(lcol);
#pragma unroll
    for (int g = 0; g < KMAX / 8; ++g) {
      const uint4 v = g4[(size_t)(g < groups ? g : groups - 1) * n + i];
      w[4 * g] = v.x;
      w[4 * g + 1] = v.y;
      w[4 * g + 2] = v.z;
      w[4 * g + 3] = v.w;
    }
  }
  __device__ __forceinline__ int operator[](int k) const {
    return (int)((w[k >> 1] >> (16 * (k & 1))) & 0xffffu);
  }
};

// Stage the records of tile `tile` (its points, then its halo) into LDS
// slots: every thread issues all of its loads before it stores any.  get(p)
// loads point p's records, put(slot, rec) stores them; the tile's points are
// lo .. n-1 (at most BLK) and its halo takes slots hb + k.  The halo ids head
// the longest chain of dependent loads (ids, then records, then the
// barrier), so they are issued first, and pre() then issues the caller's
// loads that depend on nothing staged, in their shadow.  No load sits in a
// divergent branch, so each wait covers only the loads it needs: indices
// are clamped (threads past n load point n-1; the halo list ends with a
// spare entry) and only the stores are conditional.
template <int BLK, class Rec, class Get, class Put, class Pre>
__device__ __forceinline__ void stage_tile(const Tiles &T, int tile, int lo, int n, int hb,
                                           Get get, Put put, Pre pre) {
  const int h0 = T.hoff[tile];
  const int nh = T.hoff[tile + 1] - h0;
  const int last = nh > 0 ? nh - 1 : 0;
  const int own = lo + threadIdx.x;
  const int t0 = threadIdx.x;
  int p0 = T.hids[h0 + min(t0, last)];
  int p1 = T.hids[h0 + min(t0 + BLK, last)];
  pre();
  const Rec r0 = get(own < n ? own : n - 1);
  // keeps the scheduler from moving work that needs the halo ids (and so
  // waits for them) above the loads issued in their shadow
  __builtin_amdgcn_sched_barrier(0);
  for (int b = 0;; b += 2 * BLK) {
    const int a0 = b + t0, a1 = a0 + BLK;
    const Rec r1 = get(p0), r2 = get(p1);
    if (b == 0 && own < n) put(t0, r0);
    if (a0 < nh) put(hb + a0, r1);
    if (a1 < nh) put(hb + a1, r2);
    if (b + 2 * BLK >= nh) break;
    p0 = T.hids[h0 + min(a0 + 2 * BLK, last)];
    p1 = T.hids[h0 + min(a1 + 2 * BLK, last)];
  }
}
template <int BLK, class Rec, class Get, class Put>
__device__ __forceinline__ void stage_tile(const Tiles &T, int tile, int lo, int n, Get get,
                                           Put put) {
  stage_tile<BLK, Rec>(T, tile, lo, n, n - lo < BLK ? n - lo : BLK, get, put, [] {});
}

struct XyQ {
  double2 xy;
  F4 q;
};
struct XyG {
  double2 xy;
  F8 g;
};

// tile maps: index of a tile size in lskum_plan_s::maps, kernel view, and
// the largest table a block may stage (half of a CU's LDS)
inline int tile_index(int blk) { return blk == 128 ? 0 : (blk == 512 ? 2 : 1); }
inline Tiles tiles(const TileMap &m) {
  return Tiles{m.lcol, m.hoff, m.hids, m.hmax, m.groups, m.tlo, m.ntiles};
}
// grid of one block per tile, a multiple of the XCD count
inline int grid_tiles(int ntiles) { return (ntiles + kXcds - 1) / kXcds * kXcds; }
constexpr size_t kTileLdsBytes = 80 * 1024;
// builds the tile map of the plan's current tile size if missing (synchronous)
int ensure_tile_map(lskum_plan_s *p);
// LDS slots of rows of point ids (column-major [width][n]; row i's entries
// past cnt[i] stand for i itself) on tiles of consecutive points: a tile's
// own points take slots 0..size-1 and the out-of-tile points its rows name
// (its halo, ascending in hids[hoff[t] .. hoff[t+1])) slots size + k.
// cap = 0: tiles of blk points (the last one shorter); cap > 0: a tile
// takes blk points, fewer (in steps of 8) while its points and halo exceed
// cap slots.  tlo gets the tile bounds, hmax the table slots past blk;
// hids ends with a spare entry.  LSKUM_ERR_INVALID_ARG when a tile needs
// more than 65535 slots.
int tile_slots(int32_t n, int32_t width, int blk, int cap, const int32_t *ids,
               const int32_t *cnt, std::vector<int32_t> &slots, std::vector<int32_t> &tlo,
               std::vector<int32_t> &hoff, std::vector<int32_t> &hids, int &hmax);

// launchers of the forward kernels (lskum.hip, lskum_deriv.hip, lskum_flux.hip),
// reused by the adjoint
int q_vars_launch(lskum_plan_s *p, const double *U, double *q, void *stream);
// argext (nullable): per point and component, the stencil slot that attains
// qlim (-1: the point itself), rows 0..3 for the max, 4..7 for the min
int deriv_first_launch(lskum_plan_s *p, const double *q, double *dq, double *qlim,
                       int8_t *argext, void *stream);
// one inner sweep: dq0 = the first-order solution, dqp = previous iterate
int deriv_inner_launch(lskum_plan_s *p, const double *dq0, const double *dqp, double *dqn,
                       void *stream);
// local time step (tile tables when they fit)
int local_dt_launch(lskum_plan_s *p, const double *U, double *dt, void *stream);
// flux residual for the plan's scheme variant; with st (nullable) the launch
// also applies SSP stage st->stage and writes the new state's q-variables
int flux_launch(lskum_plan_s *p, const double *q, const double *dq, const double *qlim,
                double *R, void *stream, const StageArgs *st = nullptr);

}  // namespace lskum_impl
