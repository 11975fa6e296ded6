// lskum.hip -- gfx950 kernels and C ABI of the LSKUM residual sweep.
//
// Method: arXiv 2403.13287, "Theory of Meshfree LSKUM" (eq. (9)-(16)).
// One thread per point for every sweep; points are stored in Hilbert order
// so that a wavefront's neighbour gathers hit a compact set of cache lines,
// and blocks are mapped to XCDs in contiguous point ranges so that each
// XCD's L2 holds the halo of its own range.  All arithmetic is FP64 on the
// vector ALUs; nothing here is a dense contraction, so no MFMA.
//
// Fields are point-major records (U, q, R: 4 doubles = 32 B per point;
// dq, qlim: 8 doubles = 64 B per point), so one neighbour's q, dq and qlim
// sit in one cache line each and load as 16-byte vectors.
//
// Data owned by a plan (device):
//   xy   double2 [n]         coordinates (one 16-byte gather per neighbour)
//   nrm  double2 [n]         unit normal (nx, ny)
//   kind int8    [n]
//   nbr  int32   [k_pad][n]  column-major connectivity, pad entries = own id
//   cnt  int32   [n]         real neighbours per point
//   wall int32   [n_wall]    wall loop, counter-clockwise
//   status uint32            OR of the kFlag* bits seen by the kernels
//   partial double [kNormBlocks] reduction scratch

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lskum.h"
#include "lskum_math.h"

namespace {

using lskum_math::lk_div;
using lskum_math::lk_rsqrt;

constexpr int kBlock = 256;
constexpr int kXcds = 8;
constexpr int kNormBlocks = 512;
constexpr unsigned kFlagNonPhysical = 1u;
constexpr unsigned kFlagDegenerate = 2u;

struct Geo {
  int n;
  const double2 *xy;
  const double2 *nrm;
  const int8_t *kind;
  const int32_t *nbr;  // [k_pad][n]
  const int32_t *cnt;
};

struct Flow {
  double gamma, inv_gm1, cfl, venkat_k;
  double uinf[4];
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

// ---------------------------------------------------------------------------
// launch helpers

// Blocks are dispatched to the 8 XCDs round-robin.  Re-label them so that XCD
// x processes one contiguous range of logical blocks.  The grid is a
// multiple of 8; threads past n exit at once.
__device__ __forceinline__ int xcd_block() {
  const int per = gridDim.x / kXcds;
  return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

__device__ __forceinline__ int point_index() { return xcd_block() * kBlock + threadIdx.x; }

inline int grid_for(int n) {
  int nb = (n + kBlock - 1) / kBlock;
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

__global__ void __launch_bounds__(kBlock) k_q_vars(int n, double g, double inv_gm1,
                                                   const double *__restrict__ U,
                                                   double *__restrict__ q, unsigned *status) {
  const int i = point_index();
  if (i >= n) return;
  double rho, u, v, p;
  prim_from_cons(g, ld4(U, i), rho, u, v, p);
  const unsigned f =
      (!(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p)) ? kFlagNonPhysical : 0u;
  const double beta = 0.5 * rho / p;
  F4 o;
  o.v[0] = log(rho) + log(beta) * inv_gm1 - beta * (u * u + v * v);
  o.v[1] = 2.0 * beta * u;
  o.v[2] = 2.0 * beta * v;
  o.v[3] = -2.0 * beta;
  st4(q, i, o);
  flag(status, f);
}

// ---------------------------------------------------------------------------
// block tiles
//
// A block owns kBlock consecutive points (one Hilbert tile).  Kernels that
// gather neighbour records first stage the tile's own records in LDS; about
// 80 % of the neighbours of a 1M-point airfoil cloud fall inside their own
// 256-point tile, so most gathers become LDS reads and only the remote ones
// go through the vector memory path.

__device__ __forceinline__ int tile_lo() { return xcd_block() * kBlock; }

// lj = j - lo; true when j belongs to the tile starting at lo
__device__ __forceinline__ bool in_tile(int j, int lo, int &lj) {
  lj = j - lo;
  return (unsigned)lj < (unsigned)kBlock;
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

// ---------------------------------------------------------------------------
// least-squares q-derivatives

// First-order solve (eq. (9) with dq_i = q_i - q_0) and stencil bounds.
__global__ void __launch_bounds__(kBlock) k_deriv_first(Geo G, const double *__restrict__ q,
                                                        double *__restrict__ dq,
                                                        double *__restrict__ qlim) {
  __shared__ double2 s_xy[kBlock];
  __shared__ F4 s_q[kBlock];
  const int n = G.n;
  const int lo = tile_lo();
  const int i = lo + threadIdx.x;
  const bool active = i < n;
  double2 xi = make_double2(0.0, 0.0);
  F4 q0{{0.0, 0.0, 0.0, 0.0}};
  if (active) {
    xi = G.xy[i];
    q0 = ld4(q, i);
  }
  s_xy[threadIdx.x] = xi;
  s_q[threadIdx.x] = q0;
  __syncthreads();
  if (!active) return;
  double qmax[4], qmin[4], sxq[4], syq[4];
  for (int m = 0; m < 4; ++m) {
    qmax[m] = qmin[m] = q0.v[m];
    sxq[m] = syq[m] = 0.0;
  }
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  const int c = G.cnt[i];
  const Row row{G.nbr + i, n, c, i};
  auto fetch = [&](int j, double2 &xj, F4 &qj) {
    int lj;
    if (in_tile(j, lo, lj)) {
      xj = s_xy[lj];
      qj = s_q[lj];
    } else {
      xj = G.xy[j];
      qj = ld4(q, j);
    }
  };
  int j_next = row(1);
  double2 xj;
  F4 qj;
  fetch(row(0), xj, qj);
  for (int k = 0; k < c; ++k) {
    const int j_after = row(k + 2);
    double2 xn;
    F4 qn;
    fetch(j_next, xn, qn);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
    for (int m = 0; m < 4; ++m) {
      const double d = qj.v[m] - q0.v[m];
      sxq[m] += dx * d;
      syq[m] += dy * d;
      qmax[m] = fmax(qmax[m], qj.v[m]);
      qmin[m] = fmin(qmin[m], qj.v[m]);
    }
    xj = xn;
    qj = qn;
    j_next = j_after;
  }
  const double det = sxx * syy - sxy * sxy;
  F8 g, lim;
  for (int m = 0; m < 4; ++m) {
    g.v[m] = (syy * sxq[m] - sxy * syq[m]) / det;
    g.v[4 + m] = (sxx * syq[m] - sxy * sxq[m]) / det;
    lim.v[m] = qmax[m];
    lim.v[4 + m] = qmin[m];
  }
  st8(dq, i, g);
  st8(qlim, i, lim);
}

// One Jacobi inner sweep (eq. (14)-(15)): modified differences from the
// previous iterate at both ends of each edge.
__global__ void __launch_bounds__(kBlock) k_deriv_inner(Geo G, const double *__restrict__ q,
                                                        const double *__restrict__ dqp,
                                                        double *__restrict__ dqn) {
  __shared__ double2 s_xy[kBlock];
  __shared__ F4 s_q[kBlock];
  __shared__ F8 s_g[kBlock];
  const int n = G.n;
  const int lo = tile_lo();
  const int i = lo + threadIdx.x;
  const bool active = i < n;
  double2 xi = make_double2(0.0, 0.0);
  F4 q0{{0.0, 0.0, 0.0, 0.0}};
  F8 g0{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
  if (active) {
    xi = G.xy[i];
    q0 = ld4(q, i);
    g0 = ld8(dqp, i);
  }
  s_xy[threadIdx.x] = xi;
  s_q[threadIdx.x] = q0;
  s_g[threadIdx.x] = g0;
  __syncthreads();
  if (!active) return;
  double sxq[4] = {0, 0, 0, 0}, syq[4] = {0, 0, 0, 0};
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  const int c = G.cnt[i];
  const Row row{G.nbr + i, n, c, i};
  auto fetch = [&](int j, double2 &xj, F4 &qj, F8 &gj) {
    int lj;
    if (in_tile(j, lo, lj)) {
      xj = s_xy[lj];
      qj = s_q[lj];
      gj = s_g[lj];
    } else {
      xj = G.xy[j];
      qj = ld4(q, j);
      gj = ld8(dqp, j);
    }
  };
  int j_next = row(1);
  double2 xj;
  F4 qj;
  F8 gj;
  fetch(row(0), xj, qj, gj);
  for (int k = 0; k < c; ++k) {
    const int j_after = row(k + 2);
    double2 xn;
    F4 qn;
    F8 gn;
    fetch(j_next, xn, qn, gn);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
    for (int m = 0; m < 4; ++m) {
      const double qtj = qj.v[m] - 0.5 * (dx * gj.v[m] + dy * gj.v[4 + m]);
      const double qt0 = q0.v[m] - 0.5 * (dx * g0.v[m] + dy * g0.v[4 + m]);
      const double d = qtj - qt0;
      sxq[m] += dx * d;
      syq[m] += dy * d;
    }
    xj = xn;
    qj = qn;
    gj = gn;
    j_next = j_after;
  }
  const double det = sxx * syy - sxy * sxy;
  F8 g;
  for (int m = 0; m < 4; ++m) {
    g.v[m] = (syy * sxq[m] - sxy * syq[m]) / det;
    g.v[4 + m] = (sxx * syq[m] - sxy * sxq[m]) / det;
  }
  st8(dqn, i, g);
}

// ---------------------------------------------------------------------------
// flux residual

// Venkatakrishnan-limited increment phi*delta of one q component at one end
// of an edge: D is the room to the stencil max (delta > 0) or min (delta < 0),
// phi = min(1, (D^2 + eps2 + 2 delta D)/(D^2 + 2 delta^2 + delta D + eps2)),
// phi = 1 for delta = 0.
__device__ __forceinline__ double limited(double delta, double room_max, double room_min,
                                          double eps2) {
  const double D = delta > 0.0 ? room_max : room_min;
  const double num = D * D + eps2 + 2.0 * delta * D;
  const double den = D * D + 2.0 * delta * delta + delta * D + eps2;
  const double phi = delta == 0.0 ? 1.0 : fmin(1.0, lk_div(num, den));
  return phi * delta;
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
__device__ __forceinline__ unsigned end_state(const double qt[4], const Flow &P, double tx,
                                              double ty, double nx, double ny, EndState &s) {
  constexpr double kHalfRsqrtPi = 0.28209479177387814347;  // 1 / (2 sqrt(pi))
  const double beta = -0.5 * qt[3];
  const double rsb = lk_rsqrt(beta);
  const double ib = rsb * rsb;
  const double inv2b = 0.5 * ib;
  const double u = qt[1] * inv2b;
  const double v = qt[2] * inv2b;
  const double uu = u * u + v * v;
  double rho;
  if (P.gamma_is_14)
    rho = exp(qt[0] + beta * uu) * (rsb * ib * ib);
  else
    rho = exp(qt[0] + beta * uu - log(beta) * P.inv_gm1);
  const double p = rho * inv2b;
  s.rho = rho;
  s.p = p;
  s.us = u * tx + v * ty;
  s.un = u * nx + v * ny;
  s.E = p * P.inv_gm1 + 0.5 * rho * uu;
  s.sqb = beta * rsb;
  s.bcoef = kHalfRsqrtPi * rsb;
  return (!(beta > 0.0) || !(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p))
             ? kFlagNonPhysical
             : 0u;
}

// Kinetic split flux along direction d with sign sg (+1 or -1): half-range
// moments of the Maxwellian of eq. (2) under the CIR split of eq. (3).
// ud: velocity along d, uo: the other component.  Output (mass, d-momentum,
// o-momentum, energy).
__device__ __forceinline__ void split_flux(double sg, const EndState &s, double ud, double uo,
                                           double G[4]) {
  const double S = ud * s.sqb;
  const double A = 0.5 * (1.0 + sg * erf(S));
  const double B = exp(-(S * S)) * s.bcoef;
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

__global__ void __launch_bounds__(kBlock) k_flux(Geo G, Flow P, const double *__restrict__ q,
                                                 const double *__restrict__ dq,
                                                 const double *__restrict__ qlim,
                                                 double *__restrict__ R, unsigned *status) {
  __shared__ double2 s_xy[kBlock];
  __shared__ F4 s_q[kBlock];
  __shared__ F8 s_g[kBlock];
  __shared__ F8 s_l[kBlock];
  const int n = G.n;
  const int lo = tile_lo();
  const int i = lo + threadIdx.x;
  const bool active = i < n;
  double2 xi = make_double2(0.0, 0.0);
  F4 q0{{0.0, 0.0, 0.0, 0.0}};
  F8 g0{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}}, l0 = g0;
  if (active) {
    xi = G.xy[i];
    q0 = ld4(q, i);
    g0 = ld8(dq, i);
    l0 = ld8(qlim, i);
  }
  s_xy[threadIdx.x] = xi;
  s_q[threadIdx.x] = q0;
  s_g[threadIdx.x] = g0;
  s_l[threadIdx.x] = l0;
  __syncthreads();
  if (!active) return;
  const int kind = G.kind[i];
  if (kind == 2) {
    st4(R, i, F4{{0.0, 0.0, 0.0, 0.0}});
    return;
  }
  const bool interior = kind == 0;
  const double2 nv = G.nrm[i];
  const double nx = nv.x, ny = nv.y, tx = ny, ty = -nx;
  const int c = G.cnt[i];
  const Row row{G.nbr + i, n, c, i};
  auto fetch_xy = [&](int j) {
    int lj;
    return in_tile(j, lo, lj) ? s_xy[lj] : G.xy[j];
  };

  // pass 1: geometry of the four half-plane stencils
  double sss[4] = {0, 0, 0, 0}, ssn[4] = {0, 0, 0, 0}, snn[4] = {0, 0, 0, 0};
  int cnt[4] = {0, 0, 0, 0};
  {
  int j_next = row(1);
  double2 xj = fetch_xy(row(0));
  for (int k = 0; k < c; ++k) {
    const int j_after = row(k + 2);
    const double2 xn = fetch_xy(j_next);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    const double ds = dot_rn(dx, tx, dy, ty);
    const double dn = dot_rn(dx, nx, dy, ny);
    const bool in[4] = {ds < 0.0, ds > 0.0, interior && dn < 0.0, dn > 0.0};
    for (int h = 0; h < 4; ++h) {
      const double w = in[h] ? 1.0 : 0.0;
      sss[h] += w * (ds * ds);
      ssn[h] += w * (ds * dn);
      snn[h] += w * (dn * dn);
      cnt[h] += in[h] ? 1 : 0;
    }
    xj = xn;
    j_next = j_after;
  }
  }
  unsigned f = 0;
  SplitW W[4];
  for (int h = 0; h < 4; ++h) {
    if (h == 2 && !interior) {
      W[h] = SplitW{0.0, 0.0};
      continue;
    }
    W[h] = split_weights(h < 2, cnt[h], sss[h], ssn[h], snn[h], f);
  }

  double mx0[4], mn0[4];
  for (int m = 0; m < 4; ++m) {
    mx0[m] = l0.v[m] - q0.v[m];
    mn0[m] = l0.v[4 + m] - q0.v[m];
  }
  const double K = P.venkat_k;
  double acc[4] = {0, 0, 0, 0};  // (mass, s-momentum, n-momentum, energy)

  // pass 2: limited modified q at both ends, split fluxes, weighted sums.
  // The index and coordinates are prefetched ahead; the neighbour's larger
  // records are loaded at the top of the iteration, while the own end's
  // reconstruction (which needs only the coordinates) proceeds.
  int j_next = row(1);
  int j_cur = row(0);
  double2 xj = fetch_xy(j_cur);
  for (int k = 0; k < c; ++k) {
    const int j_after = row(k + 2);
    const double2 xn = fetch_xy(j_next);
    int lj;
    F4 qj;
    F8 gj, lj8;
    if (in_tile(j_cur, lo, lj)) {
      qj = s_q[lj];
      gj = s_g[lj];
      lj8 = s_l[lj];
    } else {
      qj = ld4(q, j_cur);
      gj = ld8(dq, j_cur);
      lj8 = ld8(qlim, j_cur);
    }
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    const double ds = dot_rn(dx, tx, dy, ty);
    const double dn = dot_rn(dx, nx, dy, ny);
    const double d2 = dx * dx + dy * dy;
    const double kd = K * (d2 > 0.0 ? d2 * lk_rsqrt(d2) : 0.0);
    const double eps2 = kd * kd * kd;
    double qtj[4], qt0[4];
    for (int m = 0; m < 4; ++m) {
      const double dj = -0.5 * (dx * gj.v[m] + dy * gj.v[4 + m]);
      qtj[m] = qj.v[m] + limited(dj, lj8.v[m] - qj.v[m], lj8.v[4 + m] - qj.v[m], eps2);
      const double d0 = -0.5 * (dx * g0.v[m] + dy * g0.v[4 + m]);
      qt0[m] = q0.v[m] + limited(d0, mx0[m], mn0[m], eps2);
    }
    EndState sj, s0;
    f |= end_state(qtj, P, tx, ty, nx, ny, sj);
    f |= end_state(qt0, P, tx, ty, nx, ny, s0);

    // s-direction split: ds < 0 -> G_s^+, ds > 0 -> G_s^-
    {
      const bool pos = ds < 0.0;
      const SplitW w = pos ? W[0] : W[1];
      const double wt = ds != 0.0 ? w.a * ds + w.b * dn : 0.0;
      const double sg = pos ? 1.0 : -1.0;
      double Gj[4], G0[4];
      split_flux(sg, sj, sj.us, sj.un, Gj);
      split_flux(sg, s0, s0.us, s0.un, G0);
      acc[0] += wt * (Gj[0] - G0[0]);
      acc[1] += wt * (Gj[1] - G0[1]);
      acc[2] += wt * (Gj[2] - G0[2]);
      acc[3] += wt * (Gj[3] - G0[3]);
    }
    // n-direction split: dn < 0 -> G_n^+ (interior only), dn > 0 -> G_n^-
    {
      const bool pos = dn < 0.0;
      const SplitW w = pos ? W[2] : W[3];
      const bool used = dn > 0.0 || (pos && interior);
      const double wt = used ? w.a * ds + w.b * dn : 0.0;
      const double sg = pos ? 1.0 : -1.0;
      double Gj[4], G0[4];
      split_flux(sg, sj, sj.un, sj.us, Gj);
      split_flux(sg, s0, s0.un, s0.us, G0);
      acc[0] += wt * (Gj[0] - G0[0]);
      acc[1] += wt * (Gj[2] - G0[2]);
      acc[2] += wt * (Gj[1] - G0[1]);
      acc[3] += wt * (Gj[3] - G0[3]);
    }
    xj = xn;
    j_cur = j_next;
    j_next = j_after;
  }
  F4 r;
  r.v[0] = acc[0];
  r.v[1] = acc[1] * tx + acc[2] * nx;
  r.v[2] = acc[1] * ty + acc[2] * ny;
  r.v[3] = acc[3];
  st4(R, i, r);
  flag(status, f);
}

// ---------------------------------------------------------------------------
// local time step, Runge-Kutta stage, initial state

__global__ void __launch_bounds__(kBlock) k_local_dt(Geo G, Flow P, const double *__restrict__ U,
                                                     double *__restrict__ dt) {
  const int n = G.n;
  const int i = point_index();
  if (i >= n) return;
  const double2 xi = G.xy[i];
  double best = INFINITY;
  const int c = G.cnt[i];
  const Row row{G.nbr + i, n, c, i};
  int j_next = row(1);
  int j = row(0);
  double2 xj = G.xy[j];
  F4 Uj = ld4(U, j);
  for (int k = 0; k < c; ++k) {
    const int j_after = row(k + 2);
    const double2 xn = G.xy[j_next];
    const F4 Un = ld4(U, j_next);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    double rho, u, v, p;
    prim_from_cons(P.gamma, Uj, rho, u, v, p);
    const double speed = sqrt(u * u + v * v) + 3.0 * sqrt(p / rho);
    best = fmin(best, sqrt(dx * dx + dy * dy) / speed);
    xj = xn;
    Uj = Un;
    j_next = j_after;
  }
  dt[i] = P.cfl * best;
}

__global__ void __launch_bounds__(kBlock) k_rk_stage(Geo G, Flow P, int stage,
                                                     const double *__restrict__ Un,
                                                     const double *__restrict__ R,
                                                     const double *__restrict__ dt,
                                                     double *__restrict__ U) {
  const int n = G.n;
  const int i = point_index();
  if (i >= n) return;
  const int kind = G.kind[i];
  F4 Ui;
  if (kind == 2) {
    for (int m = 0; m < 4; ++m) Ui.v[m] = P.uinf[m];
  } else {
    const double h = 0.5 * dt[i];
    const F4 Uc = ld4(U, i), Ri = ld4(R, i);
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
  }
  st4(U, i, Ui);
}

__global__ void __launch_bounds__(kBlock) k_init_state(Geo G, Flow P, double *__restrict__ U) {
  const int n = G.n;
  const int i = point_index();
  if (i >= n) return;
  F4 Ui{{P.uinf[0], P.uinf[1], P.uinf[2], P.uinf[3]}};
  if (G.kind[i] == 1) {
    const double2 nv = G.nrm[i];
    const double mn = Ui.v[1] * nv.x + Ui.v[2] * nv.y;
    Ui.v[1] = Ui.v[1] - mn * nv.x;
    Ui.v[2] = Ui.v[2] - mn * nv.y;
  }
  st4(U, i, Ui);
}

__global__ void k_copy(size_t count, const double *__restrict__ src, double *__restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride)
    dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// deterministic reductions

__device__ __forceinline__ double block_sum(double v, double *lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  return lds[0];
}

// Block b sums R_rho^2 over the fixed range [b*chunk, (b+1)*chunk) of
// non-outer points; every thread walks a fixed strided subset.
__global__ void __launch_bounds__(kBlock) k_norm_partial(int n, int chunk, const int8_t *kind,
                                                         const double *__restrict__ R,
                                                         double *__restrict__ partial) {
  __shared__ double lds[kBlock];
  const int lo = blockIdx.x * chunk;
  const int hi = min(n, lo + chunk);
  double s = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) {
    const double r = R[4 * (size_t)i];
    if (kind[i] != 2) s += r * r;
  }
  const double t = block_sum(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kNormBlocks) k_norm_final(const double *__restrict__ partial,
                                                            double *__restrict__ out) {
  __shared__ double lds[kNormBlocks];
  const double t = block_sum(partial[threadIdx.x], lds);
  if (threadIdx.x == 0) out[0] = sqrt(t);
}

// Wall-polygon pressure integral (single block, fixed order).
__global__ void __launch_bounds__(kBlock) k_force(Geo G, Flow P, int n_wall,
                                                  const int32_t *__restrict__ wall,
                                                  const double *__restrict__ U, double mach,
                                                  double aoa, double *__restrict__ clcd) {
  __shared__ double lds[kBlock];
  const double pinf = 1.0 / P.gamma;
  const double qinf = 0.5 * mach * mach;
  double fx = 0.0, fy = 0.0;
  for (int e = threadIdx.x; e < n_wall; e += kBlock) {
    const int a = wall[e], b = wall[(e + 1) % n_wall];
    double ra, ua, va, pa, rb, ub, vb, pb;
    prim_from_cons(P.gamma, ld4(U, a), ra, ua, va, pa);
    prim_from_cons(P.gamma, ld4(U, b), rb, ub, vb, pb);
    const double cp = (0.5 * (pa + pb) - pinf) / qinf;
    const double2 xa = G.xy[a], xb = G.xy[b];
    fx += -cp * (xb.y - xa.y);
    fy += cp * (xb.x - xa.x);
  }
  const double Cx = block_sum(fx, lds);
  __syncthreads();
  const double Cy = block_sum(fy, lds);
  if (threadIdx.x == 0) {
    const double ca = cos(aoa), sa = sin(aoa);
    clcd[0] = Cy * ca - Cx * sa;
    clcd[1] = Cx * ca + Cy * sa;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// plan

struct lskum_plan_s {
  int device = 0;
  int32_t n = 0, k_pad = 0, n_wall = 0;
  lskum_params params{};
  double2 *xy = nullptr, *nrm = nullptr;
  int8_t *kind = nullptr;
  int32_t *nbr = nullptr, *cnt = nullptr, *wall = nullptr;
  unsigned *status = nullptr;
  double *partial = nullptr;
};

namespace {

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

Geo geo(const lskum_plan_s *p) { return Geo{p->n, p->xy, p->nrm, p->kind, p->nbr, p->cnt}; }

Flow flow(const lskum_plan_s *p) {
  Flow f;
  const lskum_params &q = p->params;
  f.gamma = q.gamma;
  f.inv_gm1 = 1.0 / (q.gamma - 1.0);
  f.cfl = q.cfl;
  f.venkat_k = q.venkat_k;
  f.gamma_is_14 = q.gamma == 1.4;
  const double rho = 1.0, u = q.mach * std::cos(q.aoa_rad), v = q.mach * std::sin(q.aoa_rad);
  const double pr = 1.0 / q.gamma;
  f.uinf[0] = rho;
  f.uinf[1] = rho * u;
  f.uinf[2] = rho * v;
  f.uinf[3] = pr / (q.gamma - 1.0) + 0.5 * rho * (u * u + v * v);
  return f;
}

bool params_ok(const lskum_params *p) {
  return p && std::isfinite(p->gamma) && p->gamma > 1.0 && std::isfinite(p->mach) &&
         p->mach >= 0.0 && std::isfinite(p->aoa_rad) && std::isfinite(p->cfl) && p->cfl > 0.0 &&
         std::isfinite(p->venkat_k) && p->venkat_k >= 0.0 && p->n_inner >= 0 &&
         p->n_inner <= 64 && p->reserved == 0;
}

int launched() { return hipGetLastError() == hipSuccess ? LSKUM_OK : LSKUM_ERR_HIP; }

// 4-double records need 32-byte, 8-double records 64-byte alignment.
bool a32(const void *p) { return p && ((uintptr_t)p % 32) == 0; }
bool a64(const void *p) { return p && ((uintptr_t)p % 64) == 0; }

void release(lskum_plan_s *p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipFree(p->xy);
  (void)hipFree(p->nrm);
  (void)hipFree(p->kind);
  (void)hipFree(p->nbr);
  (void)hipFree(p->cnt);
  (void)hipFree(p->wall);
  (void)hipFree(p->status);
  (void)hipFree(p->partial);
  (void)hipSetDevice(cur);
  delete p;
}

template <class T>
int upload(T **dst, const void *src, size_t count) {
  if (hipMalloc((void **)dst, count * sizeof(T) + (count == 0 ? sizeof(T) : 0)) != hipSuccess)
    return LSKUM_ERR_NO_MEMORY;
  if (count && hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return LSKUM_ERR_HIP;
  return LSKUM_OK;
}

// Size of one field of `comps` components, checked against overflow.
constexpr size_t kNumWorkFields = 4 + 4 + 8 + 8 + 8 + 4 + 1 + 1;  // Un q dq qlim work R dt norm

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" {

const char *lskum_strerror(int code) {
  switch (code) {
    case LSKUM_OK: return "ok";
    case LSKUM_ERR_INVALID_ARG: return "invalid argument";
    case LSKUM_ERR_BAD_CLOUD: return "point cloud failed validation";
    case LSKUM_ERR_HIP: return "HIP runtime error";
    case LSKUM_ERR_NONPHYSICAL: return "non-physical state (rho, p or beta <= 0, or non-finite)";
    case LSKUM_ERR_NO_MEMORY: return "device allocation failed";
    case LSKUM_ERR_DEGENERATE: return "singular half-plane stencil";
    default: return "unknown status";
  }
}

int lskum_plan_create(lskum_plan *out, const lskum_cloud *c, const lskum_params *params,
                      void *stream) {
  if (!out) return LSKUM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!c || !params_ok(params) || c->n < 1 || c->k_pad < 1 || !c->x || !c->y || !c->nx ||
      !c->ny || !c->kind || !c->row_ptr || !c->col || !c->nbr_count || c->n_wall < 0 ||
      (c->n_wall > 0 && !c->wall_loop))
    return LSKUM_ERR_INVALID_ARG;
  const int32_t n = c->n, kp = c->k_pad;
  if ((size_t)n * (size_t)kp > (size_t)INT32_MAX * 4) return LSKUM_ERR_INVALID_ARG;
  // host validation and the column-major connectivity
  std::vector<int32_t> nbr;
  try {
    nbr.resize((size_t)n * (size_t)kp);
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  if (c->row_ptr[0] != 0) return LSKUM_ERR_BAD_CLOUD;
  for (int32_t i = 0; i < n; ++i) {
    const int64_t b = c->row_ptr[i], e = c->row_ptr[i + 1];
    const int32_t cnt = c->nbr_count[i];
    if (e - b != kp || cnt < 2 || cnt > kp) return LSKUM_ERR_BAD_CLOUD;
    if (c->kind[i] < 0 || c->kind[i] > 2) return LSKUM_ERR_BAD_CLOUD;
    if (!std::isfinite(c->x[i]) || !std::isfinite(c->y[i]) || !std::isfinite(c->nx[i]) ||
        !std::isfinite(c->ny[i]))
      return LSKUM_ERR_BAD_CLOUD;
    for (int32_t k = 0; k < kp; ++k) {
      int32_t j = c->col[b + k];
      if (k < cnt) {
        if (j < 0 || j >= n || j == i) return LSKUM_ERR_BAD_CLOUD;
      } else {
        j = i;  // padding is always the point itself
      }
      nbr[(size_t)k * n + i] = j;
    }
  }
  for (int32_t e = 0; e < c->n_wall; ++e) {
    const int32_t w = c->wall_loop[e];
    if (w < 0 || w >= n || c->kind[w] != 1) return LSKUM_ERR_BAD_CLOUD;
  }
  std::vector<double2> xy((size_t)n), nrm((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    xy[i] = make_double2(c->x[i], c->y[i]);
    nrm[i] = make_double2(c->nx[i], c->ny[i]);
  }
  lskum_plan_s *p = new (std::nothrow) lskum_plan_s();
  if (!p) return LSKUM_ERR_NO_MEMORY;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return LSKUM_ERR_HIP;
  }
  p->n = n;
  p->k_pad = kp;
  p->n_wall = c->n_wall;
  p->params = *params;
  int rc = LSKUM_OK;
  if (rc == LSKUM_OK) rc = upload(&p->xy, xy.data(), (size_t)n);
  if (rc == LSKUM_OK) rc = upload(&p->nrm, nrm.data(), (size_t)n);
  if (rc == LSKUM_OK) rc = upload(&p->kind, c->kind, (size_t)n);
  if (rc == LSKUM_OK) rc = upload(&p->nbr, nbr.data(), nbr.size());
  if (rc == LSKUM_OK) rc = upload(&p->cnt, c->nbr_count, (size_t)n);
  if (rc == LSKUM_OK) rc = upload(&p->wall, c->wall_loop, (size_t)c->n_wall);
  if (rc == LSKUM_OK && hipMalloc((void **)&p->status, sizeof(unsigned)) != hipSuccess)
    rc = LSKUM_ERR_NO_MEMORY;
  if (rc == LSKUM_OK &&
      hipMalloc((void **)&p->partial, kNormBlocks * sizeof(double)) != hipSuccess)
    rc = LSKUM_ERR_NO_MEMORY;
  if (rc == LSKUM_OK && hipMemsetAsync(p->status, 0, sizeof(unsigned), S(stream)) != hipSuccess)
    rc = LSKUM_ERR_HIP;
  if (rc == LSKUM_OK && hipStreamSynchronize(S(stream)) != hipSuccess) rc = LSKUM_ERR_HIP;
  if (rc != LSKUM_OK) {
    release(p);
    return rc;
  }
  *out = p;
  return LSKUM_OK;
}

int lskum_plan_destroy(lskum_plan p) {
  if (!p) return LSKUM_ERR_INVALID_ARG;
  release(p);
  return LSKUM_OK;
}

int lskum_plan_set_params(lskum_plan p, const lskum_params *params) {
  if (!p || !params_ok(params)) return LSKUM_ERR_INVALID_ARG;
  p->params = *params;
  return LSKUM_OK;
}

int32_t lskum_plan_n(lskum_plan p) { return p ? p->n : -1; }

int lskum_init_state(lskum_plan p, double *U, void *stream) {
  if (!p || !a32(U)) return LSKUM_ERR_INVALID_ARG;
  k_init_state<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), flow(p), U);
  return launched();
}

int lskum_q_vars(lskum_plan p, const double *U, double *q, void *stream) {
  if (!p || !a32(U) || !a32(q)) return LSKUM_ERR_INVALID_ARG;
  const Flow f = flow(p);
  k_q_vars<<<grid_for(p->n), kBlock, 0, S(stream)>>>(p->n, f.gamma, f.inv_gm1, U, q, p->status);
  return launched();
}

int lskum_q_derivs(lskum_plan p, const double *q, double *dq, double *qlim, double *work,
                   void *stream) {
  if (!p || !a32(q) || !a64(dq) || !a64(qlim) || (p->params.n_inner > 0 && !a64(work)))
    return LSKUM_ERR_INVALID_ARG;
  const Geo g = geo(p);
  const int grid = grid_for(p->n);
  const int ni = p->params.n_inner;
  // ping-pong so that the last sweep writes dq
  double *a = (ni % 2 == 0) ? dq : work;
  double *b = (ni % 2 == 0) ? work : dq;
  k_deriv_first<<<grid, kBlock, 0, S(stream)>>>(g, q, a, qlim);
  for (int it = 0; it < ni; ++it) {
    k_deriv_inner<<<grid, kBlock, 0, S(stream)>>>(g, q, a, b);
    double *t = a;
    a = b;
    b = t;
  }
  return launched();
}

int lskum_flux_residual(lskum_plan p, const double *q, const double *dq, const double *qlim,
                        double *R, void *stream) {
  if (!p || !a32(q) || !a64(dq) || !a64(qlim) || !a32(R)) return LSKUM_ERR_INVALID_ARG;
  k_flux<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), flow(p), q, dq, qlim, R, p->status);
  return launched();
}

int lskum_local_dt(lskum_plan p, const double *U, double *dt, void *stream) {
  if (!p || !a32(U) || !dt) return LSKUM_ERR_INVALID_ARG;
  k_local_dt<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), flow(p), U, dt);
  return launched();
}

int lskum_rk_stage(lskum_plan p, int stage, const double *Un, const double *R, const double *dt,
                   double *U, void *stream) {
  if (!p || !a32(Un) || !a32(R) || !dt || !a32(U) || stage < 0 || stage > 3)
    return LSKUM_ERR_INVALID_ARG;
  k_rk_stage<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), flow(p), stage, Un, R, dt, U);
  return launched();
}

int lskum_residual_norm(lskum_plan p, const double *R, double *out, void *stream) {
  if (!p || !a32(R) || !out) return LSKUM_ERR_INVALID_ARG;
  const int chunk = (p->n + kNormBlocks - 1) / kNormBlocks;
  k_norm_partial<<<kNormBlocks, kBlock, 0, S(stream)>>>(p->n, chunk, p->kind, R, p->partial);
  k_norm_final<<<1, kNormBlocks, 0, S(stream)>>>(p->partial, out);
  return launched();
}

int lskum_force_coeffs(lskum_plan p, const double *U, double *clcd, void *stream) {
  if (!p || !a32(U) || !clcd || p->n_wall < 2) return LSKUM_ERR_INVALID_ARG;
  k_force<<<1, kBlock, 0, S(stream)>>>(geo(p), flow(p), p->n_wall, p->wall, U, p->params.mach,
                                       p->params.aoa_rad, clcd);
  return launched();
}

size_t lskum_workspace_bytes(lskum_plan p) {
  if (!p) return 0;
  return kNumWorkFields * align256((size_t)p->n * sizeof(double));
}

int lskum_iterate(lskum_plan p, int32_t iters, double *U, double *hist, void *ws, void *stream) {
  if (!p || !a32(U) || !ws || iters < 0 || ((uintptr_t)ws % 256) != 0) return LSKUM_ERR_INVALID_ARG;
  const size_t n = (size_t)p->n;
  const size_t f1 = align256(n * sizeof(double));
  char *base = static_cast<char *>(ws);
  double *Un = reinterpret_cast<double *>(base);
  double *q = reinterpret_cast<double *>(base + 4 * f1);
  double *dq = reinterpret_cast<double *>(base + 8 * f1);
  double *qlim = reinterpret_cast<double *>(base + 16 * f1);
  double *work = reinterpret_cast<double *>(base + 24 * f1);
  double *R = reinterpret_cast<double *>(base + 32 * f1);
  double *dt = reinterpret_cast<double *>(base + 36 * f1);
  double *scratch = reinterpret_cast<double *>(base + 37 * f1);
  const int copy_grid = grid_for((int)std::min<size_t>(4 * n, (size_t)1 << 24));
  for (int32_t it = 0; it < iters; ++it) {
    int rc = lskum_local_dt(p, U, dt, stream);
    if (rc) return rc;
    k_copy<<<copy_grid, kBlock, 0, S(stream)>>>(4 * n, U, Un);
    for (int s = 0; s < 4; ++s) {
      if ((rc = lskum_q_vars(p, U, q, stream))) return rc;
      if ((rc = lskum_q_derivs(p, q, dq, qlim, work, stream))) return rc;
      if ((rc = lskum_flux_residual(p, q, dq, qlim, R, stream))) return rc;
      if (s == 0) {
        if ((rc = lskum_residual_norm(p, R, hist ? hist + it : scratch, stream))) return rc;
      }
      if ((rc = lskum_rk_stage(p, s, Un, R, dt, U, stream))) return rc;
    }
  }
  return launched();
}

int lskum_status(lskum_plan p, void *stream) {
  if (!p) return LSKUM_ERR_INVALID_ARG;
  unsigned h = 0;
  if (hipMemcpyAsync(&h, p->status, sizeof(unsigned), hipMemcpyDeviceToHost, S(stream)) !=
          hipSuccess ||
      hipStreamSynchronize(S(stream)) != hipSuccess)
    return LSKUM_ERR_HIP;
  if (h & kFlagNonPhysical) return LSKUM_ERR_NONPHYSICAL;
  if (h & kFlagDegenerate) return LSKUM_ERR_DEGENERATE;
  return LSKUM_OK;
}

int lskum_clear_status(lskum_plan p, void *stream) {
  if (!p) return LSKUM_ERR_INVALID_ARG;
  return hipMemsetAsync(p->status, 0, sizeof(unsigned), S(stream)) == hipSuccess ? LSKUM_OK
                                                                                  : LSKUM_ERR_HIP;
}

}  // extern "C"
