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
//   cloud int32  [n]         cloud of each point; uinf double [n_clouds][4]
//   status uint32            OR of the kFlag* bits seen by the kernels
//   chunks, partial          residual-norm chunk table and partial sums

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lskum.h"
#include "lskum_impl.h"

namespace lskum_impl {

__global__ void __launch_bounds__(kBlock) k_q_vars(int n, int xcd, double g, double inv_gm1,
                                                   const double *__restrict__ U,
                                                   double *__restrict__ q, unsigned *status) {
  const int i = point_index<kBlock>(xcd);
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
// least-squares q-derivatives

// First-order solve (eq. (9) with dq_i = q_i - q_0) and stencil bounds.
// With ARG, also the slot attaining each bound (first in stencil order, the
// point itself first; -1 = the point itself), for the adjoint.
template <int BLK, bool ARG>
__global__ void __launch_bounds__(BLK) k_deriv_first(Geo G, const double *__restrict__ q,
                                                        double *__restrict__ dq,
                                                        double *__restrict__ qlim,
                                                        int8_t *__restrict__ argext) {
  __shared__ double2 s_xy[BLK];
  __shared__ double2 s_q[2][BLK];  // 16-byte planes
  const int n = G.n;
  const int lo = tile_lo<BLK>(G.xcd);
  const int i = lo + threadIdx.x;
  const bool active = i < n;
  double2 xi = make_double2(0.0, 0.0);
  F4 q0{{0.0, 0.0, 0.0, 0.0}};
  if (active) {
    xi = G.xy[i];
    q0 = ld4(q, i);
  }
  s_xy[threadIdx.x] = xi;
  pl_wr4<BLK>(s_q, threadIdx.x, q0);
  __syncthreads();
  if (!active) return;
  double qmax[4], qmin[4], sxq[4], syq[4];
  int amax[4], amin[4];
  for (int m = 0; m < 4; ++m) {
    qmax[m] = qmin[m] = q0.v[m];
    sxq[m] = syq[m] = 0.0;
    amax[m] = amin[m] = -1;
  }
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  const int c = G.cnt[i];
  const Row row{G.nbr + i, n, c, i};
  auto fetch = [&](int j, double2 &xj, F4 &qj) {
    int lj;
    if (in_tile<BLK>(j, lo, lj)) {
      xj = s_xy[lj];
      qj = pl_rd4<BLK>(s_q, lj);
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
      if (ARG) {
        if (qj.v[m] > qmax[m]) {
          qmax[m] = qj.v[m];
          amax[m] = k;
        }
        if (qj.v[m] < qmin[m]) {
          qmin[m] = qj.v[m];
          amin[m] = k;
        }
      } else {
        qmax[m] = fmax(qmax[m], qj.v[m]);
        qmin[m] = fmin(qmin[m], qj.v[m]);
      }
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
  if (ARG) {
    uint64_t packed = 0;
    for (int m = 0; m < 4; ++m) {
      packed |= (uint64_t)(uint8_t)(int8_t)amax[m] << (8 * m);
      packed |= (uint64_t)(uint8_t)(int8_t)amin[m] << (8 * (4 + m));
    }
    reinterpret_cast<uint64_t *>(argext)[i] = packed;
  }
}

// One Jacobi inner sweep (eq. (14)-(15)).  The modified differences are
// q~_j - q~_i = (q_j - q_i) - d.(g_j - g_i)/2 with g the previous iterate,
// and M_i^-1 sum_j d (q_j - q_i) is the first-order solution dq0_i, so
//   dq_i = dq0_i + g_i/2 - M_i^-1 sum_j d (d . g_j) / 2:
// the sweep gathers only the neighbours' previous derivatives.
template <int BLK>
__global__ void __launch_bounds__(BLK) k_deriv_inner(Geo G, const double *__restrict__ dq0,
                                                        const double *__restrict__ dqp,
                                                        double *__restrict__ dqn) {
  __shared__ double2 s_xy[BLK];
  __shared__ double2 s_g[4][BLK];  // 16-byte planes
  const int n = G.n;
  const int lo = tile_lo<BLK>(G.xcd);
  const int i = lo + threadIdx.x;
  const bool active = i < n;
  double2 xi = make_double2(0.0, 0.0);
  F8 g0{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
  if (active) {
    xi = G.xy[i];
    g0 = ld8(dqp, i);
  }
  s_xy[threadIdx.x] = xi;
  pl_wr8<BLK>(s_g, threadIdx.x, g0);
  __syncthreads();
  if (!active) return;
  double ax[4] = {0, 0, 0, 0}, ay[4] = {0, 0, 0, 0};
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  const int c = G.cnt[i];
  const Row row{G.nbr + i, n, c, i};
  auto fetch = [&](int j, double2 &xj, F8 &gj) {
    int lj;
    if (in_tile<BLK>(j, lo, lj)) {
      xj = s_xy[lj];
      gj = pl_rd8<BLK>(s_g, lj);
    } else {
      xj = G.xy[j];
      gj = ld8(dqp, j);
    }
  };
  int j_next = row(1);
  double2 xj;
  F8 gj;
  fetch(row(0), xj, gj);
  for (int k = 0; k < c; ++k) {
    const int j_after = row(k + 2);
    double2 xn;
    F8 gn;
    fetch(j_next, xn, gn);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
    for (int m = 0; m < 4; ++m) {
      const double t = dx * gj.v[m] + dy * gj.v[4 + m];
      ax[m] += dx * t;
      ay[m] += dy * t;
    }
    xj = xn;
    gj = gn;
    j_next = j_after;
  }
  const double det = sxx * syy - sxy * sxy;
  const F8 d0 = ld8(dq0, i);
  F8 g;
  for (int m = 0; m < 4; ++m) {
    g.v[m] = d0.v[m] + 0.5 * g0.v[m] - 0.5 * ((syy * ax[m] - sxy * ay[m]) / det);
    g.v[4 + m] = d0.v[4 + m] + 0.5 * g0.v[4 + m] - 0.5 * ((sxx * ay[m] - sxy * ax[m]) / det);
  }
  st8(dqn, i, g);
}

// ---------------------------------------------------------------------------
// derivative passes on LDS tables (tile maps)
//
// Block b stages in LDS the records of its BLK points and of their
// out-of-tile neighbours (the tile's halo, a few hundred points for a
// Hilbert-ordered cloud), loaded by all threads at once with no dependent
// round trips; each row is stored as table slots (uint16), so the gather
// loop reads LDS only.  Same arithmetic, in the same order, as k_deriv_first
// and k_deriv_inner, which remain the path for clouds whose halos do not fit.

// Reader of point i's row of table slots; entries past the count return
// the point's own slot (prefetching ahead never leaves the row).
struct SlotRow {
  const uint16_t *col;  // &lcol[i], stride n
  int n, c, own;
  __device__ __forceinline__ int operator()(int k) const {
    const int kk = k < c ? k : c - 1;
    const int sl = col[(size_t)kk * n];
    return k < c ? sl : own;
  }
};

// KMAX: rows of at most KMAX entries (slots in registers), 0: any row length
template <int BLK, bool ARG, int KMAX>
__global__ void __launch_bounds__(BLK) k_deriv_first_t(Geo G, Tiles T,
                                                          const double *__restrict__ q,
                                                          double *__restrict__ dq,
                                                          double *__restrict__ qlim,
                                                          int8_t *__restrict__ argext) {
  extern __shared__ __align__(64) unsigned char smem[];
  const int n = G.n;
  const int tile = block_id(G.xcd);
  const int lo = tile * BLK;
  if (lo >= n) return;  // blocks past the last tile (the grid is a multiple of 8)
  const int cap = BLK + T.hmax;
  // 16-byte planes (coordinates, q0 q1, q2 q3): random-slot reads spread
  // over all LDS banks, where whole 32-byte records would share few
  double2 *s_xy = reinterpret_cast<double2 *>(smem);
  double2 *s_q = s_xy + cap;
  auto rd_q = [&](int sl) {
    const double2 a = s_q[sl], b = s_q[cap + sl];
    return F4{{a.x, a.y, b.x, b.y}};
  };
  const int i = lo + threadIdx.x;
  const int c = i < n ? G.cnt[i] : 0;
  SlotRegs<KMAX ? KMAX : 1> sr;
  if (KMAX && i < n) sr.load(T.lcol + i, n, c, threadIdx.x);
  stage_tile<BLK, XyQ>(
      T, tile, lo, n, [&](int p) { return XyQ{G.xy[p], ld4(q, p)}; },
      [&](int sl, const XyQ &r) {
        s_xy[sl] = r.xy;
        s_q[sl] = make_double2(r.q.v[0], r.q.v[1]);
        s_q[cap + sl] = make_double2(r.q.v[2], r.q.v[3]);
      });
  __syncthreads();
  if (i >= n) return;
  const double2 xi = s_xy[threadIdx.x];
  const F4 q0 = rd_q(threadIdx.x);
  double qmax[4], qmin[4], sxq[4], syq[4];
  int amax[4], amin[4];
  for (int m = 0; m < 4; ++m) {
    qmax[m] = qmin[m] = q0.v[m];
    sxq[m] = syq[m] = 0.0;
    amax[m] = amin[m] = -1;
  }
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  auto edge = [&](int k, int sl) {
    const double2 xj = s_xy[sl];
    const F4 qj = rd_q(sl);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
    for (int m = 0; m < 4; ++m) {
      const double d = qj.v[m] - q0.v[m];
      sxq[m] += dx * d;
      syq[m] += dy * d;
      if (ARG) {
        if (qj.v[m] > qmax[m]) {
          qmax[m] = qj.v[m];
          amax[m] = k;
        }
        if (qj.v[m] < qmin[m]) {
          qmin[m] = qj.v[m];
          amin[m] = k;
        }
      } else {
        qmax[m] = fmax(qmax[m], qj.v[m]);
        qmin[m] = fmin(qmin[m], qj.v[m]);
      }
    }
  };
  if (KMAX) {
#pragma unroll
    for (int k = 0; k < (KMAX ? KMAX : 1); ++k)
      if (k < c) edge(k, sr.s[k]);
  } else {
    const SlotRow row{T.lcol + i, n, c, (int)threadIdx.x};
    int s_next = row(1);
    int s_cur = row(0);
    for (int k = 0; k < c; ++k) {
      const int s_after = row(k + 2);
      edge(k, s_cur);
      s_cur = s_next;
      s_next = s_after;
    }
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
  if (ARG) {
    uint64_t packed = 0;
    for (int m = 0; m < 4; ++m) {
      packed |= (uint64_t)(uint8_t)(int8_t)amax[m] << (8 * m);
      packed |= (uint64_t)(uint8_t)(int8_t)amin[m] << (8 * (4 + m));
    }
    reinterpret_cast<uint64_t *>(argext)[i] = packed;
  }
}

template <int BLK, int KMAX>
__global__ void __launch_bounds__(BLK) k_deriv_inner_t(Geo G, Tiles T,
                                                          const double *__restrict__ dq0,
                                                          const double *__restrict__ dqp,
                                                          double *__restrict__ dqn) {
  extern __shared__ __align__(64) unsigned char smem[];
  const int n = G.n;
  const int tile = block_id(G.xcd);
  const int lo = tile * BLK;
  if (lo >= n) return;
  const int cap = BLK + T.hmax;
  // 16-byte planes (coordinates, then the derivative record in four pairs)
  double2 *s_xy = reinterpret_cast<double2 *>(smem);
  double2 *s_g = s_xy + cap;
  auto rd_g = [&](int sl) {
    F8 g;
    for (int h = 0; h < 4; ++h) {
      const double2 a = s_g[h * cap + sl];
      g.v[2 * h] = a.x;
      g.v[2 * h + 1] = a.y;
    }
    return g;
  };
  const int i = lo + threadIdx.x;
  const int c = i < n ? G.cnt[i] : 0;
  SlotRegs<KMAX ? KMAX : 1> sr;
  if (KMAX && i < n) sr.load(T.lcol + i, n, c, threadIdx.x);
  stage_tile<BLK, XyG>(
      T, tile, lo, n, [&](int p) { return XyG{G.xy[p], ld8(dqp, p)}; },
      [&](int sl, const XyG &r) {
        s_xy[sl] = r.xy;
        for (int h = 0; h < 4; ++h) s_g[h * cap + sl] = make_double2(r.g.v[2 * h], r.g.v[2 * h + 1]);
      });
  __syncthreads();
  if (i >= n) return;
  const double2 xi = s_xy[threadIdx.x];
  const F8 g0 = rd_g(threadIdx.x);
  double ax[4] = {0, 0, 0, 0}, ay[4] = {0, 0, 0, 0};
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  auto edge = [&](int sl) {
    const double2 xj = s_xy[sl];
    const F8 gj = rd_g(sl);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
    for (int m = 0; m < 4; ++m) {
      const double t = dx * gj.v[m] + dy * gj.v[4 + m];
      ax[m] += dx * t;
      ay[m] += dy * t;
    }
  };
  if (KMAX) {
#pragma unroll
    for (int k = 0; k < (KMAX ? KMAX : 1); ++k)
      if (k < c) edge(sr.s[k]);
  } else {
    const SlotRow row{T.lcol + i, n, c, (int)threadIdx.x};
    int s_next = row(1);
    int s_cur = row(0);
    for (int k = 0; k < c; ++k) {
      const int s_after = row(k + 2);
      edge(s_cur);
      s_cur = s_next;
      s_next = s_after;
    }
  }
  const double det = sxx * syy - sxy * sxy;
  const F8 d0 = ld8(dq0, i);
  F8 g;
  for (int m = 0; m < 4; ++m) {
    g.v[m] = d0.v[m] + 0.5 * g0.v[m] - 0.5 * ((syy * ax[m] - sxy * ay[m]) / det);
    g.v[4 + m] = d0.v[4 + m] + 0.5 * g0.v[4 + m] - 0.5 * ((sxx * ay[m] - sxy * ax[m]) / det);
  }
  st8(dqn, i, g);
}

// ---------------------------------------------------------------------------
// flux residual

// Least-squares weights of the four half-plane stencils of every point
// (geometry only; computed when the plan is built): spw[i] = (a, b) of s+,
// s-, n+, n-, and the weight of edge d in split h is a_h ds + b_h dn.  A used
// split that is singular, and the n+ split of wall and outer points, get
// (0, 0).
__global__ void __launch_bounds__(kBlock) k_split_weights(Geo G, double *__restrict__ spw) {
  const int n = G.n;
  const int i = point_index<kBlock>(G.xcd);
  if (i >= n) return;
  const int kind = G.kind[i];
  if (kind == 2) {
    st8(spw, i, F8{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}});
    return;
  }
  const bool interior = kind == 0;
  const double2 xi = G.xy[i], nv = G.nrm[i];
  const double nx = nv.x, ny = nv.y, tx = ny, ty = -nx;
  const int c = G.cnt[i];
  double sss[4] = {0, 0, 0, 0}, ssn[4] = {0, 0, 0, 0}, snn[4] = {0, 0, 0, 0};
  int cnt[4] = {0, 0, 0, 0};
  for (int k = 0; k < c; ++k) {
    const double2 xj = G.xy[G.nbr[(size_t)k * n + i]];
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
  }
  unsigned f = 0;
  F8 out;
  for (int h = 0; h < 4; ++h) {
    SplitW w{0.0, 0.0};
    if (!(h == 2 && !interior)) w = split_weights(h < 2, cnt[h], sss[h], ssn[h], snn[h], f);
    out.v[2 * h] = w.a;
    out.v[2 * h + 1] = w.b;
  }
  st8(spw, i, out);
}

// A used split is singular exactly when its weights are (0, 0): a regular
// s-split has a = Snn/det > 0, a regular n-split b = Sss/det > 0.
__device__ __forceinline__ unsigned degenerate_splits(const F8 &W, bool interior) {
  const bool bad = W.v[0] == 0.0 || W.v[2] == 0.0 || (interior && W.v[5] == 0.0) ||
                   W.v[7] == 0.0;
  return bad ? kFlagDegenerate : 0u;
}

// Flux residual of every point: for each edge, the limited modified q at
// both ends, their states, and the split fluxes of the edge's s- and
// n-split, weighted by the point's half-plane least-squares weights.  The
// point's own records and weights are re-read from LDS at every edge
// instead of being held in registers through the loop.
// VAR: 0 the default scheme, 1 first-order flux (q~ = q), 2 min-max limiter
template <int BLK, int VAR>
__global__ void __launch_bounds__(BLK) k_flux(Geo G, Flow P, const double *__restrict__ spw,
                                                 const double *__restrict__ q,
                                                 const double *__restrict__ dq,
                                                 const double *__restrict__ qlim,
                                                 double *__restrict__ R, unsigned *status) {
  // the tile's records as 16-byte planes: q in 2, dq, qlim and the split
  // weights in 4 each (whole records would put lanes on few LDS banks)
  __shared__ double2 s_xy[BLK];
  __shared__ double2 s_q[2][BLK];
  __shared__ double2 s_g[4][BLK];
  __shared__ double2 s_l[4][BLK];
  __shared__ double2 s_w[4][BLK];
  const auto rd4 = pl_rd4<BLK>;
  const auto rd8 = pl_rd8<BLK>;
  const int n = G.n;
  const int lo = tile_lo<BLK>(G.xcd);
  const int i = lo + threadIdx.x;
  const bool active = i < n;
  {
    double2 xi = make_double2(0.0, 0.0);
    F4 q0{{0.0, 0.0, 0.0, 0.0}};
    F8 g0{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}}, l0 = g0, w0 = g0;
    if (active) {
      xi = G.xy[i];
      q0 = ld4(q, i);
      g0 = ld8(dq, i);
      l0 = ld8(qlim, i);
      w0 = ld8(spw, i);
    }
    const int t = threadIdx.x;
    s_xy[t] = xi;
    pl_wr4<BLK>(s_q, t, q0);
    pl_wr8<BLK>(s_g, t, g0);
    pl_wr8<BLK>(s_l, t, l0);
    pl_wr8<BLK>(s_w, t, w0);
  }
  __syncthreads();
  if (!active) return;
  const int kind = G.kind[i];
  if (kind == 2) {
    st4(R, i, F4{{0.0, 0.0, 0.0, 0.0}});
    return;
  }
  const bool interior = kind == 0;
  const double2 xi = s_xy[threadIdx.x];
  const double2 nv = G.nrm[i];
  const double nx = nv.x, ny = nv.y, tx = ny, ty = -nx;
  const int c = G.cnt[i];
  const Row row{G.nbr + i, n, c, i};
  auto fetch_xy = [&](int j) {
    int lj;
    return in_tile<BLK>(j, lo, lj) ? s_xy[lj] : G.xy[j];
  };
  unsigned f = degenerate_splits(rd8(s_w, threadIdx.x), interior);
  const double K = P.venkat_k;
  double acc[4] = {0, 0, 0, 0};  // (mass, s-momentum, n-momentum, energy)

  // The index and coordinates are prefetched ahead; the neighbour's larger
  // records are loaded at the top of the iteration.
  int j_next = row(1);
  int j_cur = row(0);
  double2 xj = fetch_xy(j_cur);
  for (int k = 0; k < c; ++k) {
    const int j_after = row(k + 2);
    const double2 xn = fetch_xy(j_next);
    int lj;
    F4 qj;
    F8 gj, lj8;
    if (in_tile<BLK>(j_cur, lo, lj)) {
      qj = rd4(s_q, lj);
      gj = rd8(s_g, lj);
      lj8 = rd8(s_l, lj);
    } else {
      qj = ld4(q, j_cur);
      gj = ld8(dq, j_cur);
      lj8 = ld8(qlim, j_cur);
    }
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    const double ds = dot_rn(dx, tx, dy, ty);
    const double dn = dot_rn(dx, nx, dy, ny);
    const double eps2 = edge_eps2(K, dx, dy);
    double qtj[4], qt0[4];
    {
      // keeps the compiler from hoisting the own-record reads out of the loop
      asm volatile("" ::: "memory");
      const F4 q0 = rd4(s_q, threadIdx.x);
      const F8 g0 = rd8(s_g, threadIdx.x), l0 = rd8(s_l, threadIdx.x);
      for (int m = 0; m < 4; ++m) {
        if (VAR == 1) {
          qtj[m] = qj.v[m];
          qt0[m] = q0.v[m];
          continue;
        }
        const double dj = half_step(dx, dy, gj.v[m], gj.v[4 + m]);
        const double d0 = half_step(dx, dy, g0.v[m], g0.v[4 + m]);
        if (VAR == 2) {
          qtj[m] = qj.v[m] + limited_minmax(dj, lj8.v[m] - qj.v[m], lj8.v[4 + m] - qj.v[m]);
          qt0[m] = q0.v[m] + limited_minmax(d0, l0.v[m] - q0.v[m], l0.v[4 + m] - q0.v[m]);
        } else {
          qtj[m] = qj.v[m] + limited(dj, lj8.v[m] - qj.v[m], lj8.v[4 + m] - qj.v[m], eps2);
          qt0[m] = q0.v[m] + limited(d0, l0.v[m] - q0.v[m], l0.v[4 + m] - q0.v[m], eps2);
        }
      }
    }
    EndState sj, s0;
    f |= end_state(qtj, P, tx, ty, nx, ny, sj);
    f |= end_state(qt0, P, tx, ty, nx, ny, s0);
    const F8 W = rd8(s_w, threadIdx.x);

    // s-direction split: ds < 0 -> G_s^+, ds > 0 -> G_s^-
    {
      const bool pos = ds < 0.0;
      const double wa = pos ? W.v[0] : W.v[2], wb = pos ? W.v[1] : W.v[3];
      const double wt = ds != 0.0 ? wa * ds + wb * dn : 0.0;
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
      const double wa = pos ? W.v[4] : W.v[6], wb = pos ? W.v[5] : W.v[7];
      const bool used = dn > 0.0 || (pos && interior);
      const double wt = used ? wa * ds + wb * dn : 0.0;
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
  const int i = point_index<kBlock>(G.xcd);
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

// Local time step on LDS tables: each staged slot carries 1/speed^2 of its
// point, so an edge costs |d|^2 / speed_j^2 and one square root per point
// ends the minimum: dt_i = CFL sqrt(min_j |d_ij|^2 / speed_j^2).
struct XyW {
  double2 xy;
  double w;
};

template <int BLK, int KMAX>
__global__ void __launch_bounds__(BLK) k_local_dt_t(Geo G, Flow P, Tiles T,
                                                       const double *__restrict__ U,
                                                       double *__restrict__ dt) {
  extern __shared__ __align__(64) unsigned char smem[];
  const int n = G.n;
  const int tile = block_id(G.xcd);
  const int lo = tile * BLK;
  if (lo >= n) return;
  const int cap = BLK + T.hmax;
  double2 *s_xy = reinterpret_cast<double2 *>(smem);
  double *s_w = reinterpret_cast<double *>(smem + 16 * (size_t)cap);
  const int i = lo + threadIdx.x;
  const int c = i < n ? G.cnt[i] : 0;
  SlotRegs<KMAX ? KMAX : 1> sr;
  if (KMAX && i < n) sr.load(T.lcol + i, n, c, threadIdx.x);
  stage_tile<BLK, XyW>(
      T, tile, lo, n,
      [&](int p) {
        double rho, u, v, pr;
        prim_from_cons(P.gamma, ld4(U, p), rho, u, v, pr);
        const double speed = sqrt(u * u + v * v) + 3.0 * sqrt(pr / rho);
        return XyW{G.xy[p], 1.0 / (speed * speed)};
      },
      [&](int sl, const XyW &r) {
        s_xy[sl] = r.xy;
        s_w[sl] = r.w;
      });
  __syncthreads();
  if (i >= n) return;
  const double2 xi = s_xy[threadIdx.x];
  double best = INFINITY;
  auto edge = [&](int sl) {
    const double2 xj = s_xy[sl];
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    best = fmin(best, (dx * dx + dy * dy) * s_w[sl]);
  };
  if (KMAX) {
#pragma unroll
    for (int k = 0; k < (KMAX ? KMAX : 1); ++k)
      if (k < c) edge(sr.s[k]);
  } else {
    const SlotRow row{T.lcol + i, n, c, (int)threadIdx.x};
    for (int k = 0; k < c; ++k) edge(row(k));
  }
  dt[i] = P.cfl * sqrt(best);
}

__global__ void __launch_bounds__(kBlock) k_rk_stage(Geo G, Flow P, int stage,
                                                     const double *__restrict__ Un,
                                                     const double *__restrict__ R,
                                                     const double *__restrict__ dt,
                                                     double *__restrict__ U) {
  const int n = G.n;
  const int i = point_index<kBlock>(G.xcd);
  if (i >= n) return;
  const int kind = G.kind[i];
  F4 Ui;
  if (kind == 2) {
    Ui = ld4(G.uinf, G.cloud[i]);
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

// Classical RK4 stage with L = -R: the stage inputs are Un - dt/2 R0,
// Un - dt/2 R1, Un - dt R2 and the step ends at Un - dt/6 (R0 + 2 R1 + 2 R2 + R3).
// acc carries the partial weighted sum of the stage residuals.
__global__ void __launch_bounds__(kBlock) k_rk4_stage(Geo G, Flow P, int stage,
                                                      const double *__restrict__ Un,
                                                      const double *__restrict__ R,
                                                      const double *__restrict__ dt,
                                                      double *__restrict__ acc,
                                                      double *__restrict__ U) {
  const int n = G.n;
  const int i = point_index<kBlock>(G.xcd);
  if (i >= n) return;
  const int kind = G.kind[i];
  F4 Ui;
  if (kind == 2) {
    Ui = ld4(G.uinf, G.cloud[i]);
  } else {
    const F4 U0 = ld4(Un, i), Ri = ld4(R, i);
    F4 A;
    if (stage == 0) {
      A = Ri;
    } else {
      A = ld4(acc, i);
      for (int m = 0; m < 4; ++m) A.v[m] = A.v[m] + (stage == 3 ? 1.0 : 2.0) * Ri.v[m];
    }
    if (stage < 3) st4(acc, i, A);
    const double h = stage < 2 ? 0.5 * dt[i] : (stage == 2 ? dt[i] : dt[i] / 6.0);
    const F4 &D = stage < 3 ? Ri : A;
    for (int m = 0; m < 4; ++m) Ui.v[m] = U0.v[m] - h * D.v[m];
    if (kind == 1) {
      const double2 nv = G.nrm[i];
      const double mn = Ui.v[1] * nv.x + Ui.v[2] * nv.y;
      Ui.v[1] = Ui.v[1] - mn * nv.x;
      Ui.v[2] = Ui.v[2] - mn * nv.y;
    }
  }
  st4(U, i, Ui);
}

__global__ void __launch_bounds__(kBlock) k_init_state(Geo G, double *__restrict__ U) {
  const int n = G.n;
  const int i = point_index<kBlock>(G.xcd);
  if (i >= n) return;
  F4 Ui = ld4(G.uinf, G.cloud[i]);
  if (G.kind[i] == 1) {
    const double2 nv = G.nrm[i];
    const double mn = Ui.v[1] * nv.x + Ui.v[2] * nv.y;
    Ui.v[1] = Ui.v[1] - mn * nv.x;
    Ui.v[2] = Ui.v[2] - mn * nv.y;
  }
  st4(U, i, Ui);
}

// Dirichlet rows: the free stream of its cloud at every outer point.
__global__ void __launch_bounds__(kBlock) k_far_field(Geo G, double *__restrict__ U) {
  const int i = point_index<kBlock>(G.xcd);
  if (i >= G.n || G.kind[i] != 2) return;
  st4(U, i, ld4(G.uinf, G.cloud[i]));
}

__global__ void k_copy(size_t count, const double *__restrict__ src, double *__restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride)
    dst[k] = src[k];
}

// Residual norms per cloud.  Each cloud's points are cut into fixed chunks
// (chunk table built with the plan); block b sums R_rho^2 over the non-outer
// points of chunk b, every thread walking a fixed strided subset.
__global__ void __launch_bounds__(kBlock) k_norm_partial(const int2 *__restrict__ chunks,
                                                         const int8_t *kind,
                                                         const double *__restrict__ R,
                                                         double *__restrict__ partial) {
  __shared__ double lds[kBlock];
  const int2 ch = chunks[blockIdx.x];
  double s = 0.0;
  for (int i = ch.x + (int)threadIdx.x; i < ch.y; i += kBlock) {
    const double r = R[4 * (size_t)i];
    if (kind[i] != 2) s += r * r;
  }
  const double t = block_sum(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Block c combines the partials of cloud c (chunks [first[c], first[c+1]))
// in a fixed order and writes its norm to out[row * n_clouds + c], where row
// is *counter when a counter is given (graph replays append rows; rows past
// `capacity` are not written), else 0.
__global__ void __launch_bounds__(kBlock) k_norm_final(const int32_t *__restrict__ first,
                                                       const double *__restrict__ partial,
                                                       int n_clouds, const int32_t *counter,
                                                       int capacity, double *__restrict__ out) {
  __shared__ double lds[kBlock];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int k = first[c] + (int)threadIdx.x; k < first[c + 1]; k += kBlock) s += partial[k];
  const double t = block_sum(s, lds);
  if (threadIdx.x == 0) {
    const int row = counter ? *counter : 0;
    if (row < capacity) out[(size_t)row * n_clouds + c] = sqrt(t);
  }
}

// Advance the iteration counter of graph replays (one thread).
__global__ void k_tick(int32_t *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] += 1;
}

// Zero the iteration counter (a kernel, so that it can sit inside graphs).
__global__ void k_zero_counter(int32_t *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0;
}

// Lift and drag of cloud c (block c): wall polygon wall[woff[c] .. woff[c+1]),
// trapezoidal pressure per edge, fixed-order reduction.
__global__ void __launch_bounds__(kBlock) k_force(Geo G, Flow P, const int32_t *__restrict__ woff,
                                                  const int32_t *__restrict__ wall,
                                                  const double *__restrict__ mach,
                                                  const double *__restrict__ aoa,
                                                  const double *__restrict__ U,
                                                  double *__restrict__ clcd) {
  __shared__ double lds[kBlock];
  const int c = blockIdx.x;
  const int w0 = woff[c], nw = woff[c + 1] - woff[c];
  const double pinf = 1.0 / P.gamma;
  const double qinf = 0.5 * mach[c] * mach[c];
  double fx = 0.0, fy = 0.0;
  for (int e = threadIdx.x; e < nw; e += kBlock) {
    const int a = wall[w0 + e], b = wall[w0 + (e + 1) % nw];
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
    const double ca = cos(aoa[c]), sa = sin(aoa[c]);
    clcd[2 * c] = Cy * ca - Cx * sa;
    clcd[2 * c + 1] = Cx * ca + Cy * sa;
  }
}

}  // namespace lskum_impl

using namespace lskum_impl;

struct lskum_graph_s {
  lskum_plan_s *plan = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
};

namespace lskum_impl {

int tile_slots(int32_t n, int32_t width, int blk, const int32_t *ids, const int32_t *cnt,
               std::vector<int32_t> &slots, std::vector<int32_t> &hoff,
               std::vector<int32_t> &hids, int &hmax) {
  const int32_t nt = (n + blk - 1) / blk;
  std::vector<int32_t> ext;
  hmax = 0;
  try {
    slots.resize((size_t)width * n);
    hoff.assign((size_t)nt + 1, 0);
    hids.clear();
    hids.reserve((size_t)n);
    for (int32_t t = 0; t < nt; ++t) {
      const int32_t lo = t * blk, hi = std::min(n, lo + blk);
      ext.clear();
      for (int32_t i = lo; i < hi; ++i)
        for (int32_t s = 0; s < cnt[i]; ++s) {
          const int32_t j = ids[(size_t)s * n + i];
          if (j < lo || j >= hi) ext.push_back(j);
        }
      std::sort(ext.begin(), ext.end());
      ext.erase(std::unique(ext.begin(), ext.end()), ext.end());
      if ((int64_t)blk + (int64_t)ext.size() > 65535) return LSKUM_ERR_INVALID_ARG;
      hmax = std::max(hmax, (int)ext.size());
      hoff[(size_t)t + 1] = hoff[(size_t)t] + (int32_t)ext.size();
      hids.insert(hids.end(), ext.begin(), ext.end());
      for (int32_t i = lo; i < hi; ++i)
        for (int32_t s = 0; s < width; ++s) {
          const int32_t j = s < cnt[i] ? ids[(size_t)s * n + i] : i;
          slots[(size_t)s * n + i] =
              (j >= lo && j < hi)
                  ? j - lo
                  : blk + (int32_t)(std::lower_bound(ext.begin(), ext.end(), j) - ext.begin());
        }
    }
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  return LSKUM_OK;
}

namespace {

// Tile map of tile size blk from the host connectivity (column-major, pads =
// own id): every row entry's LDS slot as uint16, and each tile's halo.
int build_tile_map(lskum_plan_s *p, int blk, const int32_t *nbr, const int32_t *cnt) {
  TileMap &m = p->maps[tile_index(blk)];
  if (m.blk == blk) return LSKUM_OK;
  std::vector<int32_t> slots, hoff, hids;
  std::vector<uint16_t> lcol;
  int hmax = 0;
  int rc = tile_slots(p->n, p->k_pad, blk, nbr, cnt, slots, hoff, hids, hmax);
  if (rc) return rc;
  try {
    lcol.assign(slots.begin(), slots.end());
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  if ((rc = upload(&m.lcol, lcol.data(), lcol.size())) ||
      (rc = upload(&m.hoff, hoff.data(), hoff.size())) ||
      (rc = upload(&m.hids, hids.data(), hids.size())))
    return rc;
  m.hmax = (hmax + 3) / 4 * 4;
  m.blk = blk;
  return LSKUM_OK;
}

}  // namespace

int ensure_tile_map(lskum_plan_s *p) {
  if (p->maps[tile_index(p->block)].blk == p->block) return LSKUM_OK;
  std::vector<int32_t> nbr((size_t)p->n * p->k_pad), cnt((size_t)p->n);
  if (hipMemcpy(nbr.data(), p->nbr, nbr.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(cnt.data(), p->cnt, cnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
          hipSuccess)
    return LSKUM_ERR_HIP;
  return build_tile_map(p, p->block, nbr.data(), cnt.data());
}

int q_vars_launch(lskum_plan_s *p, const double *U, double *q, void *stream) {
  const Flow f = flow(p);
  k_q_vars<<<grid_for(p->n), kBlock, 0, S(stream)>>>(p->n, p->xcd, f.gamma, f.inv_gm1, U, q,
                                                     p->status);
  return launched();
}

// tiled derivative launches: slot rows in registers for rows of <= 32 entries
#define LSKUM_DERIV_T(kern, blk, kmax_ok, ...)                                        \
  do {                                                                                \
    if (kmax_ok) kern<__VA_ARGS__, 32><<<gr, blk, lds, st>>>(g, t, ARGS_);            \
    else kern<__VA_ARGS__, 0><<<gr, blk, lds, st>>>(g, t, ARGS_);                     \
  } while (0)

int deriv_first_launch(lskum_plan_s *p, const double *q, double *dq, double *qlim,
                       int8_t *argext, void *stream) {
  const Geo g = geo(p);
  const int gr = grid_for(p->n, p->block);
  hipStream_t st = S(stream);
  const TileMap &m = p->maps[tile_index(p->block)];
  const size_t lds = (size_t)(p->block + m.hmax) * 48;
  if (m.blk == p->block && lds <= kTileLdsBytes) {
    const Tiles t = tiles(m);
    const bool k32 = p->k_pad <= 32;
#define ARGS_ q, dq, qlim, argext
    switch (p->block) {
      case 128:
        if (argext) LSKUM_DERIV_T(k_deriv_first_t, 128, k32, 128, true);
        else LSKUM_DERIV_T(k_deriv_first_t, 128, k32, 128, false);
        break;
      case 512:
        if (argext) LSKUM_DERIV_T(k_deriv_first_t, 512, k32, 512, true);
        else LSKUM_DERIV_T(k_deriv_first_t, 512, k32, 512, false);
        break;
      default:
        if (argext) LSKUM_DERIV_T(k_deriv_first_t, 256, k32, 256, true);
        else LSKUM_DERIV_T(k_deriv_first_t, 256, k32, 256, false);
        break;
    }
#undef ARGS_
    return launched();
  }
  switch (p->block) {
    case 128:
      if (argext) k_deriv_first<128, true><<<gr, 128, 0, st>>>(g, q, dq, qlim, argext);
      else k_deriv_first<128, false><<<gr, 128, 0, st>>>(g, q, dq, qlim, nullptr);
      break;
    case 512:
      if (argext) k_deriv_first<512, true><<<gr, 512, 0, st>>>(g, q, dq, qlim, argext);
      else k_deriv_first<512, false><<<gr, 512, 0, st>>>(g, q, dq, qlim, nullptr);
      break;
    default:
      if (argext) k_deriv_first<256, true><<<gr, 256, 0, st>>>(g, q, dq, qlim, argext);
      else k_deriv_first<256, false><<<gr, 256, 0, st>>>(g, q, dq, qlim, nullptr);
      break;
  }
  return launched();
}

int deriv_inner_launch(lskum_plan_s *p, const double *dq0, const double *dqp, double *dqn,
                       void *stream) {
  const TileMap &m = p->maps[tile_index(p->block)];
  const size_t lds = (size_t)(p->block + m.hmax) * 80;
  if (m.blk == p->block && lds <= kTileLdsBytes) {
    const int gr = grid_for(p->n, p->block);
    const Tiles t = tiles(m);
    const Geo g = geo(p);
    hipStream_t st = S(stream);
    const bool k32 = p->k_pad <= 32;
#define ARGS_ dq0, dqp, dqn
    switch (p->block) {
      case 128: LSKUM_DERIV_T(k_deriv_inner_t, 128, k32, 128); break;
      case 512: LSKUM_DERIV_T(k_deriv_inner_t, 512, k32, 512); break;
      default: LSKUM_DERIV_T(k_deriv_inner_t, 256, k32, 256); break;
    }
#undef ARGS_
    return launched();
  }
  LSKUM_TILED(k_deriv_inner, p, stream, geo(p), dq0, dqp, dqn);
  return launched();
}

int local_dt_launch(lskum_plan_s *p, const double *U, double *dt, void *stream) {
  const TileMap &m = p->maps[tile_index(p->block)];
  const size_t lds = (size_t)(p->block + m.hmax) * 24;
  const Geo g = geo(p);
  const Flow f = flow(p);
  hipStream_t st = S(stream);
  if (m.blk == p->block && lds <= kTileLdsBytes) {
    const int gr = grid_for(p->n, p->block);
    const Tiles t = tiles(m);
    const bool k32 = p->k_pad <= 32;
#define LSKUM_DT_T(blk)                                                                  \
  do {                                                                                   \
    if (k32) k_local_dt_t<blk, 32><<<gr, blk, lds, st>>>(g, f, t, U, dt);                \
    else k_local_dt_t<blk, 0><<<gr, blk, lds, st>>>(g, f, t, U, dt);                     \
  } while (0)
    switch (p->block) {
      case 128: LSKUM_DT_T(128); break;
      case 512: LSKUM_DT_T(512); break;
      default: LSKUM_DT_T(256); break;
    }
#undef LSKUM_DT_T
    return launched();
  }
  k_local_dt<<<grid_for(p->n), kBlock, 0, st>>>(g, f, U, dt);
  return launched();
}

}  // namespace lskum_impl

namespace {

bool params_ok(const lskum_params *p) {
  return p && std::isfinite(p->gamma) && p->gamma > 1.0 && std::isfinite(p->mach) &&
         p->mach >= 0.0 && std::isfinite(p->aoa_rad) && std::isfinite(p->cfl) && p->cfl > 0.0 &&
         std::isfinite(p->venkat_k) && p->venkat_k >= 0.0 && p->n_inner >= 0 &&
         p->n_inner <= 64 &&
         (p->options & ~(LSKUM_FIRST_ORDER | LSKUM_MINMAX | LSKUM_RK4)) == 0;
}

// every cloud valid, and the settings the kernels share equal across clouds
bool batch_params_ok(int32_t nc, const lskum_params *p) {
  if (!p || nc < 1) return false;
  for (int32_t c = 0; c < nc; ++c) {
    if (!params_ok(p + c)) return false;
    if (p[c].gamma != p[0].gamma || p[c].cfl != p[0].cfl || p[c].venkat_k != p[0].venkat_k ||
        p[c].n_inner != p[0].n_inner || p[c].options != p[0].options)
      return false;
  }
  return true;
}

bool tuning_ok(const lskum_tuning *t) {
  return !t || ((t->block == 0 || t->block == 128 || t->block == 256 || t->block == 512) &&
                (t->xcd_contiguous == 0 || t->xcd_contiguous == 1));
}

void free_stream_state(const lskum_params &q, double U[4]) {
  const double rho = 1.0, u = q.mach * std::cos(q.aoa_rad), v = q.mach * std::sin(q.aoa_rad);
  U[0] = rho;
  U[1] = rho * u;
  U[2] = rho * v;
  U[3] = (1.0 / q.gamma) / (q.gamma - 1.0) + 0.5 * rho * (u * u + v * v);
}

void release(lskum_plan_s *p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  void *bufs[] = {p->xy,     p->nrm,  p->kind,   p->nbr,         p->cnt,     p->cloud,
                  p->wall,   p->woff, p->uinf,   p->mach,        p->aoa,     p->chunks,
                  p->chunk_first, p->partial, p->norm_scratch, p->counter, p->status,
                  p->in_cnt, p->in_ent, p->spw, p->lsg, p->outer, p->ooff};
  for (void *b : bufs) (void)hipFree(b);
  for (TileMap &m : p->maps) {
    (void)hipFree(m.lcol);
    (void)hipFree(m.hoff);
    (void)hipFree(m.hids);
  }
  (void)hipSetDevice(cur);
  delete p;
}

constexpr size_t kNumWorkFields = 4 + 4 + 8 + 8 + 16 + 4 + 1 + 4;  // Un q dq qlim work R dt acc

// Validate one cloud and append it (point ids shifted by base) to the
// concatenated host arrays.
int append_cloud(const lskum_cloud *c, int32_t kp, int32_t base, int32_t cloud_id,
                 std::vector<int32_t> &rows, std::vector<double2> &xy, std::vector<double2> &nrm,
                 std::vector<int8_t> &kind, std::vector<int32_t> &cnt, std::vector<int32_t> &cid,
                 std::vector<int32_t> &wall) {
  if (!c || c->n < 1 || c->k_pad != kp || !c->x || !c->y || !c->nx || !c->ny || !c->kind ||
      !c->row_ptr || !c->col || !c->nbr_count || c->n_wall < 0 || (c->n_wall > 0 && !c->wall_loop))
    return LSKUM_ERR_INVALID_ARG;
  const int32_t n = c->n;
  if (c->row_ptr[0] != 0) return LSKUM_ERR_BAD_CLOUD;
  for (int32_t i = 0; i < n; ++i) {
    const int64_t b = c->row_ptr[i], e = c->row_ptr[i + 1];
    const int32_t k = c->nbr_count[i];
    if (e - b != kp || k < 2 || k > kp) return LSKUM_ERR_BAD_CLOUD;
    if (c->kind[i] < 0 || c->kind[i] > 2) return LSKUM_ERR_BAD_CLOUD;
    if (!std::isfinite(c->x[i]) || !std::isfinite(c->y[i]) || !std::isfinite(c->nx[i]) ||
        !std::isfinite(c->ny[i]))
      return LSKUM_ERR_BAD_CLOUD;
    for (int32_t s = 0; s < kp; ++s) {
      int32_t j = c->col[b + s];
      if (s < k) {
        if (j < 0 || j >= n || j == i) return LSKUM_ERR_BAD_CLOUD;
      } else {
        j = i;  // padding is always the point itself
      }
      rows.push_back(base + j);
    }
    xy.push_back(make_double2(c->x[i], c->y[i]));
    nrm.push_back(make_double2(c->nx[i], c->ny[i]));
    kind.push_back(c->kind[i]);
    cnt.push_back(k);
    cid.push_back(cloud_id);
  }
  std::vector<char> on_loop((size_t)n, 0);
  for (int32_t e = 0; e < c->n_wall; ++e) {
    const int32_t w = c->wall_loop[e];
    if (w < 0 || w >= n || c->kind[w] != 1 || on_loop[(size_t)w]) return LSKUM_ERR_BAD_CLOUD;
    on_loop[(size_t)w] = 1;
    wall.push_back(base + w);
  }
  return LSKUM_OK;
}

int upload_uinf(lskum_plan_s *p) {
  std::vector<double> u((size_t)4 * p->n_clouds), mach(p->n_clouds), aoa(p->n_clouds);
  for (int32_t c = 0; c < p->n_clouds; ++c) {
    free_stream_state(p->params[c], &u[4 * (size_t)c]);
    mach[c] = p->params[c].mach;
    aoa[c] = p->params[c].aoa_rad;
  }
  if (hipMemcpy(p->uinf, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(p->mach, mach.data(), mach.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(p->aoa, aoa.data(), aoa.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess)
    return LSKUM_ERR_HIP;
  return LSKUM_OK;
}

// flux launch for the plan's tile size and scheme variant
#define LSKUM_FLUX(p, stream, ...)                                                           \
  do {                                                                                       \
    const int g_ = grid_for((p)->n, (p)->block);                                             \
    const int v_ = flux_variant(p);                                                          \
    switch ((p)->block * 4 + v_) {                                                           \
      case 128 * 4 + 0: k_flux<128, 0><<<g_, 128, 0, S(stream)>>>(__VA_ARGS__); break;       \
      case 128 * 4 + 1: k_flux<128, 1><<<g_, 128, 0, S(stream)>>>(__VA_ARGS__); break;       \
      case 128 * 4 + 2: k_flux<128, 2><<<g_, 128, 0, S(stream)>>>(__VA_ARGS__); break;       \
      case 512 * 4 + 0: k_flux<512, 0><<<g_, 512, 0, S(stream)>>>(__VA_ARGS__); break;       \
      case 512 * 4 + 1: k_flux<512, 1><<<g_, 512, 0, S(stream)>>>(__VA_ARGS__); break;       \
      case 512 * 4 + 2: k_flux<512, 2><<<g_, 512, 0, S(stream)>>>(__VA_ARGS__); break;       \
      case 256 * 4 + 1: k_flux<256, 1><<<g_, 256, 0, S(stream)>>>(__VA_ARGS__); break;       \
      case 256 * 4 + 2: k_flux<256, 2><<<g_, 256, 0, S(stream)>>>(__VA_ARGS__); break;       \
      default: k_flux<256, 0><<<g_, 256, 0, S(stream)>>>(__VA_ARGS__); break;                \
    }                                                                                        \
  } while (0)

int norm_launch(lskum_plan_s *p, const double *R, double *out, const int32_t *counter,
                int capacity, void *stream) {
  k_norm_partial<<<p->n_chunks, kBlock, 0, S(stream)>>>(p->chunks, p->kind, R, p->partial);
  k_norm_final<<<p->n_clouds, kBlock, 0, S(stream)>>>(p->chunk_first, p->partial, p->n_clouds,
                                                      counter, capacity, out);
  return launched();
}

// First-order solve, then n_inner sweeps.  work holds two [n][8] fields:
// the first-order solution (kept through the sweeps) and the ping-pong
// partner of dq, arranged so that the last sweep writes dq.
int q_derivs_launch(lskum_plan_s *p, const double *q, double *dq, double *qlim, double *work,
                    void *stream) {
  const int ni = p->params[0].n_inner;
  if (ni == 0) return deriv_first_launch(p, q, dq, qlim, nullptr, stream);
  double *dq0 = work + (size_t)8 * p->n;
  int rc = deriv_first_launch(p, q, dq0, qlim, nullptr, stream);
  const double *prev = dq0;
  for (int k = 1; k <= ni && rc == LSKUM_OK; ++k) {
    double *next = ((ni - k) % 2 == 0) ? dq : work;
    rc = deriv_inner_launch(p, dq0, prev, next, stream);
    prev = next;
  }
  return rc;
}

// The iteration body shared by lskum_iterate and graph capture.  With a
// counter, norms go to hist[*counter] and the counter advances after each
// iteration (graph replays); without one, iteration k writes hist[k].
int run_iterations(lskum_plan_s *p, int32_t iters, double *U, double *hist, int32_t hist_rows,
                   void *ws, int32_t *counter, void *stream) {
  const size_t n = (size_t)p->n;
  const size_t f1 = align256(n * sizeof(double));
  char *base = static_cast<char *>(ws);
  double *Un = reinterpret_cast<double *>(base);
  double *q = reinterpret_cast<double *>(base + 4 * f1);
  double *dq = reinterpret_cast<double *>(base + 8 * f1);
  double *qlim = reinterpret_cast<double *>(base + 16 * f1);
  double *work = reinterpret_cast<double *>(base + 24 * f1);
  double *R = reinterpret_cast<double *>(base + 40 * f1);
  double *dt = reinterpret_cast<double *>(base + 44 * f1);
  double *acc = reinterpret_cast<double *>(base + 45 * f1);
  const bool rk4 = (p->params[0].options & LSKUM_RK4) != 0;
  const Geo g = geo(p);
  const Flow f = flow(p);
  const int grid = grid_for(p->n);
  const int copy_grid = grid_for((int)std::min<size_t>(4 * n, (size_t)1 << 24));
  int rc;
  for (int32_t it = 0; it < iters; ++it) {
    if ((rc = local_dt_launch(p, U, dt, stream))) return rc;
    k_copy<<<copy_grid, kBlock, 0, S(stream)>>>(4 * n, U, Un);
    for (int s = 0; s < 4; ++s) {
      if ((rc = q_vars_launch(p, U, q, stream))) return rc;
      // the first-order flux reads no derivatives
      if (flux_variant(p) != 1 && (rc = q_derivs_launch(p, q, dq, qlim, work, stream))) return rc;
      LSKUM_FLUX(p, stream, g, f, p->spw, q, dq, qlim, R, p->status);
      if (s == 0) {
        if (counter)
          rc = norm_launch(p, R, hist ? hist : p->norm_scratch, counter, hist ? hist_rows : 1,
                           stream);
        else
          rc = norm_launch(p, R, hist ? hist + (size_t)it * p->n_clouds : p->norm_scratch,
                           nullptr, 1, stream);
        if (rc) return rc;
      }
      if (rk4)
        k_rk4_stage<<<grid, kBlock, 0, S(stream)>>>(g, f, s, Un, R, dt, acc, U);
      else
        k_rk_stage<<<grid, kBlock, 0, S(stream)>>>(g, f, s, Un, R, dt, U);
    }
    if (counter) k_tick<<<1, 64, 0, S(stream)>>>(counter);
  }
  return launched();
}

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

int lskum_batch_plan_create(lskum_plan *out, int32_t n_clouds, const lskum_cloud *clouds,
                            const lskum_params *params, const lskum_tuning *tuning,
                            void *stream) {
  if (!out) return LSKUM_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_clouds < 1 || !clouds || !batch_params_ok(n_clouds, params) || !tuning_ok(tuning))
    return LSKUM_ERR_INVALID_ARG;
  const int32_t kp = clouds[0].k_pad;
  int64_t total = 0;
  for (int32_t c = 0; c < n_clouds; ++c) total += clouds[c].n;
  if (kp < 1 || total < 1 || total > INT32_MAX / 2 || total * (int64_t)kp > (int64_t)INT32_MAX * 4)
    return LSKUM_ERR_INVALID_ARG;
  const int32_t n = (int32_t)total;
  // host validation, concatenation (ids shifted per cloud)
  std::vector<int32_t> rows, cnt, cid, wall, woff(1, 0), offset(1, 0);
  std::vector<double2> xy, nrm;
  std::vector<int8_t> kind;
  try {
    rows.reserve((size_t)n * kp);
    xy.reserve(n);
    nrm.reserve(n);
    kind.reserve(n);
    cnt.reserve(n);
    cid.reserve(n);
    for (int32_t c = 0; c < n_clouds; ++c) {
      const int rc = append_cloud(clouds + c, kp, offset.back(), c, rows, xy, nrm, kind, cnt, cid,
                                  wall);
      if (rc) return rc;
      offset.push_back(offset.back() + clouds[c].n);
      woff.push_back((int32_t)wall.size());
    }
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  // column-major connectivity
  std::vector<int32_t> nbr((size_t)n * kp);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t s = 0; s < kp; ++s) nbr[(size_t)s * n + i] = rows[(size_t)i * kp + s];
  rows.clear();
  rows.shrink_to_fit();
  // largest in-degree (the width of the adjoint's transposed connectivity)
  int32_t k_in = 1;
  try {
    std::vector<int32_t> indeg((size_t)n, 0);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t s = 0; s < cnt[(size_t)i]; ++s) {
        const int32_t d = ++indeg[(size_t)nbr[(size_t)s * n + i]];
        if (d > k_in) k_in = d;
      }
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  // residual-norm chunks, per cloud
  std::vector<int2> chunks;
  std::vector<int32_t> chunk_first(1, 0);
  for (int32_t c = 0; c < n_clouds; ++c) {
    for (int32_t a = offset[c]; a < offset[c + 1]; a += kNormChunk)
      chunks.push_back(make_int2(a, std::min(a + kNormChunk, offset[c + 1])));
    chunk_first.push_back((int32_t)chunks.size());
  }
  lskum_plan_s *p = new (std::nothrow) lskum_plan_s();
  if (!p) return LSKUM_ERR_NO_MEMORY;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return LSKUM_ERR_HIP;
  }
  p->n = n;
  p->k_pad = kp;
  p->n_clouds = n_clouds;
  p->n_wall = (int32_t)wall.size();
  p->n_chunks = (int32_t)chunks.size();
  p->k_in = k_in;
  p->params.assign(params, params + n_clouds);
  p->offset = offset;
  if (tuning) {
    p->block = tuning->block ? tuning->block : 256;
    p->xcd = tuning->xcd_contiguous;
  }
  int rc = LSKUM_OK;
  if (rc == LSKUM_OK) rc = upload(&p->xy, xy.data(), xy.size());
  if (rc == LSKUM_OK) rc = upload(&p->nrm, nrm.data(), nrm.size());
  if (rc == LSKUM_OK) rc = upload(&p->kind, kind.data(), kind.size());
  if (rc == LSKUM_OK) rc = upload(&p->nbr, nbr.data(), nbr.size());
  if (rc == LSKUM_OK) rc = upload(&p->cnt, cnt.data(), cnt.size());
  if (rc == LSKUM_OK) rc = upload(&p->cloud, cid.data(), cid.size());
  if (rc == LSKUM_OK) rc = upload(&p->wall, wall.data(), wall.size());
  if (rc == LSKUM_OK) rc = upload(&p->woff, woff.data(), woff.size());
  if (rc == LSKUM_OK) rc = upload(&p->chunks, chunks.data(), chunks.size());
  if (rc == LSKUM_OK) rc = upload(&p->chunk_first, chunk_first.data(), chunk_first.size());
  if (rc == LSKUM_OK && (hipMalloc((void **)&p->uinf, 4 * sizeof(double) * n_clouds) != hipSuccess ||
                         hipMalloc((void **)&p->mach, sizeof(double) * n_clouds) != hipSuccess ||
                         hipMalloc((void **)&p->aoa, sizeof(double) * n_clouds) != hipSuccess ||
                         hipMalloc((void **)&p->partial, sizeof(double) * chunks.size()) != hipSuccess ||
                         hipMalloc((void **)&p->norm_scratch, sizeof(double) * n_clouds) != hipSuccess ||
                         hipMalloc((void **)&p->counter, sizeof(int32_t)) != hipSuccess ||
                         hipMalloc((void **)&p->status, sizeof(unsigned)) != hipSuccess))
    rc = LSKUM_ERR_NO_MEMORY;
  if (rc == LSKUM_OK) rc = upload_uinf(p);
  if (rc == LSKUM_OK) rc = build_tile_map(p, p->block, nbr.data(), cnt.data());
  if (rc == LSKUM_OK && hipMalloc((void **)&p->spw, (size_t)n * 8 * sizeof(double)) != hipSuccess)
    rc = LSKUM_ERR_NO_MEMORY;
  if (rc == LSKUM_OK) {
    k_split_weights<<<grid_for(n), kBlock, 0, S(stream)>>>(geo(p), p->spw);
    rc = launched();
  }
  if (rc == LSKUM_OK && (hipMemsetAsync(p->status, 0, sizeof(unsigned), S(stream)) != hipSuccess ||
                         hipMemsetAsync(p->counter, 0, sizeof(int32_t), S(stream)) != hipSuccess ||
                         hipStreamSynchronize(S(stream)) != hipSuccess))
    rc = LSKUM_ERR_HIP;
  if (rc != LSKUM_OK) {
    release(p);
    return rc;
  }
  *out = p;
  return LSKUM_OK;
}

int lskum_plan_create(lskum_plan *out, const lskum_cloud *cloud, const lskum_params *params,
                      void *stream) {
  if (!out) return LSKUM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!cloud || !params_ok(params)) return LSKUM_ERR_INVALID_ARG;
  return lskum_batch_plan_create(out, 1, cloud, params, nullptr, stream);
}

int lskum_plan_destroy(lskum_plan p) {
  if (!p) return LSKUM_ERR_INVALID_ARG;
  release(p);
  return LSKUM_OK;
}

int lskum_plan_set_params(lskum_plan p, const lskum_params *params) {
  if (!p || !batch_params_ok(p->n_clouds, params)) return LSKUM_ERR_INVALID_ARG;
  p->params.assign(params, params + p->n_clouds);
  return upload_uinf(p);
}

int lskum_plan_set_tuning(lskum_plan p, const lskum_tuning *tuning) {
  if (!p || !tuning || !tuning_ok(tuning)) return LSKUM_ERR_INVALID_ARG;
  p->block = tuning->block ? tuning->block : 256;
  p->xcd = tuning->xcd_contiguous;
  return ensure_tile_map(p);
}

int32_t lskum_plan_n(lskum_plan p) { return p ? p->n : -1; }

int32_t lskum_plan_clouds(lskum_plan p) { return p ? p->n_clouds : -1; }

int32_t lskum_plan_offset(lskum_plan p, int32_t cloud) {
  if (!p || cloud < 0 || cloud > p->n_clouds) return -1;
  return p->offset[cloud];
}

int lskum_init_state(lskum_plan p, double *U, void *stream) {
  if (!p || !a32(U)) return LSKUM_ERR_INVALID_ARG;
  k_init_state<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), U);
  return launched();
}

int lskum_set_far_field(lskum_plan p, double *U, void *stream) {
  if (!p || !a32(U)) return LSKUM_ERR_INVALID_ARG;
  k_far_field<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), U);
  return launched();
}

int lskum_q_vars(lskum_plan p, const double *U, double *q, void *stream) {
  if (!p || !a32(U) || !a32(q)) return LSKUM_ERR_INVALID_ARG;
  return q_vars_launch(p, U, q, stream);
}

int lskum_q_derivs(lskum_plan p, const double *q, double *dq, double *qlim, double *work,
                   void *stream) {
  if (!p || !a32(q) || !a64(dq) || !a64(qlim) || (p->params[0].n_inner > 0 && !a64(work)))
    return LSKUM_ERR_INVALID_ARG;
  return q_derivs_launch(p, q, dq, qlim, work, stream);
}

int lskum_flux_residual(lskum_plan p, const double *q, const double *dq, const double *qlim,
                        double *R, void *stream) {
  if (!p || !a32(q) || !a64(dq) || !a64(qlim) || !a32(R)) return LSKUM_ERR_INVALID_ARG;
  LSKUM_FLUX(p, stream, geo(p), flow(p), p->spw, q, dq, qlim, R, p->status);
  return launched();
}

int lskum_local_dt(lskum_plan p, const double *U, double *dt, void *stream) {
  if (!p || !a32(U) || !dt) return LSKUM_ERR_INVALID_ARG;
  return local_dt_launch(p, U, dt, stream);
}

int lskum_rk_stage(lskum_plan p, int stage, const double *Un, const double *R, const double *dt,
                   double *U, void *stream) {
  if (!p || !a32(Un) || !a32(R) || !dt || !a32(U) || stage < 0 || stage > 3)
    return LSKUM_ERR_INVALID_ARG;
  k_rk_stage<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), flow(p), stage, Un, R, dt, U);
  return launched();
}

int lskum_rk4_stage(lskum_plan p, int stage, const double *Un, const double *R, const double *dt,
                    double *acc, double *U, void *stream) {
  if (!p || !a32(Un) || !a32(R) || !dt || !a32(acc) || !a32(U) || stage < 0 || stage > 3)
    return LSKUM_ERR_INVALID_ARG;
  k_rk4_stage<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), flow(p), stage, Un, R, dt, acc,
                                                        U);
  return launched();
}

int lskum_residual_norm(lskum_plan p, const double *R, double *out, void *stream) {
  if (!p || !a32(R) || !out) return LSKUM_ERR_INVALID_ARG;
  return norm_launch(p, R, out, nullptr, 1, stream);
}

int lskum_force_coeffs(lskum_plan p, const double *U, double *clcd, void *stream) {
  if (!p || !a32(U) || !clcd) return LSKUM_ERR_INVALID_ARG;
  k_force<<<p->n_clouds, kBlock, 0, S(stream)>>>(geo(p), flow(p), p->woff, p->wall, p->mach,
                                                 p->aoa, U, clcd);
  return launched();
}

size_t lskum_workspace_bytes(lskum_plan p) {
  if (!p) return 0;
  return kNumWorkFields * align256((size_t)p->n * sizeof(double));
}

int lskum_iterate(lskum_plan p, int32_t iters, double *U, double *hist, void *ws, void *stream) {
  if (!p || !a32(U) || !ws || iters < 0 || ((uintptr_t)ws % 256) != 0) return LSKUM_ERR_INVALID_ARG;
  return run_iterations(p, iters, U, hist, iters, ws, nullptr, stream);
}

int lskum_graph_create(lskum_graph *out, lskum_plan p, int32_t iters, double *U, double *hist,
                       int32_t hist_rows, void *ws, void *stream) {
  if (!out) return LSKUM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!p || iters < 1 || !a32(U) || !ws || ((uintptr_t)ws % 256) != 0 ||
      (hist && hist_rows < 1))
    return LSKUM_ERR_INVALID_ARG;
  lskum_graph_s *g = new (std::nothrow) lskum_graph_s();
  if (!g) return LSKUM_ERR_NO_MEMORY;
  g->plan = p;
  int rc = LSKUM_OK;
  if (hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking) != hipSuccess) rc = LSKUM_ERR_HIP;
  if (rc == LSKUM_OK &&
      hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
    rc = LSKUM_ERR_HIP;
  if (rc == LSKUM_OK) {
    const int r2 = run_iterations(p, iters, U, hist, hist_rows, ws, p->counter, g->capture);
    const hipError_t e = hipStreamEndCapture(g->capture, &g->graph);
    if (r2 != LSKUM_OK) rc = r2;
    else if (e != hipSuccess) rc = LSKUM_ERR_HIP;
  }
  if (rc == LSKUM_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = LSKUM_ERR_HIP;
  if (rc == LSKUM_OK) {
    // start the history at row 0 (a kernel on the caller's stream)
    k_zero_counter<<<1, 64, 0, S(stream)>>>(p->counter);
    rc = launched();
  }
  if (rc != LSKUM_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->capture) (void)hipStreamDestroy(g->capture);
    delete g;
    return rc;
  }
  *out = g;
  return LSKUM_OK;
}

int lskum_graph_launch(lskum_graph g, void *stream) {
  if (!g || !g->exec) return LSKUM_ERR_INVALID_ARG;
  return hipGraphLaunch(g->exec, S(stream)) == hipSuccess ? LSKUM_OK : LSKUM_ERR_HIP;
}

int lskum_graph_destroy(lskum_graph g) {
  if (!g) return LSKUM_ERR_INVALID_ARG;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->capture) (void)hipStreamDestroy(g->capture);
  delete g;
  return LSKUM_OK;
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
