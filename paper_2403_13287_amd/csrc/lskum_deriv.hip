// lskum_deriv.hip -- gfx950 kernels of the least-squares q-derivatives and
// of the local time step (arXiv 2403.13287, eq. (9), (14)-(15)), with their
// launchers.  These are gathers bound by memory latency and LDS traffic; the
// library compiles this file with the iterative-ILP scheduler of the AMDGPU
// back end, which makes them about 5 % faster than the default one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "lskum.h"
#include "lskum_impl.h"

namespace lskum_impl {

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
// Block b stages in LDS the records of the points of tile b (up to BLK
// consecutive points, fewer where their halo would make the table exceed
// 2 BLK slots) and of their out-of-tile neighbours (the tile's halo, a few
// hundred points for a Hilbert-ordered cloud), loaded by all threads at
// once: the halo ids, then the records, are the only dependent round trips;
// each row is stored as table slots (uint16), so the gather loop reads LDS
// only.  Same arithmetic, in the same order, as k_deriv_first and
// k_deriv_inner, which remain the path for clouds whose halos do not fit.

// Reader of point i's row of table slots; entries past the count return
// the point's own slot (prefetching ahead never leaves the row).
struct SlotRow {
  const uint16_t *lcol;  // [groups][n][8]
  int n, i, c, own;
  __device__ __forceinline__ int operator()(int k) const {
    const int kk = k < c ? k : c - 1;
    const int sl = lcol[((size_t)(kk >> 3) * n + i) * 8 + (kk & 7)];
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
  if (tile >= T.ntiles) return;  // blocks past the last tile (the grid is a multiple of 8)
  const int lo = T.tlo[tile], hi = T.tlo[tile + 1];
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
  int c = 0;
  SlotGroups<KMAX ? KMAX : 8> sr;
  stage_tile<BLK, XyQ>(
      T, tile, lo, hi, hi - lo, [&](int p) { return XyQ{G.xy[p], ld4(q, p)}; },
      [&](int sl, const XyQ &r) {
        s_xy[sl] = r.xy;
        s_q[sl] = make_double2(r.q.v[0], r.q.v[1]);
        s_q[cap + sl] = make_double2(r.q.v[2], r.q.v[3]);
      },
      [&] {
        const int ic = i < hi ? i : hi - 1;
        c = G.cnt[ic];
        if (KMAX) sr.load(T.lcol, n, ic, T.groups);
      });
  __syncthreads();
  if (i >= hi) return;
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
      if (k < c) edge(k, sr[k]);
  } else {
    const SlotRow row{T.lcol, n, i, c, (int)threadIdx.x};
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
  if (tile >= T.ntiles) return;  // blocks past the last tile (the grid is a multiple of 8)
  const int lo = T.tlo[tile], hi = T.tlo[tile + 1];
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
  int c = 0;
  SlotGroups<KMAX ? KMAX : 8> sr;
  F8 d0{};  // the first-order solution, loaded with the table
  stage_tile<BLK, XyG>(
      T, tile, lo, hi, hi - lo, [&](int p) { return XyG{G.xy[p], ld8(dqp, p)}; },
      [&](int sl, const XyG &r) {
        s_xy[sl] = r.xy;
        for (int h = 0; h < 4; ++h) s_g[h * cap + sl] = make_double2(r.g.v[2 * h], r.g.v[2 * h + 1]);
      },
      [&] {
        const int ic = i < hi ? i : hi - 1;
        c = G.cnt[ic];
        if (KMAX) sr.load(T.lcol, n, ic, T.groups);
        d0 = ld8(dq0, ic);
      });
  __syncthreads();
  if (i >= hi) return;
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
      if (k < c) edge(sr[k]);
  } else {
    const SlotRow row{T.lcol, n, i, c, (int)threadIdx.x};
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
  F8 g;
  for (int m = 0; m < 4; ++m) {
    g.v[m] = d0.v[m] + 0.5 * g0.v[m] - 0.5 * ((syy * ax[m] - sxy * ay[m]) / det);
    g.v[4 + m] = d0.v[4 + m] + 0.5 * g0.v[4 + m] - 0.5 * ((sxx * ay[m] - sxy * ax[m]) / det);
  }
  st8(dqn, i, g);
}

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
  if (tile >= T.ntiles) return;  // blocks past the last tile (the grid is a multiple of 8)
  const int lo = T.tlo[tile], hi = T.tlo[tile + 1];
  const int cap = BLK + T.hmax;
  double2 *s_xy = reinterpret_cast<double2 *>(smem);
  double *s_w = reinterpret_cast<double *>(smem + 16 * (size_t)cap);
  const int i = lo + threadIdx.x;
  int c = 0;
  SlotGroups<KMAX ? KMAX : 8> sr;
  stage_tile<BLK, XyW>(
      T, tile, lo, hi, hi - lo,
      [&](int p) {
        double rho, u, v, pr;
        prim_from_cons(P.gamma, ld4(U, p), rho, u, v, pr);
        const double speed = sqrt(u * u + v * v) + 3.0 * sqrt(pr / rho);
        return XyW{G.xy[p], 1.0 / (speed * speed)};
      },
      [&](int sl, const XyW &r) {
        s_xy[sl] = r.xy;
        s_w[sl] = r.w;
      },
      [&] {
        const int ic = i < hi ? i : hi - 1;
        c = G.cnt[ic];
        if (KMAX) sr.load(T.lcol, n, ic, T.groups);
      });
  __syncthreads();
  if (i >= hi) return;
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
      if (k < c) edge(sr[k]);
  } else {
    const SlotRow row{T.lcol, n, i, c, (int)threadIdx.x};
    for (int k = 0; k < c; ++k) edge(row(k));
  }
  dt[i] = P.cfl * sqrt(best);
}

}  // namespace lskum_impl

// ---------------------------------------------------------------------------
// launchers

namespace lskum_impl {

// tiled derivative launches: slot rows in registers for rows of <= 32 entries
#define LSKUM_DERIV_T(kern, blk, kmax_ok, ...)                                        \
  do {                                                                                \
    if (kmax_ok) kern<__VA_ARGS__, 32><<<gr, blk, lds, st>>>(g, t, ARGS_);            \
    else kern<__VA_ARGS__, 0><<<gr, blk, lds, st>>>(g, t, ARGS_);                     \
  } while (0)

// The derivative passes and the local time step walk XCD-contiguous ranges
// whatever the plan's block mapping: a tile's halo then sits in the L2 of
// the XCD that runs the tile.  The flux kernel, which gains more from an
// even spread of the work over the XCDs, follows the plan's mapping.
inline Geo gather_geo(const lskum_plan_s *p) {
  Geo g = geo(p);
  g.xcd = 1;
  return g;
}

int deriv_first_launch(lskum_plan_s *p, const double *q, double *dq, double *qlim,
                       int8_t *argext, void *stream) {
  const Geo g = gather_geo(p);
  hipStream_t st = S(stream);
  const TileMap &m = p->maps[tile_index(p->block)];
  const size_t lds = (size_t)(p->block + m.hmax) * 48;
  if (m.blk == p->block && lds <= kTileLdsBytes) {
    const int gr = grid_tiles(m.ntiles);
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
  const int gd = grid_for(p->n, p->block);
  switch (p->block) {
    case 128:
      if (argext) k_deriv_first<128, true><<<gd, 128, 0, st>>>(g, q, dq, qlim, argext);
      else k_deriv_first<128, false><<<gd, 128, 0, st>>>(g, q, dq, qlim, nullptr);
      break;
    case 512:
      if (argext) k_deriv_first<512, true><<<gd, 512, 0, st>>>(g, q, dq, qlim, argext);
      else k_deriv_first<512, false><<<gd, 512, 0, st>>>(g, q, dq, qlim, nullptr);
      break;
    default:
      if (argext) k_deriv_first<256, true><<<gd, 256, 0, st>>>(g, q, dq, qlim, argext);
      else k_deriv_first<256, false><<<gd, 256, 0, st>>>(g, q, dq, qlim, nullptr);
      break;
  }
  return launched();
}

int deriv_inner_launch(lskum_plan_s *p, const double *dq0, const double *dqp, double *dqn,
                       void *stream) {
  const TileMap &m = p->maps[tile_index(p->block)];
  const size_t lds = (size_t)(p->block + m.hmax) * 80;
  if (m.blk == p->block && lds <= kTileLdsBytes) {
    const int gr = grid_tiles(m.ntiles);
    const Tiles t = tiles(m);
    const Geo g = gather_geo(p);
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
  LSKUM_TILED(k_deriv_inner, p, stream, gather_geo(p), dq0, dqp, dqn);
  return launched();
}

int local_dt_launch(lskum_plan_s *p, const double *U, double *dt, void *stream) {
  const TileMap &m = p->maps[tile_index(p->block)];
  const size_t lds = (size_t)(p->block + m.hmax) * 24;
  const Geo g = gather_geo(p);
  const Flow f = flow(p);
  hipStream_t st = S(stream);
  if (m.blk == p->block && lds <= kTileLdsBytes) {
    const int gr = grid_tiles(m.ntiles);
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
