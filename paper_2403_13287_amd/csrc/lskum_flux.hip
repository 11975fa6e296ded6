// lskum_flux.hip -- gfx950 kernel of the flux residual (arXiv 2403.13287,
// eq. (10)-(12) with the modified q of eq. (14)) and its launcher.  The
// kernel is bound by FP64 issue at two waves per SIMD; it has a file of its
// own so that its compiler settings are chosen apart from the gathers'.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "lskum.h"
#include "lskum_impl.h"

namespace lskum_impl {

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
// VAR: 0 the default scheme, 1 first-order flux (q~ = q), 2 min-max limiter.
// FUSE: then the point's SSP stage update, which reads only the point's own
// residual, state, U^n and dt, and the q-variables of its new state into
// S.q_next (the next stage's q; the q read here stays unchanged for the
// other threads' neighbour loads).
// G14: gamma = 1.4, known when compiled: the end states' density needs no
// log, and the kernel carries neither the general-gamma branch nor that
// branch's constants, which otherwise hold vector registers through the
// loop (192 -> 179 VGPRs).
template <int BLK, int VAR, bool FUSE, bool G14>
__global__ void __launch_bounds__(BLK) k_flux(Geo G, Flow P, const double *__restrict__ spw,
                                                 const double *__restrict__ q,
                                                 const double *__restrict__ dq,
                                                 const double *__restrict__ qlim,
                                                 double *__restrict__ R, unsigned *status,
                                                 StageArgs S) {
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
  // the stage update and next q of this point, once its residual r is known
  auto finish = [&](const F4 &r, unsigned f) {
    st4(R, i, r);
    if (FUSE) {
      const F4 Uc = ld4(S.U, i);
      if (S.stage == 0) st4(S.Un, i, Uc);
      const F4 Ui = ssp_stage(G, i, kind, S.stage, S.Un, Uc, r, S.dt[i]);
      st4(S.U, i, Ui);
      F4 qn;
      f |= q_of_state(P, Ui, qn);
      st4(S.q_next, i, qn);
    }
    flag(status, f);
  };
  if (kind == 2) {
    finish(F4{{0.0, 0.0, 0.0, 0.0}}, 0u);
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
    f |= end_state<G14 ? 1 : 0>(qtj, P, tx, ty, nx, ny, sj);
    f |= end_state<G14 ? 1 : 0>(qt0, P, tx, ty, nx, ny, s0);

    // s-direction split: ds < 0 -> G_s^+, ds > 0 -> G_s^-
    {
      const bool pos = ds < 0.0;
      // only the pair of the side the edge falls on is read: plane 0 (s+) or 1 (s-)
      const double2 wp = s_w[pos ? 0 : 1][threadIdx.x];
      const double wa = wp.x, wb = wp.y;
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
      const double2 wp = s_w[pos ? 2 : 3][threadIdx.x];  // n+ or n-
      const double wa = wp.x, wb = wp.y;
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
  finish(r, f);
}

}  // namespace lskum_impl

namespace lskum_impl {

// The flux launch for the plan's scheme variant.  The flux kernel stages
// only its own block's records (it has no tile tables), so its block size is
// independent of the plan's tile size and tuned on its own (64, 128 or 256
// points; 64 by default: one-wavefront blocks shorten the tail of each
// launch).  Results do not depend on it (each point's sums run in its row
// order).
template <int BLK>
void flux_launch_blk(lskum_plan_s *p, const Geo &g, const Flow &f, const double *q,
                     const double *dq, const double *qlim, double *R, hipStream_t st,
                     const StageArgs *stage) {
  const int gr = grid_for(p->n, BLK);
  const StageArgs sa = stage ? *stage : StageArgs{-1, nullptr, nullptr, nullptr, nullptr};
#define LSKUM_FLUX_G(var, g14)                                                          \
  do {                                                                                  \
    if (stage)                                                                          \
      k_flux<BLK, var, true, g14><<<gr, BLK, 0, st>>>(g, f, p->spw, q, dq, qlim, R,    \
                                                       p->status, sa);                 \
    else                                                                                \
      k_flux<BLK, var, false, g14><<<gr, BLK, 0, st>>>(g, f, p->spw, q, dq, qlim, R,   \
                                                        p->status, sa);                \
  } while (0)
#define LSKUM_FLUX_V(var)        \
  do {                           \
    if (f.gamma_is_14)           \
      LSKUM_FLUX_G(var, true);   \
    else                         \
      LSKUM_FLUX_G(var, false);  \
  } while (0)
  switch (flux_variant(p)) {
    case 1: LSKUM_FLUX_V(1); break;
    case 2: LSKUM_FLUX_V(2); break;
    default: LSKUM_FLUX_V(0); break;
  }
#undef LSKUM_FLUX_V
#undef LSKUM_FLUX_G
}

int flux_launch(lskum_plan_s *p, const double *q, const double *dq, const double *qlim,
                double *R, void *stream, const StageArgs *stage) {
  const Geo g = geo(p);
  const Flow f = flow(p);
  hipStream_t st = S(stream);
  switch (p->flux_block) {
    case 128: flux_launch_blk<128>(p, g, f, q, dq, qlim, R, st, stage); break;
    case 256: flux_launch_blk<256>(p, g, f, q, dq, qlim, R, st, stage); break;
    default: flux_launch_blk<64>(p, g, f, q, dq, qlim, R, st, stage); break;
  }
  return launched();
}

}  // namespace lskum_impl
