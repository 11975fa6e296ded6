// lskum_adjoint.hip -- vector-Jacobian products of the residual sweep and of
// the force coefficients (gfx950).
//
// Reverse mode written by hand over the forward formulas (arXiv 2403.13287,
// eq. (9)-(15) and the kinetic split fluxes of eq. (2)-(3)), differentiating
// the branch the forward takes at every limiter, stencil max/min and split
// membership test.  Nothing is stored between the forward and the adjoint:
// a VJP call recomputes q, the first-order derivatives with the slots that
// attain the stencil bounds, and every inner-iteration iterate, then runs the
// passes backwards.
//
// Every kernel writes only its own point's outputs, so results are
// deterministic.  Where the forward gathers from neighbours (point i reads
// point j's data), the reverse has to send cotangents from i to j; that
// transposed direction is also a gather, over the in-edges of j (the rows
// that list j), kept as a padded column-major table built once per plan.
//
// Adjoint data of a plan (device, built by the first VJP call):
//   in_cnt int32 [n]       in-degree of each point
//   in_ent int32 [k_in][n] column-major: entry e of point j is
//                          (slot << 25) | i for the e-th row i listing j (at
//                          `slot`), sorted by i then slot; k_in = largest
//                          in-degree
//   lsg    F8    [n]       least-squares geometry: M^-1 = [[a, b], [b, c]] of
//                          the point's normal matrix, and sum of its edge
//                          vectors (sdx, sdy)
//   outer, ooff            outer points of each cloud

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "lskum.h"
#include "lskum_impl.h"

namespace lskum_impl {
namespace {

constexpr double kInvSqrtPi = 0.56418958354775628695;  // 1 / sqrt(pi)

// ---------------------------------------------------------------------------
// reverse of the point formulas

// Cotangents of limited(delta, room_max, room_min, eps2) = phi*delta given
// the cotangent ob of its result: of delta, and of the room it used
// (sel = +1: room_max, -1: room_min, 0: none).
struct LimRev {
  double ddelta, droom;
  int sel;
};

__device__ __forceinline__ LimRev limited_rev(double delta, double room_max, double room_min,
                                              double eps2, double ob) {
  if (delta == 0.0) return LimRev{ob, 0.0, 0};
  const double D = delta > 0.0 ? room_max : room_min;
  const double num = D * D + eps2 + 2.0 * delta * D;
  const double den = D * D + 2.0 * delta * delta + delta * D + eps2;
  const double r = lskum_math::lk_div1(num, den);  // the forward's quotient
  if (!(r < 1.0)) return LimRev{ob, 0.0, 0};  // phi = 1
  // r = num/den: dr/ddelta = (2D - r (4 delta + D))/den,
  //              dr/dD     = (2D + 2 delta - r (2D + delta))/den
  const double rden = lk_div(1.0, den);
  const double r_delta = (2.0 * D - r * (4.0 * delta + D)) * rden;
  const double r_D = (2.0 * D + 2.0 * delta - r * (2.0 * D + delta)) * rden;
  return LimRev{ob * (r + delta * r_delta), ob * delta * r_D, delta > 0.0 ? 1 : -1};
}

// cotangents of the fields of EndState
struct EndBar {
  double rho, us, un, p, E, sqb, bcoef;
};

// Reverse of split_flux: Gb = cotangent of G (mass, d-momentum, o-momentum,
// energy); adds to the end-state cotangents and to those of ud and uo.
__device__ __forceinline__ void split_flux_rev(double sg, const EndState &s, double ud, double uo,
                                               const double Gb[4], EndBar &b, double &udb,
                                               double &uob) {
  const double S = ud * s.sqb;
  const double ex = lskum_math::lk_exp(-(S * S));
  const double A = 0.5 * (1.0 + sg * lskum_math::lk_erf(S));
  const double B = ex * s.bcoef;
  const double F = ud * A + sg * B;
  const double Fb = Gb[0] * s.rho + Gb[2] * s.rho * uo;
  b.rho += Gb[0] * F + Gb[1] * (ud * ud * A + sg * ud * B) + Gb[2] * uo * F;
  uob += Gb[2] * s.rho * F;
  const double Ab = Gb[1] * (s.p + s.rho * ud * ud) + Gb[3] * (s.E + s.p) * ud + Fb * ud;
  const double Bb = sg * (Gb[1] * s.rho * ud + Gb[3] * (s.E + 0.5 * s.p) + Fb);
  double u_b = Gb[1] * (2.0 * s.rho * ud * A + sg * s.rho * B) + Gb[3] * (s.E + s.p) * A + Fb * A;
  b.p += Gb[1] * A + Gb[3] * (ud * A + 0.5 * sg * B);
  b.E += Gb[3] * F;
  // A = (1 + sg erf S)/2, B = exp(-S^2) bcoef, S = ud sqrt(beta)
  const double Sb = Ab * sg * kInvSqrtPi * ex - 2.0 * S * B * Bb;
  b.bcoef += Bb * ex;
  u_b += Sb * s.sqb;
  b.sqb += Sb * ud;
  udb += u_b;
}

// Reverse of end_state: cotangent of the modified q from that of the state.
__device__ __forceinline__ void end_state_rev(const Flow &P, double tx, double ty, double nx,
                                              double ny, const EndState &s, const EndExtra &x,
                                              const EndBar &b, double qb[4]) {
  const double a = P.inv_gm1;
  const double inv2b = 0.5 * x.ib;
  // E = p a + rho uu / 2
  double pb = b.p + a * b.E;
  double rhob = b.rho + 0.5 * x.uu * b.E;
  double uub = 0.5 * s.rho * b.E;
  // (us, un) = rotation of (u, v)
  double ub = b.us * tx + b.un * nx;
  double vb = b.us * ty + b.un * ny;
  // p = rho / (2 beta)
  rhob += pb * inv2b;
  double betab = -pb * s.p * x.ib;
  // rho = exp(q1 + beta uu) beta^(-a)
  qb[0] = rhob * s.rho;
  uub += rhob * s.rho * x.beta;
  betab += rhob * s.rho * (x.uu - a * x.ib);
  // uu = u^2 + v^2
  ub += 2.0 * x.u * uub;
  vb += 2.0 * x.v * uub;
  // u = q2 / (2 beta), v = q3 / (2 beta)
  qb[1] = ub * inv2b;
  qb[2] = vb * inv2b;
  betab -= (ub * x.u + vb * x.v) * x.ib;
  // sqb = sqrt(beta), bcoef = 1/(2 sqrt(pi beta))
  betab += 0.5 * b.sqb * s.sqb * x.ib - 0.5 * b.bcoef * s.bcoef * x.ib;
  // beta = -q4 / 2
  qb[3] = -0.5 * betab;
}

// ---------------------------------------------------------------------------
// flux residual, reverse
//
// Point i's residual holds, per edge (i, j) and split, wt (G(q~_j) - G(q~_i))
// with wt a least-squares weight of i's half-plane stencil (geometry only).
// The two ends of an edge therefore reverse independently, each from the
// seed of row i rotated into i's frame:
//   own end (q~_i): k_flux_rev_own, one thread per row i over its edges;
//   neighbour end (q~_j): k_flux_gather, one thread per point j over the
//     rows that list it, recomputing each edge from the source's half-plane
//     weights (computed with the plan), normal and seed.
// Neither end's intermediate is stored: the reverse of an edge end is
// recomputed where its cotangent is consumed.

// Weights and seeds of edge d = x_j - x_i of row i: split weights wt_s, wt_n
// (zero for an unused split), signs, and the seeds of both splits in their
// (mass, d-momentum, o-momentum, energy) order, times `sign` (+1 for the
// neighbour end, -1 for the own end).
struct EdgeSeed {
  double ds, dn, sg_s, sg_n, wt_s, wt_n;
  double Gs[4], Gn[4];
};

__device__ __forceinline__ EdgeSeed edge_seed(double dx, double dy, double tx, double ty, double nx,
                                              double ny, bool interior, const F8 &W,
                                              const double ab[4], double sign) {
  EdgeSeed e;
  e.ds = dot_rn(dx, tx, dy, ty);
  e.dn = dot_rn(dx, nx, dy, ny);
  const bool s_pos = e.ds < 0.0, n_pos = e.dn < 0.0;
  const double sa = s_pos ? W.v[0] : W.v[2], sb = s_pos ? W.v[1] : W.v[3];
  const double na = n_pos ? W.v[4] : W.v[6], nb = n_pos ? W.v[5] : W.v[7];
  e.wt_s = e.ds != 0.0 ? sa * e.ds + sb * e.dn : 0.0;
  e.wt_n = (e.dn > 0.0 || (n_pos && interior)) ? na * e.ds + nb * e.dn : 0.0;
  e.sg_s = s_pos ? 1.0 : -1.0;
  e.sg_n = n_pos ? 1.0 : -1.0;
  const double ws = sign * e.wt_s, wn = sign * e.wt_n;
  e.Gs[0] = ws * ab[0];
  e.Gs[1] = ws * ab[1];
  e.Gs[2] = ws * ab[2];
  e.Gs[3] = ws * ab[3];
  e.Gn[0] = wn * ab[0];
  e.Gn[1] = wn * ab[2];
  e.Gn[2] = wn * ab[1];
  e.Gn[3] = wn * ab[3];
  return e;
}

// Seed of row i in its own frame: R = rotation of (mass, s-momentum,
// n-momentum, energy).
__device__ __forceinline__ void frame_seed(const F4 &rb, double tx, double ty, double nx,
                                           double ny, double ab[4]) {
  ab[0] = rb.v[0];
  ab[1] = rb.v[1] * tx + rb.v[2] * ty;
  ab[2] = rb.v[1] * nx + rb.v[2] * ny;
  ab[3] = rb.v[3];
}

// Reverse of one end of one edge: the end's record (qe, ge, le), the edge
// vector d as row i sees it and row i's frame.  Adds the cotangents of the
// end's q, dq and qlim records to qb, gb, lb.
template <bool G14>
__device__ __forceinline__ unsigned end_reverse(const Flow &P, const F4 &qe, const F8 &ge,
                                                const F8 &le, double dx, double dy, double eps2,
                                                double tx, double ty, double nx, double ny,
                                                const EdgeSeed &e, double qb[4], double gb[8],
                                                double lb[8]) {
  double qt[4], d[4], rmax[4], rmin[4];
  for (int m = 0; m < 4; ++m) {
    d[m] = half_step(dx, dy, ge.v[m], ge.v[4 + m]);
    rmax[m] = le.v[m] - qe.v[m];
    rmin[m] = le.v[4 + m] - qe.v[m];
    qt[m] = qe.v[m] + limited(d[m], rmax[m], rmin[m], eps2);
  }
  EndState st;
  EndExtra ex;
  const unsigned f = end_state_t<true, G14 ? 1 : 0>(qt, P, tx, ty, nx, ny, st, &ex);
  EndBar b{0, 0, 0, 0, 0, 0, 0};
  if (e.wt_s != 0.0) split_flux_rev(e.sg_s, st, st.us, st.un, e.Gs, b, b.us, b.un);
  if (e.wt_n != 0.0) split_flux_rev(e.sg_n, st, st.un, st.us, e.Gn, b, b.un, b.us);
  double qtb[4];
  end_state_rev(P, tx, ty, nx, ny, st, ex, b, qtb);
  // q~ = q + phi delta, delta = -(d . grad q)/2
  for (int m = 0; m < 4; ++m) {
    const LimRev r = limited_rev(d[m], rmax[m], rmin[m], eps2, qtb[m]);
    // the room is qlim - q: its cotangent goes to the bound used and, with
    // the opposite sign, to q (selects, not an indexed update, so the
    // accumulators stay in registers)
    const double to_max = r.sel > 0 ? r.droom : 0.0;
    const double to_min = r.sel < 0 ? r.droom : 0.0;
    qb[m] += qtb[m] - (to_max + to_min);
    gb[m] += -0.5 * dx * r.ddelta;
    gb[4 + m] += -0.5 * dy * r.ddelta;
    lb[m] += to_max;
    lb[4 + m] += to_min;
  }
  return f;
}

// Own end of every edge of row i: writes the own-end parts of qbar_i, gbar_i
// and lbar_i.  The thread's own record is re-read from LDS at every edge
// rather than held in registers through the loop (two waves per SIMD).
// G14: compiled for gamma = 1.4 (as the forward flux kernel).
template <int BLK, bool G14>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(2)))
k_flux_rev_own(Geo G, Flow P, const double *__restrict__ spw, const double *__restrict__ q,
               const double *__restrict__ dq, const double *__restrict__ qlim,
               const double *__restrict__ Rb, double *__restrict__ qbar,
               double *__restrict__ gbar, double *__restrict__ lbar, unsigned *status) {
  __shared__ double2 s_xy[BLK];
  __shared__ double2 s_q[2][BLK];  // 16-byte planes
  __shared__ double2 s_g[4][BLK];
  __shared__ double2 s_l[4][BLK];
  const int n = G.n;
  const int lo = tile_lo<BLK>(G.xcd);
  const int i = lo + threadIdx.x;
  const bool active = i < n;
  {
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
    pl_wr4<BLK>(s_q, threadIdx.x, q0);
    pl_wr8<BLK>(s_g, threadIdx.x, g0);
    pl_wr8<BLK>(s_l, threadIdx.x, l0);
  }
  __syncthreads();
  if (!active) return;
  double qb[4] = {0, 0, 0, 0};
  double gb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double lb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int kind = G.kind[i];
  unsigned f = 0;
  if (kind != 2) {  // outer rows: R = 0 depends on nothing
    const bool interior = kind == 0;
    const double2 xi = s_xy[threadIdx.x];
    const double2 nv = G.nrm[i];
    const double nx = nv.x, ny = nv.y, tx = ny, ty = -nx;
    const F8 W = ld8(spw, i);
    double ab[4];
    frame_seed(ld4(Rb, i), tx, ty, nx, ny, ab);
    const double K = P.venkat_k;
    const int c = G.cnt[i];
    const Row row{G.nbr + i, n, c, i};
    auto fetch_xy = [&](int j) {
      int lj;
      return in_tile<BLK>(j, lo, lj) ? s_xy[lj] : G.xy[j];
    };
    int j_next = row(1);
    double2 xj = fetch_xy(row(0));
    for (int k = 0; k < c; ++k) {
      const int j_after = row(k + 2);
      const double2 xn = fetch_xy(j_next);
      const double dx = xj.x - xi.x, dy = xj.y - xi.y;
      const EdgeSeed e = edge_seed(dx, dy, tx, ty, nx, ny, interior, W, ab, -1.0);
      // keeps the compiler from hoisting the own-record reads out of the loop
      asm volatile("" ::: "memory");
      const F4 q0 = pl_rd4<BLK>(s_q, threadIdx.x);
      const F8 g0 = pl_rd8<BLK>(s_g, threadIdx.x), l0 = pl_rd8<BLK>(s_l, threadIdx.x);
      f |= end_reverse<G14>(P, q0, g0, l0, dx, dy, edge_eps2(K, dx, dy), tx, ty, nx, ny, e, qb, gb, lb);
      xj = xn;
      j_next = j_after;
    }
  }
  st4(qbar, i, F4{{qb[0], qb[1], qb[2], qb[3]}});
  st8(gbar, i, F8{{gb[0], gb[1], gb[2], gb[3], gb[4], gb[5], gb[6], gb[7]}});
  st8(lbar, i, F8{{lb[0], lb[1], lb[2], lb[3], lb[4], lb[5], lb[6], lb[7]}});
  flag(status, f);
}

// s = M^-1 g per component: (s_x, s_y) = [[a, b], [b, c]] (g_x, g_y)
__device__ __forceinline__ void apply_minv(const F8 &L, const double g[8], double s[8]) {
  for (int m = 0; m < 4; ++m) {
    s[m] = L.v[0] * g[m] + L.v[1] * g[4 + m];
    s[4 + m] = L.v[1] * g[m] + L.v[2] * g[4 + m];
  }
}

// Reader of point j's in-edge row (column-major).  Entries at or past the
// in-degree c read the last real entry, and a point with no in-edge reads
// (slot 0, j), so prefetching ahead never leaves the table.
struct InRow {
  const int32_t *ent;  // &in_ent[j], stride n
  int n, c, j;
  __device__ __forceinline__ int operator()(int e) const {
    if (c == 0) return j;
    const int ee = e < c ? e : c - 1;
    return ent[(size_t)ee * n];
  }
};

// Neighbour end of every edge that reads point j, as a gather over j's
// in-edges: each edge (i, j) is recomputed from row i's frame, split
// weights and seed.  Adds the own-end parts left by k_flux_rev_own; in
// place: qbar_j, lbar_j complete, and sbar_j (holding the own-end gbar_j on
// entry) becomes M_j^-1 gbar_j, the seed of the derivative reverse.
template <int BLK, bool G14>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(2)))
k_flux_gather(Geo G, Flow P, const int32_t *__restrict__ in_cnt,
              const int32_t *__restrict__ in_ent, const double *__restrict__ lsg,
              const double *__restrict__ spw, const double *__restrict__ q,
              const double *__restrict__ dq, const double *__restrict__ qlim,
              const double *__restrict__ Rb, double *__restrict__ qbar,
              double *__restrict__ sbar, double *__restrict__ lbar) {
  __shared__ double2 s_xy[BLK];
  __shared__ double2 s_nrm[BLK];
  __shared__ double2 s_w[4][BLK];  // 16-byte planes
  __shared__ double2 s_rb[2][BLK];
  __shared__ double2 s_q[2][BLK];
  __shared__ double2 s_g[4][BLK];
  __shared__ double2 s_l[4][BLK];
  __shared__ int8_t s_kind[BLK];
  const int n = G.n;
  const int lo = tile_lo<BLK>(G.xcd);
  const int j = lo + threadIdx.x;
  const bool active = j < n;
  {
    double2 x = make_double2(0.0, 0.0), nv = x;
    F8 w{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}}, g = w, l = w;
    F4 r{{0.0, 0.0, 0.0, 0.0}}, qq = r;
    int8_t kd = 2;
    if (active) {
      x = G.xy[j];
      nv = G.nrm[j];
      w = ld8(spw, j);
      r = ld4(Rb, j);
      qq = ld4(q, j);
      g = ld8(dq, j);
      l = ld8(qlim, j);
      kd = G.kind[j];
    }
    s_xy[threadIdx.x] = x;
    s_nrm[threadIdx.x] = nv;
    pl_wr8<BLK>(s_w, threadIdx.x, w);
    pl_wr4<BLK>(s_rb, threadIdx.x, r);
    pl_wr4<BLK>(s_q, threadIdx.x, qq);
    pl_wr8<BLK>(s_g, threadIdx.x, g);
    pl_wr8<BLK>(s_l, threadIdx.x, l);
    s_kind[threadIdx.x] = kd;
  }
  __syncthreads();
  if (!active) return;
  double qb[4] = {0, 0, 0, 0};
  double gb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double lb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const double2 xj = s_xy[threadIdx.x];
  const double K = P.venkat_k;
  const int c = in_cnt[j];
  const InRow row{in_ent + j, n, c, j};
  int ent_next = row(0);
  for (int e = 0; e < c; ++e) {
    const int i = ent_next & kPointMask;
    ent_next = row(e + 1);
    int li;
    double2 xi, nv;
    F8 W;
    F4 rb;
    int ki;
    if (in_tile<BLK>(i, lo, li)) {
      ki = s_kind[li];
      xi = s_xy[li];
      nv = s_nrm[li];
      W = pl_rd8<BLK>(s_w, li);
      rb = pl_rd4<BLK>(s_rb, li);
    } else {
      ki = G.kind[i];
      xi = G.xy[i];
      nv = G.nrm[i];
      W = ld8(spw, i);
      rb = ld4(Rb, i);
    }
    if (ki == 2) continue;  // outer rows have no residual
    const double nx = nv.x, ny = nv.y, tx = ny, ty = -nx;
    double ab[4];
    frame_seed(rb, tx, ty, nx, ny, ab);
    // the edge as row i sees it: d = x_j - x_i
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    const EdgeSeed es = edge_seed(dx, dy, tx, ty, nx, ny, ki == 0, W, ab, 1.0);
    asm volatile("" ::: "memory");
    const F4 qj = pl_rd4<BLK>(s_q, threadIdx.x);
    const F8 gj = pl_rd8<BLK>(s_g, threadIdx.x), lj = pl_rd8<BLK>(s_l, threadIdx.x);
    end_reverse<G14>(P, qj, gj, lj, dx, dy, edge_eps2(K, dx, dy), tx, ty, nx, ny, es, qb, gb, lb);
  }
  const F4 qo = ld4(qbar, j);
  const F8 go = ld8(sbar, j), lo8 = ld8(lbar, j);
  for (int m = 0; m < 4; ++m) qb[m] += qo.v[m];
  for (int m = 0; m < 8; ++m) {
    gb[m] += go.v[m];
    lb[m] += lo8.v[m];
  }
  double sv[8];
  apply_minv(ld8(lsg, j), gb, sv);
  st4(qbar, j, F4{{qb[0], qb[1], qb[2], qb[3]}});
  st8(sbar, j, F8{{sv[0], sv[1], sv[2], sv[3], sv[4], sv[5], sv[6], sv[7]}});
  st8(lbar, j, F8{{lb[0], lb[1], lb[2], lb[3], lb[4], lb[5], lb[6], lb[7]}});
}

// ---------------------------------------------------------------------------
// least-squares derivatives, reverse
//
// A derivative pass computes dq_i = M_i^-1 sum_{j in N(i)} d_ij (q~_j - q~_i)
// per component, with q~ = q - (d . g_prev)/2 (inner sweeps, d the edge
// vector seen from i) or q~ = q (first-order pass).  With s_i = M_i^-1 gbar_i
// (M symmetric), the cotangents are
//   qbar_j      += d_ij . s_i                  (every row i listing j)
//   qbar_i      -= (sum_j d_ij) . s_i
//   gbar_prev_j -= d_ij (d_ij . s_i) / 2       (inner sweeps)
//   gbar_prev_i += M_i s_i / 2 = gbar_i / 2    (inner sweeps)
// so the next seed is s_prev_j = s_j/2 - M_j^-1 sum_i d_ij (d_ij . s_i) / 2.

// Point j's part of an inner-sweep reverse, from its in-edge sums
// aq = sum d.s_i, (ax, ay) = sum d (d.s_i) and its own seed sj.
__device__ __forceinline__ void inner_rev_tail(int j, const F8 &sj, const double aq[4],
                                               const double ax[4], const double ay[4],
                                               const double *__restrict__ lsg,
                                               double *__restrict__ qbar,
                                               double *__restrict__ s_out) {
  const F8 L = ld8(lsg, j);
  F4 qb = ld4(qbar, j);
  F8 so;
  for (int m = 0; m < 4; ++m) {
    qb.v[m] += aq[m] - (L.v[3] * sj.v[m] + L.v[4] * sj.v[4 + m]);
    so.v[m] = 0.5 * sj.v[m] - 0.5 * (L.v[0] * ax[m] + L.v[1] * ay[m]);
    so.v[4 + m] = 0.5 * sj.v[4 + m] - 0.5 * (L.v[1] * ax[m] + L.v[2] * ay[m]);
  }
  st4(qbar, j, qb);
  st8(s_out, j, so);
}

template <int BLK>
__global__ void __launch_bounds__(BLK) k_inner_rev(Geo G, const int32_t *__restrict__ in_cnt,
                                                      const int32_t *__restrict__ in_ent,
                                                      const double *__restrict__ lsg,
                                                      const double *__restrict__ s_in,
                                                      double *__restrict__ qbar,
                                                      double *__restrict__ s_out) {
  __shared__ double2 s_xy[BLK];
  __shared__ double2 s_s[4][BLK];  // 16-byte planes
  const int n = G.n;
  const int lo = tile_lo<BLK>(G.xcd);
  const int j = lo + threadIdx.x;
  const bool active = j < n;
  double2 xj = make_double2(0.0, 0.0);
  F8 sj{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
  if (active) {
    xj = G.xy[j];
    sj = ld8(s_in, j);
  }
  s_xy[threadIdx.x] = xj;
  pl_wr8<BLK>(s_s, threadIdx.x, sj);
  __syncthreads();
  if (!active) return;
  auto fetch = [&](int i, double2 &x, F8 &sv) {
    int li;
    if (in_tile<BLK>(i, lo, li)) {
      x = s_xy[li];
      sv = pl_rd8<BLK>(s_s, li);
    } else {
      x = G.xy[i];
      sv = ld8(s_in, i);
    }
  };
  double aq[4] = {0, 0, 0, 0}, ax[4] = {0, 0, 0, 0}, ay[4] = {0, 0, 0, 0};
  const int c = in_cnt[j];
  const InRow row{in_ent + j, n, c, j};
  int ent_next = row(1);
  double2 xi;
  F8 si;
  fetch(row(0) & kPointMask, xi, si);
  for (int e = 0; e < c; ++e) {
    const int ent_after = row(e + 2);
    double2 xn;
    F8 sn;
    fetch(ent_next & kPointMask, xn, sn);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    for (int m = 0; m < 4; ++m) {
      const double t = dx * si.v[m] + dy * si.v[4 + m];
      aq[m] += t;
      ax[m] += dx * t;
      ay[m] += dy * t;
    }
    xi = xn;
    si = sn;
    ent_next = ent_after;
  }
  inner_rev_tail(j, sj, aq, ax, ay, lsg, qbar, s_out);
}

// Point j's part of the first-order reverse and of eq. (13) reverse, from
// the accumulated q cotangent qb (in-edges and bounds) and its own seed sj:
// writes the cotangent of U_j.
__device__ __forceinline__ void first_rev_tail(const Flow &P, int j, const F8 &sj, double qb[4],
                                               const double *__restrict__ lsg,
                                               const double *__restrict__ U,
                                               double *__restrict__ Ubar) {
  const F8 L = ld8(lsg, j);
  for (int m = 0; m < 4; ++m) qb[m] -= L.v[3] * sj.v[m] + L.v[4] * sj.v[4 + m];

  // eq. (13) reverse: q = (ln rho + a ln beta - beta uu, 2 beta u, 2 beta v,
  // -2 beta), beta = rho/(2p), p = (gamma-1)(E - rho uu/2)
  const double g = P.gamma, a = P.inv_gm1;
  double rho, u, v, p;
  prim_from_cons(g, ld4(U, j), rho, u, v, p);
  const double beta = 0.5 * rho / p;
  const double uu = u * u + v * v;
  const double betab = qb[0] * (a / beta - uu) + 2.0 * u * qb[1] + 2.0 * v * qb[2] - 2.0 * qb[3];
  const double rhob = qb[0] / rho + betab / (2.0 * p);
  const double pb = -betab * beta / p;
  const double ub = -2.0 * beta * u * qb[0] + 2.0 * beta * qb[1];
  const double vb = -2.0 * beta * v * qb[0] + 2.0 * beta * qb[2];
  const double gm1 = g - 1.0;
  F4 o;
  o.v[0] = rhob + pb * gm1 * 0.5 * uu - (ub * u + vb * v) / rho;
  o.v[1] = ub / rho - pb * gm1 * u;
  o.v[2] = vb / rho - pb * gm1 * v;
  o.v[3] = pb * gm1;
  st4(Ubar, j, o);
}

// First-order pass, reverse, then eq. (13) reverse: the cotangent of U.
// Stencil bounds route their cotangent to the slot that attained them.
template <int BLK>
__global__ void __launch_bounds__(BLK) k_first_rev(Geo G, Flow P,
                                                      const int32_t *__restrict__ in_cnt,
                                                      const int32_t *__restrict__ in_ent,
                                                      const double *__restrict__ lsg,
                                                      const double *__restrict__ s0,
                                                      const int8_t *__restrict__ argext,
                                                      const double *__restrict__ lbar,
                                                      const double *__restrict__ U,
                                                      const double *__restrict__ qbar,
                                                      double *__restrict__ Ubar) {
  __shared__ double2 s_xy[BLK];
  __shared__ double2 s_s[4][BLK];  // 16-byte planes
  __shared__ uint64_t s_a[BLK];
  const uint64_t *arg = reinterpret_cast<const uint64_t *>(argext);
  const int n = G.n;
  const int lo = tile_lo<BLK>(G.xcd);
  const int j = lo + threadIdx.x;
  const bool active = j < n;
  double2 xj = make_double2(0.0, 0.0);
  F8 sj{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
  uint64_t aj = 0;
  if (active) {
    xj = G.xy[j];
    sj = ld8(s0, j);
    aj = arg[j];
  }
  s_xy[threadIdx.x] = xj;
  pl_wr8<BLK>(s_s, threadIdx.x, sj);
  s_a[threadIdx.x] = aj;
  __syncthreads();
  if (!active) return;
  double qb[4];
  {
    const F4 o = ld4(qbar, j);
    const F8 lo8 = ld8(lbar, j);
    for (int m = 0; m < 4; ++m) {
      qb[m] = o.v[m];
      if ((int8_t)(aj >> (8 * m)) == -1) qb[m] += lo8.v[m];
      if ((int8_t)(aj >> (8 * (4 + m))) == -1) qb[m] += lo8.v[4 + m];
    }
  }
  auto fetch = [&](int i, double2 &x, F8 &sv, uint64_t &a) {
    int li;
    if (in_tile<BLK>(i, lo, li)) {
      x = s_xy[li];
      sv = pl_rd8<BLK>(s_s, li);
      a = s_a[li];
    } else {
      x = G.xy[i];
      sv = ld8(s0, i);
      a = arg[i];
    }
  };
  const int c = in_cnt[j];
  const InRow row{in_ent + j, n, c, j};
  int ent_next = row(1);
  int ent = row(0);
  double2 xi;
  F8 si;
  uint64_t ai;
  fetch(ent & kPointMask, xi, si, ai);
  for (int e = 0; e < c; ++e) {
    const int ent_after = row(e + 2);
    double2 xn;
    F8 sn;
    uint64_t an;
    fetch(ent_next & kPointMask, xn, sn, an);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    for (int m = 0; m < 4; ++m) qb[m] += dx * si.v[m] + dy * si.v[4 + m];
    const int slot = ent >> kSlotShift;
    bool hit = false;
    for (int h = 0; h < 8; ++h) hit |= (int8_t)(ai >> (8 * h)) == slot;
    if (hit) {
      const F8 li8 = ld8(lbar, ent & kPointMask);
      for (int m = 0; m < 4; ++m) {
        if ((int8_t)(ai >> (8 * m)) == slot) qb[m] += li8.v[m];
        if ((int8_t)(ai >> (8 * (4 + m))) == slot) qb[m] += li8.v[4 + m];
      }
    }
    xi = xn;
    si = sn;
    ai = an;
    ent = ent_next;
    ent_next = ent_after;
  }
  first_rev_tail(P, j, sj, qb, lsg, U, Ubar);
}

// The two reverse gathers above on tile tables of the in-edge rows: the
// coordinates and seeds (and bound slots) of a tile's points and of the
// sources outside it are staged in LDS as 16-byte planes, and each point's
// in-edge entries are held in registers (rows of at most KMAX entries; 0:
// any length, entries read as the loop goes).  Same arithmetic in the same
// order as k_inner_rev and k_first_rev.
struct XyS {
  double2 xy;
  F8 s;
};
struct XySA {  // plain members: a 64-byte aligned F8 member kept this record on the stack
  double2 xy;
  double s[8];
  uint64_t a;
};

template <int BLK, int KMAX>
__global__ void __launch_bounds__(BLK) k_inner_rev_t(Geo G, Tiles T,
                                                        const uint32_t *__restrict__ lent, int rows,
                                                        const int32_t *__restrict__ in_cnt,
                                                        const double *__restrict__ lsg,
                                                        const double *__restrict__ s_in,
                                                        double *__restrict__ qbar,
                                                        double *__restrict__ s_out) {
  extern __shared__ __align__(64) unsigned char smem[];
  const int n = G.n;
  const int tile = block_id(G.xcd);
  if (tile >= T.ntiles) return;  // blocks past the last tile (the grid is a multiple of 8)
  const int lo = T.tlo[tile], hi = T.tlo[tile + 1];
  const int cap = BLK + T.hmax;
  double2 *s_xy = reinterpret_cast<double2 *>(smem);
  double2 *s_s = s_xy + cap;  // 4 planes
  auto rd_s = [&](int sl) {
    F8 r;
    for (int h = 0; h < 4; ++h) {
      const double2 v = s_s[h * cap + sl];
      r.v[2 * h] = v.x;
      r.v[2 * h + 1] = v.y;
    }
    return r;
  };
  const int j = lo + threadIdx.x;
  int c = 0;
  SlotRegs<KMAX ? KMAX : 1, uint32_t> sr;
  stage_tile<BLK, XyS>(
      T, tile, lo, hi, hi - lo, [&](int p) { return XyS{G.xy[p], ld8(s_in, p)}; },
      [&](int sl, const XyS &r) {
        s_xy[sl] = r.xy;
        for (int h = 0; h < 4; ++h) s_s[h * cap + sl] = make_double2(r.s.v[2 * h], r.s.v[2 * h + 1]);
      },
      [&] {
        const int jc = j < hi ? j : hi - 1;
        c = in_cnt[jc];
        if (KMAX) sr.load_rows(lent + jc, n, rows);
      });
  __syncthreads();
  if (j >= hi) return;
  const double2 xj = s_xy[threadIdx.x];
  const F8 sj = rd_s(threadIdx.x);
  double aq[4] = {0, 0, 0, 0}, ax[4] = {0, 0, 0, 0}, ay[4] = {0, 0, 0, 0};
  auto edge = [&](uint32_t ent) {
    const int sl = (int)(ent & 0xffffu);
    const double2 xi = s_xy[sl];
    const F8 si = rd_s(sl);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    for (int m = 0; m < 4; ++m) {
      const double t = dx * si.v[m] + dy * si.v[4 + m];
      aq[m] += t;
      ax[m] += dx * t;
      ay[m] += dy * t;
    }
  };
  if (KMAX) {
#pragma unroll
    for (int e = 0; e < (KMAX ? KMAX : 1); ++e)
      if (e < c) edge((uint32_t)sr.s[e]);
  } else {
    for (int e = 0; e < c; ++e) edge(lent[(size_t)e * n + j]);
  }
  inner_rev_tail(j, sj, aq, ax, ay, lsg, qbar, s_out);
}

template <int BLK, int KMAX>
__global__ void __launch_bounds__(BLK) k_first_rev_t(Geo G, Flow P, Tiles T,
                                                        const uint32_t *__restrict__ lent, int rows,
                                                        const int32_t *__restrict__ in_cnt,
                                                        const double *__restrict__ lsg,
                                                        const double *__restrict__ s0,
                                                        const int8_t *__restrict__ argext,
                                                        const double *__restrict__ lbar,
                                                        const double *__restrict__ U,
                                                        const double *__restrict__ qbar,
                                                        double *__restrict__ Ubar) {
  extern __shared__ __align__(64) unsigned char smem[];
  const uint64_t *arg = reinterpret_cast<const uint64_t *>(argext);
  const int n = G.n;
  const int tile = block_id(G.xcd);
  if (tile >= T.ntiles) return;  // blocks past the last tile (the grid is a multiple of 8)
  const int lo = T.tlo[tile], hi = T.tlo[tile + 1];
  const int cap = BLK + T.hmax;
  double2 *s_xy = reinterpret_cast<double2 *>(smem);
  double2 *s_s = s_xy + cap;                                // 4 planes
  uint64_t *s_a = reinterpret_cast<uint64_t *>(s_s + 4 * cap);
  auto rd_s = [&](int sl) {
    F8 r;
    for (int h = 0; h < 4; ++h) {
      const double2 v = s_s[h * cap + sl];
      r.v[2 * h] = v.x;
      r.v[2 * h + 1] = v.y;
    }
    return r;
  };
  const int j = lo + threadIdx.x;
  int c = 0;
  SlotRegs<KMAX ? KMAX : 1, uint32_t> sr;
  stage_tile<BLK, XySA>(
      T, tile, lo, hi, hi - lo,
      [&](int p) {
        const F8 s = ld8(s0, p);
        return XySA{G.xy[p], {s.v[0], s.v[1], s.v[2], s.v[3], s.v[4], s.v[5], s.v[6], s.v[7]},
                    arg[p]};
      },
      [&](int sl, const XySA &r) {
        s_xy[sl] = r.xy;
        for (int h = 0; h < 4; ++h) s_s[h * cap + sl] = make_double2(r.s[2 * h], r.s[2 * h + 1]);
        s_a[sl] = r.a;
      },
      [&] {
        const int jc = j < hi ? j : hi - 1;
        c = in_cnt[jc];
        if (KMAX) sr.load_rows(lent + jc, n, rows);
      });
  __syncthreads();
  if (j >= hi) return;
  const double2 xj = s_xy[threadIdx.x];
  const F8 sj = rd_s(threadIdx.x);
  const uint64_t aj = s_a[threadIdx.x];
  double qb[4];
  {
    const F4 o = ld4(qbar, j);
    const F8 lo8 = ld8(lbar, j);
    for (int m = 0; m < 4; ++m) {
      qb[m] = o.v[m];
      if ((int8_t)(aj >> (8 * m)) == -1) qb[m] += lo8.v[m];
      if ((int8_t)(aj >> (8 * (4 + m))) == -1) qb[m] += lo8.v[4 + m];
    }
  }
  const int h0 = T.hoff[tile];
  const int hb = hi - lo;  // the tile's points; its halo slots follow
  auto edge = [&](uint32_t ent) {
    const int sl = (int)(ent & 0xffffu);
    const int slot = (int)(ent >> 16);
    const double2 xi = s_xy[sl];
    const F8 si = rd_s(sl);
    const uint64_t ai = s_a[sl];
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    for (int m = 0; m < 4; ++m) qb[m] += dx * si.v[m] + dy * si.v[4 + m];
    bool hit = false;
    for (int h = 0; h < 8; ++h) hit |= (int8_t)(ai >> (8 * h)) == slot;
    if (hit) {
      const int i = sl < hb ? lo + sl : T.hids[h0 + sl - hb];
      const F8 li8 = ld8(lbar, i);
      for (int m = 0; m < 4; ++m) {
        if ((int8_t)(ai >> (8 * m)) == slot) qb[m] += li8.v[m];
        if ((int8_t)(ai >> (8 * (4 + m))) == slot) qb[m] += li8.v[4 + m];
      }
    }
  };
  if (KMAX) {
#pragma unroll
    for (int e = 0; e < (KMAX ? KMAX : 1); ++e)
      if (e < c) edge((uint32_t)sr.s[e]);
  } else {
    for (int e = 0; e < c; ++e) edge(lent[(size_t)e * n + j]);
  }
  first_rev_tail(P, j, sj, qb, lsg, U, Ubar);
}

// theta cotangent of cloud c (block c): the outer rows hold U_inf(M, alpha);
// their cotangents are projected on dU_inf/d(M, alpha) and then cleared.
__global__ void __launch_bounds__(kBlock) k_theta_rev(const int32_t *__restrict__ ooff,
                                                      const int32_t *__restrict__ outer,
                                                      const double *__restrict__ mach,
                                                      const double *__restrict__ aoa,
                                                      double *__restrict__ Ubar,
                                                      double *__restrict__ thetabar) {
  __shared__ double lds[kBlock];
  const int c = blockIdx.x;
  const double M = mach[c], ca = cos(aoa[c]), sa = sin(aoa[c]);
  // U_inf = (1, M cos a, M sin a, p_inf/(gamma-1) + M^2/2)
  double tm = 0.0, ta = 0.0;
  for (int k = ooff[c] + (int)threadIdx.x; k < ooff[c + 1]; k += kBlock) {
    const int j = outer[k];
    const F4 b = ld4(Ubar, j);
    tm += b.v[1] * ca + b.v[2] * sa + b.v[3] * M;
    ta += -b.v[1] * M * sa + b.v[2] * M * ca;
    st4(Ubar, j, F4{{0.0, 0.0, 0.0, 0.0}});
  }
  const double TM = block_sum(tm, lds);
  __syncthreads();
  const double TA = block_sum(ta, lds);
  if (threadIdx.x == 0) {
    thetabar[2 * c] = TM;
    thetabar[2 * c + 1] = TA;
  }
}

// One pseudo-time step of the steady adjoint at every point:
// r = Pi(Ubar - g), Lambda <- Pi(Lambda - dt/2 r), where Pi clears outer
// rows and the normal momentum of wall rows.  |r| is left in Ubar[i][0]
// for the residual norm.
__global__ void __launch_bounds__(kBlock) k_adjoint_step(Geo G, const double *__restrict__ dt,
                                                         const double *__restrict__ g,
                                                         double *__restrict__ Ub,
                                                         double *__restrict__ Lam) {
  const int i = point_index<kBlock>(G.xcd);
  if (i >= G.n) return;
  const int kind = G.kind[i];
  const F4 b = ld4(Ub, i), gi = ld4(g, i);
  F4 r, l = ld4(Lam, i);
  for (int m = 0; m < 4; ++m) r.v[m] = kind == 2 ? 0.0 : b.v[m] - gi.v[m];
  const double h = 0.5 * dt[i];
  for (int m = 0; m < 4; ++m) l.v[m] = kind == 2 ? 0.0 : l.v[m] - h * r.v[m];
  if (kind == 1) {
    const double2 nv = G.nrm[i];
    const double rn = r.v[1] * nv.x + r.v[2] * nv.y;
    r.v[1] -= rn * nv.x;
    r.v[2] -= rn * nv.y;
    const double ln = l.v[1] * nv.x + l.v[2] * nv.y;
    l.v[1] -= ln * nv.x;
    l.v[2] -= ln * nv.y;
  }
  st4(Lam, i, l);
  const double rr = r.v[0] * r.v[0] + r.v[1] * r.v[1] + r.v[2] * r.v[2] + r.v[3] * r.v[3];
  st4(Ub, i, F4{{sqrt(rr), 0.0, 0.0, 0.0}});
}

// Total derivative of an output at a steady state, per cloud and theta
// component k: total = dJ/dtheta|_U - thetabar(Lambda); the partial is also
// copied out when requested.
__global__ void k_adjoint_total(int count, const double *__restrict__ part,
                                const double *__restrict__ tr, double *__restrict__ total,
                                double *__restrict__ partial) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  total[k] = part[k] - tr[k];
  if (partial) partial[k] = part[k];
}

// Least-squares geometry of every point (built once per plan).
__global__ void __launch_bounds__(kBlock) k_ls_geometry(Geo G, double *__restrict__ lsg) {
  const int n = G.n;
  const int i = point_index<kBlock>(G.xcd);
  if (i >= n) return;
  const double2 xi = G.xy[i];
  const int c = G.cnt[i];
  double sxx = 0.0, sxy = 0.0, syy = 0.0, sx = 0.0, sy = 0.0;
  for (int k = 0; k < c; ++k) {
    const double2 xj = G.xy[G.nbr[(size_t)k * n + i]];
    const double dx = xj.x - xi.x, dy = xj.y - xi.y;
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
    sx += dx;
    sy += dy;
  }
  const double det = sxx * syy - sxy * sxy;
  st8(lsg, i, F8{{syy / det, -sxy / det, sxx / det, sx, sy, 0.0, 0.0, 0.0}});
}

// ---------------------------------------------------------------------------
// force coefficients, reverse

__global__ void k_zero(size_t count, double *__restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride)
    dst[k] = 0.0;
}

// Cloud c (block c): with Cx, Cy recomputed, the cotangent Jb = (Jb_l, Jb_d)
// of (Cl, Cd) gives Cx_b = -Jb_l sin a + Jb_d cos a, Cy_b = Jb_l cos a +
// Jb_d sin a, Cp_b(e) = -Cx_b dy_e + Cy_b dx_e, and each wall point takes
// half of the Cp cotangents of its two edges, divided by the dynamic pressure
// (through p(U)).  theta: Cx, Cy scale as 1/M^2 at fixed U, and (Cl, Cd)
// turns with alpha, so dJ/dM = -2 Jb.C/M and dJ/dalpha = -Jb_l Cd + Jb_d Cl.
__global__ void __launch_bounds__(kBlock) k_force_rev(Geo G, Flow P,
                                                      const int32_t *__restrict__ woff,
                                                      const int32_t *__restrict__ wall,
                                                      const double *__restrict__ mach,
                                                      const double *__restrict__ aoa,
                                                      const double *__restrict__ U,
                                                      const double *__restrict__ Jb,
                                                      double *__restrict__ Ubar,
                                                      double *__restrict__ thetabar) {
  __shared__ double lds[kBlock];
  const int c = blockIdx.x;
  const int w0 = woff[c], nw = woff[c + 1] - woff[c];
  const double g = P.gamma, pinf = 1.0 / g;
  const double M = mach[c], qinf = 0.5 * M * M;
  const double ca = cos(aoa[c]), sa = sin(aoa[c]);
  double fx = 0.0, fy = 0.0;
  for (int e = threadIdx.x; e < nw; e += kBlock) {
    const int a = wall[w0 + e], b = wall[w0 + (e + 1) % nw];
    double ra, ua, va, pa, rb, ub, vb, pb;
    prim_from_cons(g, ld4(U, a), ra, ua, va, pa);
    prim_from_cons(g, ld4(U, b), rb, ub, vb, pb);
    const double cp = (0.5 * (pa + pb) - pinf) / qinf;
    const double2 xa = G.xy[a], xb = G.xy[b];
    fx += -cp * (xb.y - xa.y);
    fy += cp * (xb.x - xa.x);
  }
  const double Cx = block_sum(fx, lds);
  __syncthreads();
  const double Cy = block_sum(fy, lds);
  const double jl = Jb[2 * c], jd = Jb[2 * c + 1];
  const double cxb = -jl * sa + jd * ca, cyb = jl * ca + jd * sa;
  for (int e = threadIdx.x; e < nw; e += kBlock) {
    const int a = wall[w0 + e];
    const int prev = wall[w0 + (e + nw - 1) % nw], next = wall[w0 + (e + 1) % nw];
    const double2 xp = G.xy[prev], xa = G.xy[a], xn = G.xy[next];
    // edges (prev, a) and (a, next)
    const double cpb1 = -cxb * (xa.y - xp.y) + cyb * (xa.x - xp.x);
    const double cpb2 = -cxb * (xn.y - xa.y) + cyb * (xn.x - xa.x);
    const double p_b = 0.5 * (cpb1 + cpb2) / qinf;
    double rho, u, v, p;
    prim_from_cons(g, ld4(U, a), rho, u, v, p);
    const double gm1 = g - 1.0;
    st4(Ubar, a, F4{{p_b * gm1 * 0.5 * (u * u + v * v), -p_b * gm1 * u, -p_b * gm1 * v,
                     p_b * gm1}});
  }
  if (threadIdx.x == 0) {
    const double Cl = Cy * ca - Cx * sa, Cd = Cx * ca + Cy * sa;
    thetabar[2 * c] = -2.0 * (jl * Cl + jd * Cd) / M;
    thetabar[2 * c + 1] = -jl * Cd + jd * Cl;
  }
}

// ---------------------------------------------------------------------------
// host side

size_t f1_bytes(const lskum_plan_s *p) { return align256((size_t)p->n * sizeof(double)); }

int n_levels(const lskum_plan_s *p) { return p->params[0].n_inner + 1; }

// workspace layout, in units of one double per point (f1)
struct VjpWs {
  double *q, *dq0, *qlim, *qbar, *sa, *sb, *lbar;
  int8_t *argext;
};

VjpWs vjp_layout(const lskum_plan_s *p, void *ws) {
  const size_t f1 = f1_bytes(p);
  char *b = static_cast<char *>(ws);
  VjpWs w;
  size_t o = 0;
  w.q = reinterpret_cast<double *>(b + o);
  o += 4 * f1;
  w.dq0 = reinterpret_cast<double *>(b + o);
  o += 8 * f1 * (size_t)n_levels(p);
  w.qlim = reinterpret_cast<double *>(b + o);
  o += 8 * f1;
  w.qbar = reinterpret_cast<double *>(b + o);
  o += 4 * f1;
  w.sa = reinterpret_cast<double *>(b + o);
  o += 8 * f1;
  w.sb = reinterpret_cast<double *>(b + o);
  o += 8 * f1;
  w.lbar = reinterpret_cast<double *>(b + o);
  o += 8 * f1;
  w.argext = reinterpret_cast<int8_t *>(b + o);
  return w;
}

size_t vjp_bytes(const lskum_plan_s *p) {
  const size_t f1 = f1_bytes(p);
  const size_t fields = 4 + 8 * (size_t)n_levels(p) + 8 + 4 + 8 + 8 + 8 + 1;
  return fields * f1;
}

template <class T>
int download(std::vector<T> &dst, const T *src, size_t count) {
  dst.resize(count);
  if (count && hipMemcpy(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess)
    return LSKUM_ERR_HIP;
  return LSKUM_OK;
}

// Transposed connectivity, least-squares geometry and outer lists.
// Synchronous.
int adjoint_prepare(lskum_plan_s *p, void *stream) {
  if (p->adj_ready) return LSKUM_OK;
  if (p->n > kPointMask || p->k_pad > 64 || p->k_in < 1 ||
      (int64_t)p->k_in * p->n > (int64_t)INT32_MAX)
    return LSKUM_ERR_INVALID_ARG;
  if (hipStreamSynchronize(S(stream)) != hipSuccess) return LSKUM_ERR_HIP;
  const int32_t n = p->n, kp = p->k_pad, ki = p->k_in;
  std::vector<int32_t> nbr, cnt;
  std::vector<int8_t> kind;
  std::vector<int32_t> in_cnt, in_ent, outer, ooff;
  int rc = LSKUM_OK;
  try {
    if ((rc = download(nbr, p->nbr, (size_t)n * kp)) || (rc = download(cnt, p->cnt, (size_t)n)) ||
        (rc = download(kind, p->kind, (size_t)n)))
      return rc;
    in_cnt.assign((size_t)n, 0);
    in_ent.resize((size_t)ki * n);
    for (int32_t j = 0; j < n; ++j) in_ent[(size_t)j] = j;  // a point with no in-edge
    for (int32_t i = 0; i < n; ++i)  // i ascending, then slot: rows sorted
      for (int32_t s = 0; s < cnt[(size_t)i]; ++s) {
        const int32_t j = nbr[(size_t)s * n + i];
        const int32_t e = in_cnt[(size_t)j]++;
        if (e >= ki) return LSKUM_ERR_BAD_CLOUD;  // k_in is the largest in-degree
        in_ent[(size_t)e * n + j] = (s << kSlotShift) | i;
      }
    ooff.push_back(0);
    for (int32_t c = 0; c < p->n_clouds; ++c) {
      for (int32_t i = p->offset[(size_t)c]; i < p->offset[(size_t)c + 1]; ++i)
        if (kind[(size_t)i] == 2) outer.push_back(i);
      ooff.push_back((int32_t)outer.size());
    }
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  if ((rc = upload(&p->in_cnt, in_cnt.data(), in_cnt.size())) ||
      (rc = upload(&p->in_ent, in_ent.data(), in_ent.size())) ||
      (rc = upload(&p->outer, outer.data(), outer.size())) ||
      (rc = upload(&p->ooff, ooff.data(), ooff.size())))
    return rc;
  if (hipMalloc((void **)&p->lsg, (size_t)n * 8 * sizeof(double)) != hipSuccess)
    return LSKUM_ERR_NO_MEMORY;
  k_ls_geometry<<<grid_for(n), kBlock, 0, S(stream)>>>(geo(p), p->lsg);
  if ((rc = launched())) return rc;
  if (hipStreamSynchronize(S(stream)) != hipSuccess) return LSKUM_ERR_HIP;
  p->adj_ready = true;
  return LSKUM_OK;
}

// free whatever a failed preparation left
void adjoint_reset(lskum_plan_s *p) {
  void *bufs[] = {p->in_cnt, p->in_ent, p->lsg, p->outer, p->ooff,
                  p->in_map.tlo, p->in_map.lent, p->in_map.hoff, p->in_map.hids};
  for (void *b : bufs) (void)hipFree(b);
  p->in_cnt = p->in_ent = p->outer = p->ooff = nullptr;
  p->lsg = nullptr;
  p->in_map = InTileMap{};
  p->adj_ready = false;
}

// Tile tables of the in-edge rows for the plan's tile size (synchronous;
// rebuilt when the tile size changes).
// Points per tile of the in-edge tables: the plan's tile size, at most 256
// (the transposed gathers measured slower on 512-point tiles).
inline int in_tile_size(const lskum_plan_s *p) { return std::min(p->block, 256); }

int ensure_in_tiles(lskum_plan_s *p, void *stream) {
  InTileMap &m = p->in_map;
  if (m.blk == p->block) return LSKUM_OK;
  // earlier VJP calls on this stream may still read the old tables
  if (hipStreamSynchronize(S(stream)) != hipSuccess) return LSKUM_ERR_HIP;
  (void)hipFree(m.tlo);
  (void)hipFree(m.lent);
  (void)hipFree(m.hoff);
  (void)hipFree(m.hids);
  m = InTileMap{};
  const int32_t n = p->n, ki = p->k_in;
  std::vector<int32_t> ent, cnt, ids, slots, tlo, hoff, hids;
  std::vector<uint32_t> lent;
  int hmax = 0, rc;
  if ((rc = download(ent, p->in_ent, (size_t)ki * n)) || (rc = download(cnt, p->in_cnt, (size_t)n)))
    return rc;
  try {
    ids.resize(ent.size());
    for (size_t e = 0; e < ent.size(); ++e) ids[e] = ent[e] & kPointMask;
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  // Tiles capped at 2 tile table slots as for the forward passes' tables
  // and at what the first-order reverse's 88-byte slots fit in the LDS
  // budget; fixed tiles where capping would shrink them a lot.
  const int tile = in_tile_size(p);
  const int cap = std::min(2 * tile, (int)(kTileLdsBytes / 88) / 4 * 4);
  rc = tile_slots(n, ki, tile, cap, ids.data(), cnt.data(), slots, tlo, hoff, hids, hmax);
  const int64_t fixed_tiles = ((int64_t)n + tile - 1) / tile;
  if (!rc && (int64_t)tlo.size() - 1 > fixed_tiles + fixed_tiles / 8 + 8)
    rc = tile_slots(n, ki, tile, 0, ids.data(), cnt.data(), slots, tlo, hoff, hids, hmax);
  if (rc) return rc;
  try {
    lent.resize(slots.size());
    for (int32_t e = 0; e < ki; ++e)
      for (int32_t j = 0; j < n; ++j) {
        const size_t x = (size_t)e * n + j;
        const uint32_t row_slot = e < cnt[(size_t)j] ? (uint32_t)(ent[x] >> kSlotShift) : 0u;
        lent[x] = (uint32_t)slots[x] | (row_slot << 16);
      }
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  if ((rc = upload(&m.lent, lent.data(), lent.size())) ||
      (rc = upload(&m.tlo, tlo.data(), tlo.size())) ||
      (rc = upload(&m.hoff, hoff.data(), hoff.size())) ||
      (rc = upload(&m.hids, hids.data(), hids.size())))
    return rc;
  m.hmax = (hmax + 3) / 4 * 4;
  m.ntiles = (int)tlo.size() - 1;
  m.blk = p->block;
  return LSKUM_OK;
}

#define LSKUM_TILED_ADJ(kern, p, stream, ...)                                                \
  do {                                                                                       \
    const int g_ = grid_for((p)->n, (p)->block);                                             \
    switch ((p)->block) {                                                                    \
      case 128: kern<128><<<g_, 128, 0, S(stream)>>>(__VA_ARGS__); break;                    \
      case 512: kern<512><<<g_, 512, 0, S(stream)>>>(__VA_ARGS__); break;                    \
      default: kern<256><<<g_, 256, 0, S(stream)>>>(__VA_ARGS__); break;                     \
    }                                                                                        \
  } while (0)

int prepare_checked(lskum_plan_s *p, void *stream) {
  if (p->params[0].options & (LSKUM_FIRST_ORDER | LSKUM_MINMAX))  // the default residual only
    return LSKUM_ERR_INVALID_ARG;
  int rc = adjoint_prepare(p, stream);
  if (!rc) rc = ensure_in_tiles(p, stream);
  if (rc) adjoint_reset(p);
  return rc;
}

// q, the first-order derivatives with the slots attaining the bounds, and
// every inner iterate of U, into the workspace.
int forward_recompute(lskum_plan_s *p, const VjpWs &w, const double *U, void *stream) {
  const int K = p->params[0].n_inner;
  const size_t lev = 8 * f1_bytes(p) / sizeof(double);  // doubles between iterates
  int rc;
  if ((rc = q_vars_launch(p, U, w.q, stream))) return rc;
  if ((rc = deriv_first_launch(p, w.q, w.dq0, w.qlim, w.argext, stream))) return rc;
  for (int k = 1; k <= K; ++k)
    if ((rc = deriv_inner_launch(p, w.dq0, w.dq0 + (k - 1) * lev, w.dq0 + k * lev, stream)))
      return rc;
  return LSKUM_OK;
}

// Reverse passes from the residual cotangent Rbar to Ubar (every row,
// outer rows included): flux, its transposed gather, inner sweeps K..1,
// first-order pass and q-variables.
int reverse_passes(lskum_plan_s *p, const VjpWs &w, const double *U, const double *Rbar,
                   double *Ubar, void *stream) {
  const int K = p->params[0].n_inner;
  const size_t lev = 8 * f1_bytes(p) / sizeof(double);
  const double *dqK = w.dq0 + (size_t)K * lev;
  const Geo g = geo(p);
  const Flow f = flow(p);
  {
    // the two flux reverses have no tile tables: one-wavefront blocks
    // shorten their launch tails, as for the forward flux
    const int g64 = grid_for(p->n, 64);
    if (f.gamma_is_14) {
      k_flux_rev_own<64, true><<<g64, 64, 0, S(stream)>>>(g, f, p->spw, w.q, dqK, w.qlim, Rbar,
                                                          w.qbar, w.sa, w.lbar, p->status);
      k_flux_gather<64, true><<<g64, 64, 0, S(stream)>>>(g, f, p->in_cnt, p->in_ent, p->lsg,
                                                         p->spw, w.q, dqK, w.qlim, Rbar, w.qbar,
                                                         w.sa, w.lbar);
    } else {
      k_flux_rev_own<64, false><<<g64, 64, 0, S(stream)>>>(g, f, p->spw, w.q, dqK, w.qlim, Rbar,
                                                           w.qbar, w.sa, w.lbar, p->status);
      k_flux_gather<64, false><<<g64, 64, 0, S(stream)>>>(g, f, p->in_cnt, p->in_ent, p->lsg,
                                                          p->spw, w.q, dqK, w.qlim, Rbar, w.qbar,
                                                          w.sa, w.lbar);
    }
  }
  // the derivative reverses on the in-edge tile tables when a block's
  // table fits the LDS budget
  const InTileMap &m = p->in_map;
  const Tiles t{nullptr, m.hoff, m.hids, m.hmax, 0, m.tlo, m.ntiles};
  const int tile = in_tile_size(p);
  const size_t cap = (size_t)tile + m.hmax;
  const bool tiled = m.blk == p->block && cap * 88 <= kTileLdsBytes;
  const bool k48 = p->k_in <= 48;
  const int gr = grid_tiles(m.ntiles);
  hipStream_t st = S(stream);
#define LSKUM_REV_T(kern, lds, ...)                                                      \
  do {                                                                                   \
    switch (tile) {  /* 128 or 256 */                                                    \
      case 128:                                                                          \
        if (k48) kern<128, 48><<<gr, 128, lds, st>>>(__VA_ARGS__);                       \
        else kern<128, 0><<<gr, 128, lds, st>>>(__VA_ARGS__);                            \
        break;                                                                           \
      default:                                                                           \
        if (k48) kern<256, 48><<<gr, 256, lds, st>>>(__VA_ARGS__);                       \
        else kern<256, 0><<<gr, 256, lds, st>>>(__VA_ARGS__);                            \
        break;                                                                           \
    }                                                                                    \
  } while (0)
  double *cur = w.sa, *nxt = w.sb;
  for (int k = K; k >= 1; --k) {
    if (tiled)
      LSKUM_REV_T(k_inner_rev_t, cap * 80, g, t, m.lent, p->k_in, p->in_cnt, p->lsg, cur,
                  w.qbar, nxt);
    else
      LSKUM_TILED_ADJ(k_inner_rev, p, stream, g, p->in_cnt, p->in_ent, p->lsg, cur, w.qbar, nxt);
    double *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (tiled)
    LSKUM_REV_T(k_first_rev_t, cap * 88, g, f, t, m.lent, p->k_in, p->in_cnt, p->lsg, cur,
                w.argext, w.lbar, U, w.qbar, Ubar);
  else
    LSKUM_TILED_ADJ(k_first_rev, p, stream, g, f, p->in_cnt, p->in_ent, p->lsg, cur, w.argext,
                    w.lbar, U, w.qbar, Ubar);
#undef LSKUM_REV_T
  return launched();
}

}  // namespace
}  // namespace lskum_impl

using namespace lskum_impl;

extern "C" {

size_t lskum_vjp_workspace_bytes(lskum_plan p) {
  if (!p) return 0;
  return vjp_bytes(p);
}

int lskum_flux_residual_vjp(lskum_plan p, const double *U, const double *Rbar, double *Ubar,
                            double *thetabar, void *ws, void *stream) {
  if (!p || !a32(U) || !a32(Rbar) || !a32(Ubar) || !thetabar || !ws ||
      ((uintptr_t)ws % 256) != 0)
    return LSKUM_ERR_INVALID_ARG;
  int rc = prepare_checked(p, stream);
  if (rc) return rc;
  const VjpWs w = vjp_layout(p, ws);
  if ((rc = forward_recompute(p, w, U, stream))) return rc;
  if ((rc = reverse_passes(p, w, U, Rbar, Ubar, stream))) return rc;
  k_theta_rev<<<p->n_clouds, kBlock, 0, S(stream)>>>(p->ooff, p->outer, p->mach, p->aoa, Ubar,
                                                     thetabar);
  return launched();
}

// The steady adjoint's workspace: the VJP's, then dt [n], Ubar [n][4] and
// two [n_clouds][2] theta cotangents.
size_t lskum_adjoint_workspace_bytes(lskum_plan p) {
  if (!p) return 0;
  return vjp_bytes(p) + 5 * f1_bytes(p) + align256(4 * (size_t)p->n_clouds * sizeof(double));
}

int lskum_adjoint_iterate(lskum_plan p, const double *U, const double *g, double *Lambda,
                          int32_t iters, double *hist, void *ws, void *stream) {
  if (!p || !a32(U) || !a32(g) || !a32(Lambda) || iters < 0 || !ws ||
      ((uintptr_t)ws % 256) != 0)
    return LSKUM_ERR_INVALID_ARG;
  int rc = prepare_checked(p, stream);
  if (rc) return rc;
  const VjpWs w = vjp_layout(p, ws);
  char *extra = static_cast<char *>(ws) + vjp_bytes(p);
  double *dt = reinterpret_cast<double *>(extra);
  double *Ub = reinterpret_cast<double *>(extra + f1_bytes(p));
  if ((rc = lskum_local_dt(p, U, dt, stream))) return rc;
  if ((rc = forward_recompute(p, w, U, stream))) return rc;
  const Geo geo_ = geo(p);
  for (int32_t k = 0; k < iters; ++k) {
    if ((rc = reverse_passes(p, w, U, Lambda, Ub, stream))) return rc;
    k_adjoint_step<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo_, dt, g, Ub, Lambda);
    if (hist && (rc = lskum_residual_norm(p, Ub, hist + (size_t)k * p->n_clouds, stream)))
      return rc;
  }
  return launched();
}

int lskum_adjoint_total(lskum_plan p, const double *U, const double *Lambda, const double *Jbar,
                        double *total, double *partial, void *ws, void *stream) {
  if (!p || !a32(U) || !a32(Lambda) || !Jbar || !total || !ws || ((uintptr_t)ws % 256) != 0)
    return LSKUM_ERR_INVALID_ARG;
  const size_t nc2 = 2 * (size_t)p->n_clouds * sizeof(double);
  if (!writes_disjoint({Span{total, nc2}, Span{partial, partial ? nc2 : 0}},
                       {Span{U, 32 * (size_t)p->n}, Span{Lambda, 32 * (size_t)p->n},
                        Span{Jbar, nc2}, Span{ws, lskum_adjoint_workspace_bytes(p)}}))
    return LSKUM_ERR_INVALID_ARG;
  char *extra = static_cast<char *>(ws) + vjp_bytes(p);
  double *Ub = reinterpret_cast<double *>(extra + f1_bytes(p));
  double *part = reinterpret_cast<double *>(extra + 5 * f1_bytes(p));
  double *tr = part + 2 * (size_t)p->n_clouds;
  int rc;
  // the partial at fixed U (its U cotangent, written to Ub, is not needed)
  if ((rc = lskum_force_coeffs_vjp(p, U, Jbar, Ub, part, stream))) return rc;
  // theta cotangent of the residual with Rbar = Lambda
  if ((rc = lskum_flux_residual_vjp(p, U, Lambda, Ub, tr, ws, stream))) return rc;
  const int count = 2 * p->n_clouds;
  k_adjoint_total<<<(count + 63) / 64, 64, 0, S(stream)>>>(count, part, tr, total, partial);
  return launched();
}

int lskum_force_coeffs_vjp(lskum_plan p, const double *U, const double *Jbar, double *Ubar,
                           double *thetabar, void *stream) {
  if (!p || !a32(U) || !Jbar || !a32(Ubar) || !thetabar) return LSKUM_ERR_INVALID_ARG;
  const size_t count = 4 * (size_t)p->n;
  k_zero<<<grid_for((int)std::min<size_t>(count, (size_t)1 << 24)), kBlock, 0, S(stream)>>>(count,
                                                                                          Ubar);
  k_force_rev<<<p->n_clouds, kBlock, 0, S(stream)>>>(geo(p), flow(p), p->woff, p->wall, p->mach,
                                                     p->aoa, U, Jbar, Ubar, thetabar);
  return launched();
}

}  // extern "C"
