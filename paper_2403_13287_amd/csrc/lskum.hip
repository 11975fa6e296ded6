// lskum.hip -- gfx950 plans, small kernels (q-variables, stage updates,
// reductions) and the C ABI of the LSKUM residual sweep; the flux kernel is
// in lskum_flux.hip, the derivative and time-step gathers in lskum_deriv.hip.
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
#include <mutex>
#include <new>
#include <vector>

#include "lskum.h"
#include "lskum_impl.h"

namespace lskum_impl {

__global__ void __launch_bounds__(kBlock) k_q_vars(int n, int xcd, Flow P,
                                                   const double *__restrict__ U,
                                                   double *__restrict__ q, unsigned *status) {
  const int i = point_index<kBlock>(xcd);
  if (i >= n) return;
  F4 o;
  const unsigned f = q_of_state(P, ld4(U, i), o);
  st4(q, i, o);
  flag(status, f);
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

// ---------------------------------------------------------------------------
// local time step, Runge-Kutta stage, initial state

__global__ void __launch_bounds__(kBlock) k_rk_stage(Geo G, Flow P, int stage,
                                                     double *__restrict__ Un,
                                                     const double *__restrict__ R,
                                                     const double *__restrict__ dt,
                                                     double *__restrict__ U) {
  const int n = G.n;
  const int i = point_index<kBlock>(G.xcd);
  if (i >= n) return;
  const int kind = G.kind[i];
  const F4 Uc = ld4(U, i);
  if (stage == 0) st4(Un, i, Uc);  // the step's U^n, for the third stage
  const F4 Ui = kind == 2 ? ld4(G.uinf, G.cloud[i])
                          : ssp_stage(G, i, kind, stage, Un, Uc, ld4(R, i), dt[i]);
  st4(U, i, Ui);
}

// Classical RK4 stage with L = -R: the stage inputs are Un - dt/2 R0,
// Un - dt/2 R1, Un - dt R2 and the step ends at Un - dt/6 (R0 + 2 R1 + 2 R2 + R3).
// acc carries the partial weighted sum of the stage residuals.
__global__ void __launch_bounds__(kBlock) k_rk4_stage(Geo G, Flow P, int stage,
                                                      double *__restrict__ Un,
                                                      const double *__restrict__ R,
                                                      const double *__restrict__ dt,
                                                      double *__restrict__ acc,
                                                      double *__restrict__ U) {
  const int n = G.n;
  const int i = point_index<kBlock>(G.xcd);
  if (i >= n) return;
  const int kind = G.kind[i];
  // stage 0: the incoming U is the step's U^n, which the later stages read
  const F4 U0 = stage == 0 ? ld4(U, i) : ld4(Un, i);
  if (stage == 0) st4(Un, i, U0);
  F4 Ui;
  if (kind == 2) {
    Ui = ld4(G.uinf, G.cloud[i]);
  } else {
    const F4 Ri = ld4(R, i);
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
// in a fixed order and writes its norm to out[row * row_stride + c * cloud_stride],
// where row is *counter when a counter is given (graph replays append rows;
// rows past `capacity` are not written), else 0.
__global__ void __launch_bounds__(kBlock) k_norm_final(const int32_t *__restrict__ first,
                                                       const double *__restrict__ partial,
                                                       size_t row_stride, size_t cloud_stride,
                                                       const int32_t *counter, int capacity,
                                                       double *__restrict__ out) {
  __shared__ double lds[kBlock];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int k = first[c] + (int)threadIdx.x; k < first[c + 1]; k += kBlock) s += partial[k];
  const double t = block_sum(s, lds);
  if (threadIdx.x == 0) {
    const int row = counter ? *counter : 0;
    if (row < capacity) out[(size_t)row * row_stride + (size_t)c * cloud_stride] = sqrt(t);
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

int tile_slots(int32_t n, int32_t width, int blk, int cap, const int32_t *ids,
               const int32_t *cnt, std::vector<int32_t> &slots, std::vector<int32_t> &tlo,
               std::vector<int32_t> &hoff, std::vector<int32_t> &hids, int &hmax) {
  std::vector<int32_t> ext;
  // the out-of-tile points named by the rows of points lo .. hi-1, ascending
  auto halo = [&](int32_t lo, int32_t hi) {
    ext.clear();
    for (int32_t i = lo; i < hi; ++i)
      for (int32_t s = 0; s < cnt[i]; ++s) {
        const int32_t j = ids[(size_t)s * n + i];
        if (j < lo || j >= hi) ext.push_back(j);
      }
    std::sort(ext.begin(), ext.end());
    ext.erase(std::unique(ext.begin(), ext.end()), ext.end());
  };
  hmax = 0;
  try {
    slots.resize((size_t)width * n);
    tlo.assign(1, 0);
    hoff.assign(1, 0);
    hids.clear();
    hids.reserve((size_t)n);
    for (int32_t lo = 0; lo < n;) {
      int32_t size = std::min<int32_t>(blk, n - lo);
      halo(lo, lo + size);
      if (cap > 0)
        while (size > 1 && size + (int64_t)ext.size() > cap) {
          size = size > 8 ? size - 8 : size - 1;
          halo(lo, lo + size);
        }
      const int32_t hi = lo + size, base = size;
      if ((int64_t)base + (int64_t)ext.size() > 65535) return LSKUM_ERR_INVALID_ARG;
      hmax = std::max(hmax, base + (int)ext.size() - blk);
      hoff.push_back(hoff.back() + (int32_t)ext.size());
      hids.insert(hids.end(), ext.begin(), ext.end());
      tlo.push_back(hi);
      for (int32_t i = lo; i < hi; ++i)
        for (int32_t s = 0; s < width; ++s) {
          const int32_t j = s < cnt[i] ? ids[(size_t)s * n + i] : i;
          slots[(size_t)s * n + i] =
              (j >= lo && j < hi)
                  ? j - lo
                  : base + (int32_t)(std::lower_bound(ext.begin(), ext.end(), j) - ext.begin());
        }
      lo = hi;
    }
    // a spare entry (point 0) after the last tile's halo: readers clamp
    // their indices into a tile's list, which then stays in bounds when the
    // list is empty
    hids.push_back(0);
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
  std::vector<int32_t> slots, tlo, hoff, hids;
  std::vector<uint16_t> lcol;
  int hmax = 0;
  // Tiles capped at 2 blk table slots: the inner sweep's table (80 B a
  // slot) then takes 40 KB at blk = 256, four blocks to a CU's 160 KB where
  // the largest halo of fixed tiles would allow three.  Where capping
  // shrinks the tiles a lot (clouds not ordered along a space-filling
  // curve), fixed tiles instead: their tables exceed the LDS budget and the
  // direct-gather kernels run.
  int rc = tile_slots(p->n, p->k_pad, blk, 2 * blk, nbr, cnt, slots, tlo, hoff, hids, hmax);
  const int64_t fixed_tiles = ((int64_t)p->n + blk - 1) / blk;
  if (!rc && (int64_t)tlo.size() - 1 > fixed_tiles + fixed_tiles / 8 + 8)
    rc = tile_slots(p->n, p->k_pad, blk, 0, nbr, cnt, slots, tlo, hoff, hids, hmax);
  if (rc) return rc;
  // slots grouped by 8 entries of a row: [groups][n][8], 16 bytes per point
  // and group (entries past k_pad: slot 0, never read)
  const int groups = (p->k_pad + 7) / 8;
  const size_t n = (size_t)p->n;
  try {
    lcol.assign((size_t)groups * n * 8, 0);
    for (int32_t s = 0; s < p->k_pad; ++s)
      for (size_t i = 0; i < n; ++i)
        lcol[((size_t)(s >> 3) * n + i) * 8 + (s & 7)] = (uint16_t)slots[s * n + i];
  } catch (const std::bad_alloc &) {
    return LSKUM_ERR_NO_MEMORY;
  }
  if ((rc = upload(&m.lcol, lcol.data(), lcol.size())) ||
      (rc = upload(&m.tlo, tlo.data(), tlo.size())) ||
      (rc = upload(&m.hoff, hoff.data(), hoff.size())) ||
      (rc = upload(&m.hids, hids.data(), hids.size())))
    return rc;
  m.hmax = (hmax + 3) / 4 * 4;
  m.groups = groups;
  m.ntiles = (int)tlo.size() - 1;
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
  k_q_vars<<<grid_for(p->n), kBlock, 0, S(stream)>>>(p->n, p->xcd, f, U, q, p->status);
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
                (t->xcd_contiguous == 0 || t->xcd_contiguous == 1) &&
                (t->flux_block == 0 || t->flux_block == 64 || t->flux_block == 128 ||
                 t->flux_block == 256));
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
    (void)hipFree(m.tlo);
    (void)hipFree(m.lcol);
    (void)hipFree(m.hoff);
    (void)hipFree(m.hids);
  }
  // the adjoint's in-edge tile tables (built by the first VJP call)
  (void)hipFree(p->in_map.tlo);
  (void)hipFree(p->in_map.lent);
  (void)hipFree(p->in_map.hoff);
  (void)hipFree(p->in_map.hids);
  (void)hipSetDevice(cur);
  delete p;
}

constexpr size_t kNumWorkFields = 4 + 4 + 8 + 8 + 16 + 4 + 1 + 4 + 4;  // Un q dq qlim work R dt acc q2

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

// Layout of a residual-norm history: entry (row, cloud) at
// row * row_stride + cloud * cloud_stride.
struct HistLayout {
  size_t row_stride, cloud_stride;
};

int norm_launch(lskum_plan_s *p, const double *R, double *out, const int32_t *counter,
                int capacity, void *stream, HistLayout lay) {
  k_norm_partial<<<p->n_chunks, kBlock, 0, S(stream)>>>(p->chunks, p->kind, R, p->partial);
  k_norm_final<<<p->n_clouds, kBlock, 0, S(stream)>>>(p->chunk_first, p->partial, lay.row_stride,
                                                      lay.cloud_stride, counter, capacity, out);
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

// The iteration body shared by lskum_iterate, lskum_batch_run and graph
// capture.  With a counter, norms go to row *counter of hist and the counter
// advances after each iteration (graph replays); without one, iteration k
// writes row k.
int run_iterations(lskum_plan_s *p, int32_t iters, double *U, double *hist, int32_t hist_rows,
                   void *ws, int32_t *counter, void *stream, HistLayout lay) {
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
  double *q2 = reinterpret_cast<double *>(base + 49 * f1);
  const bool rk4 = (p->params[0].options & LSKUM_RK4) != 0;
  const Geo g = geo(p);
  const Flow f = flow(p);
  const int grid = grid_for(p->n);
  int rc;
  for (int32_t it = 0; it < iters; ++it) {
    // (the first stage's launch stores U, the step's U^n, in Un)
    if ((rc = local_dt_launch(p, U, dt, stream))) return rc;
    for (int s = 0; s < 4; ++s) {
      // SSP stages run fused into the flux launch, which also writes the
      // next stage's q (ping-pong buffers); q_vars only starts the sequence
      if ((rk4 || (it == 0 && s == 0)) && (rc = q_vars_launch(p, U, q, stream))) return rc;
      // the first-order flux reads no derivatives
      if (flux_variant(p) != 1 && (rc = q_derivs_launch(p, q, dq, qlim, work, stream))) return rc;
      const StageArgs sa{s, Un, dt, U, q2};
      if ((rc = flux_launch(p, q, dq, qlim, R, stream, rk4 ? nullptr : &sa))) return rc;
      if (s == 0) {
        const HistLayout scratch{0, 1};
        if (counter)
          rc = norm_launch(p, R, hist ? hist : p->norm_scratch, counter, hist ? hist_rows : 1,
                           stream, hist ? lay : scratch);
        else
          rc = norm_launch(p, R, hist ? hist + (size_t)it * lay.row_stride : p->norm_scratch,
                           nullptr, 1, stream, hist ? lay : scratch);
        if (rc) return rc;
      }
      if (rk4) {
        k_rk4_stage<<<grid, kBlock, 0, S(stream)>>>(g, f, s, Un, R, dt, acc, U);
      } else {
        double *t = q;
        q = q2;
        q2 = t;
      }
    }
    if (counter) k_tick<<<1, 64, 0, S(stream)>>>(counter);
  }
  return launched();
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of lskum_q_derivs_static, the entry point for callers that
// cannot allocate: the [n][16] work buffer of the inner sweeps for up to
// kScratchPoints points (128 MiB).  Every GPU the library runs on holds its
// own copy until the process ends.  Host code never passes `scratch` itself
// (in host code the name stands for a host-side shadow); it passes the
// device address resolved once per device below.
namespace {

constexpr size_t kScratchPoints = (size_t)1 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[16 * kScratchPoints];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
int g_scratch_rc[kMaxDevices];  // 0: not resolved yet; LSKUM_OK or LSKUM_ERR_HIP once tried

// Resolve the device address of `scratch` on `device`, which must be the
// current device: once per device (plan creation calls it), later calls read
// the stored result.
int resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return LSKUM_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_rc[device] == 0) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_rc[device] = (e == hipSuccess && ptr) ? LSKUM_OK : LSKUM_ERR_HIP;
    if (e != hipSuccess) (void)hipGetLastError();  // do not leave the error for the next call
    g_scratch_ptr[device] = g_scratch_rc[device] == LSKUM_OK ? ptr : nullptr;
  }
  return g_scratch_rc[device];
}

// The stored device address of `scratch` on `device` (nullptr if its
// resolution failed).
void *scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_rc[device] == LSKUM_OK ? g_scratch_ptr[device] : nullptr;
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
    case LSKUM_ERR_SCRATCH_LIMIT:
      return "the cloud exceeds the static scratch of lskum_q_derivs_static (1048576 points)";
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
    p->block = tuning->block ? tuning->block : 512;
    p->xcd = tuning->xcd_contiguous;
    p->flux_block = tuning->flux_block ? tuning->flux_block : 64;
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
  // the static scratch's address on this device, for lskum_q_derivs_static;
  // a failure here is reported by that entry point, not by plan creation
  (void)resolve_scratch(p->device);
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
  p->block = tuning->block ? tuning->block : 512;
  p->xcd = tuning->xcd_contiguous;
  p->flux_block = tuning->flux_block ? tuning->flux_block : 64;
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
  const bool inner = p && p->params[0].n_inner > 0;
  if (!p || !a32(q) || !a64(dq) || !a64(qlim) || (inner && !a64(work)))
    return LSKUM_ERR_INVALID_ARG;
  const size_t n = (size_t)p->n;
  // neighbours read q and the previous iterate while dq, qlim and work are written
  if (!writes_disjoint({Span{dq, 64 * n}, Span{qlim, 64 * n}, Span{work, inner ? 128 * n : 0}},
                       {Span{q, 32 * n}}))
    return LSKUM_ERR_INVALID_ARG;
  return q_derivs_launch(p, q, dq, qlim, work, stream);
}

int lskum_q_derivs_static(lskum_plan p, const double *q, double *dq, double *qlim,
                          void *stream) {
  if (!p || !a32(q) || !a64(dq) || !a64(qlim)) return LSKUM_ERR_INVALID_ARG;
  const size_t n = (size_t)p->n;
  if (!writes_disjoint({Span{dq, 64 * n}, Span{qlim, 64 * n}}, {Span{q, 32 * n}}))
    return LSKUM_ERR_INVALID_ARG;
  double *work = nullptr;
  if (p->params[0].n_inner > 0) {
    if (n > kScratchPoints) return LSKUM_ERR_SCRATCH_LIMIT;
    work = static_cast<double *>(scratch_on(p->device));
    if (!work) return LSKUM_ERR_HIP;
  }
  // the same launches as lskum_q_derivs; every entry of work is written
  // before it is read, so nothing needs clearing between calls
  return q_derivs_launch(p, q, dq, qlim, work, stream);
}

int lskum_flux_residual(lskum_plan p, const double *q, const double *dq, const double *qlim,
                        double *R, void *stream) {
  if (!p || !a32(q) || !a64(dq) || !a64(qlim) || !a32(R)) return LSKUM_ERR_INVALID_ARG;
  const size_t n = (size_t)p->n;
  if (!writes_disjoint({Span{R, 32 * n}}, {Span{q, 32 * n}, Span{dq, 64 * n}, Span{qlim, 64 * n}}))
    return LSKUM_ERR_INVALID_ARG;
  return flux_launch(p, q, dq, qlim, R, stream);
}

int lskum_flux_residual_stage(lskum_plan p, int stage, const double *q, const double *dq,
                              const double *qlim, double *Un, const double *dt, double *R,
                              double *U, double *q_next, void *stream) {
  if (!p || !a32(q) || !a64(dq) || !a64(qlim) || !a32(R) || !a32(Un) || !dt || !a32(U) ||
      !a32(q_next) || stage < 0 || stage > 3)
    return LSKUM_ERR_INVALID_ARG;
  // other points read q, dq and qlim as neighbours while R, U, q_next (and
  // at stage 0 Un) are written; a point stores R before it reads its own U,
  // Un and dt
  const size_t n = (size_t)p->n;
  if (!writes_disjoint({Span{R, 32 * n}, Span{U, 32 * n}, Span{q_next, 32 * n}, Span{Un, 32 * n}},
                       {Span{q, 32 * n}, Span{dq, 64 * n}, Span{qlim, 64 * n}, Span{dt, 8 * n}}))
    return LSKUM_ERR_INVALID_ARG;
  const StageArgs sa{stage, Un, dt, U, q_next};
  return flux_launch(p, q, dq, qlim, R, stream, &sa);
}

int lskum_local_dt(lskum_plan p, const double *U, double *dt, void *stream) {
  if (!p || !a32(U) || !dt) return LSKUM_ERR_INVALID_ARG;
  return local_dt_launch(p, U, dt, stream);
}

int lskum_rk_stage(lskum_plan p, int stage, double *Un, const double *R, const double *dt,
                   double *U, void *stream) {
  if (!p || !a32(Un) || !a32(R) || !dt || !a32(U) || stage < 0 || stage > 3)
    return LSKUM_ERR_INVALID_ARG;
  const size_t n = (size_t)p->n;
  if (!writes_disjoint({Span{U, 32 * n}, Span{Un, 32 * n}}, {Span{R, 32 * n}, Span{dt, 8 * n}}))
    return LSKUM_ERR_INVALID_ARG;
  k_rk_stage<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), flow(p), stage, Un, R, dt, U);
  return launched();
}

int lskum_rk4_stage(lskum_plan p, int stage, double *Un, const double *R, const double *dt,
                    double *acc, double *U, void *stream) {
  if (!p || !a32(Un) || !a32(R) || !dt || !a32(acc) || !a32(U) || stage < 0 || stage > 3)
    return LSKUM_ERR_INVALID_ARG;
  const size_t n = (size_t)p->n;
  if (!writes_disjoint({Span{U, 32 * n}, Span{Un, 32 * n}, Span{acc, 32 * n}},
                       {Span{R, 32 * n}, Span{dt, 8 * n}}))
    return LSKUM_ERR_INVALID_ARG;
  k_rk4_stage<<<grid_for(p->n), kBlock, 0, S(stream)>>>(geo(p), flow(p), stage, Un, R, dt, acc,
                                                        U);
  return launched();
}

int lskum_residual_norm(lskum_plan p, const double *R, double *out, void *stream) {
  if (!p || !a32(R) || !out) return LSKUM_ERR_INVALID_ARG;
  return norm_launch(p, R, out, nullptr, 1, stream, HistLayout{0, 1});
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
  return run_iterations(p, iters, U, hist, iters, ws, nullptr, stream,
                        HistLayout{(size_t)p->n_clouds, 1});
}

int lskum_batch_run(lskum_plan p, int32_t iters, double *U, double *hist, void *ws,
                    void *stream) {
  if (!p || !a32(U) || !ws || iters < 0 || ((uintptr_t)ws % 256) != 0) return LSKUM_ERR_INVALID_ARG;
  if (hist && !writes_disjoint({Span{hist, (size_t)iters * p->n_clouds * sizeof(double)}},
                               {Span{U, (size_t)p->n * 4 * sizeof(double)},
                                Span{ws, lskum_workspace_bytes(p)}}))
    return LSKUM_ERR_INVALID_ARG;
  return run_iterations(p, iters, U, hist, iters, ws, nullptr, stream,
                        HistLayout{1, (size_t)iters});
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
    const int r2 = run_iterations(p, iters, U, hist, hist_rows, ws, p->counter, g->capture,
                                  HistLayout{(size_t)p->n_clouds, 1});
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
