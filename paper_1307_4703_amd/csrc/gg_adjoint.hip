// gfx950 kernels of the discrete adjoint of the compound lattice.
//
// The compound update t -> t+1 is affine in g for a given fluid velocity
// field (the fluid does not feel the compound: the one-way coupling of the
// Results section). With C = sum_j g_j and W_j(u) = w_j (1 + e_j.u/cs2):
//   collision  g*_i = (1 - w) g_i + (w W_i - k w_i) C + w_i R      (Eqs. 2, 8, 9)
//   links      G(z,i) = g*_i(z - e_i)      fluid source
//              G(z,i) = g*_opp(z)          wall or closed valve
//              G(z,i) = -g*_opp(z) + 2 w_i C_in   open inlet
//              G(z,i) = g*_i(z)            open outlet
// The adjoint step takes lam = dL/dG(t+1) and gives dL/dg(t): each node
// gathers lam* = dL/dg* over every use of its post-collision populations
// (a pull over the links), then applies the transposed collision matrix.
// Parameter gradients accumulate on the way: dL/dR per node, dL/dC_in per
// segment, dL/domega_g per work-group.
#include "gg_adjoint.h"
#include "gg_device.h"

namespace gg {

namespace {

struct Ph {
  uint32_t open;
  const GG_CONST double *cin;
};

__device__ __forceinline__ Ph phase_of(CDesc &L, int64_t t) {
  if (L.n_phases == 0) return {0xFFFFFFFFu, L.seg_cin};
  int64_t tau = (t - L.t_origin) % L.period;
  if (tau < 0) tau += L.period;
  int k = 0;
  while (k + 1 < L.n_phases && L.phase_start[k + 1] <= tau) ++k;
  return {L.phase_open[k], L.phase_cin[k]};
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Work-group sum into one value (every thread of the group must call).
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wsum(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < BS / 64; ++k) s += lds[k];
  return s;
}

template <class W>
__device__ __forceinline__ const GG_GLOBAL W *at(const void *base, int64_t plane, int i, uint32_t node) {
  return (const GG_GLOBAL W *)((const GG_GLOBAL char *)((const GG_GLOBAL W *)base + (int64_t)i * plane) +
                               node * (uint32_t)sizeof(W));
}
template <class W>
__device__ __forceinline__ GG_GLOBAL W *atw(void *base, int64_t plane, int i, uint32_t node) {
  return (GG_GLOBAL W *)((GG_GLOBAL char *)((GG_GLOBAL W *)base + (int64_t)i * plane) +
                         node * (uint32_t)sizeof(W));
}

// Deviations df, dg of the current state in natural order (parity from *L.t).
template <class S>
__device__ __forceinline__ void gather_state(CDesc &L, uint32_t node, uint8_t lc, int x, int y,
                                             typename Pop<S>::T *f, typename Pop<S>::T *g) {
  using P = Pop<S>;
  using W = typename P::W;
  const bool odd = (*(const GG_CONST int64_t *)L.t & 1) != 0;
  const int xm = (x == 0 && L.periodic_x) ? L.nx - 1 : x - 1;
  const int xp = (x == L.nx - 1 && L.periodic_x) ? 0 : x + 1;
  const int ym = (y == 0 && L.periodic_y) ? L.ny - 1 : y - 1;
  const int yp = (y == L.ny - 1 && L.periodic_y) ? 0 : y + 1;
  const Planes<W> pl(L);
  // population j of this node: its own slot j, or at an odd step the slot
  // opp(j) of the upstream neighbour x - e_j where that one is fluid
  auto slot = [&](int j, int k) -> const GG_GLOBAL W * {
    if (odd && j > 0 && !((lc >> (OPP[j] - 1)) & 1)) {
      const int xx = EX[OPP[j]] > 0 ? xp : (EX[OPP[j]] < 0 ? xm : x);
      const int yy = EY[OPP[j]] > 0 ? yp : (EY[OPP[j]] < 0 ? ym : y);
      return pl.at(k + OPP[j], (uint32_t)(L.node0 + yy * L.pitch + xx));
    }
    return pl.at(k + j, node);
  };
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = P::ld(slot(i, 0));
#pragma unroll
  for (int i = 0; i < 5; ++i) g[i] = P::ld(slot(i, 9));
}

// Seed: lam(x,i) = weight(x) (C(x) - target(x)) at the final state; the loss
// 1/2 sum weight (C - target)^2 goes into per-work-group partial sums.
template <class S>
__global__ void __launch_bounds__(256)
    k_seed(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles, int n_tiles,
           int tx_shift, const double *__restrict__ weight, const double *__restrict__ target,
           void *__restrict__ lam, double *__restrict__ partial) {
  using T = typename Pop<S>::T;
  __shared__ double lds[4];
  const int tile = blockIdx.x;
  if (tile >= n_tiles) return;
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int x = tl.x0 + (int)(threadIdx.x & ((1 << tx_shift) - 1));
  const int y = tl.y0 + (int)(threadIdx.x >> tx_shift);
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  const uint8_t lc = (x < L.nx && y < L.ny) ? ((const GG_GLOBAL uint8_t *)L.link)[node] : NOT_FLUID;
  double loss = 0.0;
  if (lc != NOT_FLUID) {
    T f[9], g[5];
    gather_state<S>(L, node, lc, x, y, f, g);
    const double C = L.c_shift + ((double)g[0] + (double)g[1] + (double)g[2] + (double)g[3] +
                                  (double)g[4]);
    const int k = y * L.nx + x;
    const double r = weight[k] * (C - target[k]);
    loss = 0.5 * weight[k] * (C - target[k]) * (C - target[k]);
    for (int i = 0; i < 5; ++i) *atw<double>(lam, L.plane, i, node) = r;
  }
  const double s = block_sum<256>(loss, lds);
  if (threadIdx.x == 0) partial[tile] += s;
}

// Sums one lane gathers for the parameter gradients: dL/dR of its node
// (the current adjoint step), dL/domega_g, and dL/dC_in of up to two inlet
// segments.
struct AdjAcc {
  int sa = -1, sb = -1;
  double ma = 0.0, mb = 0.0, dw = 0.0;
  __device__ __forceinline__ void add_cin(int s, double d) {
    if (sa < 0 || sa == s) {
      sa = s;
      ma += d;
    } else {
      sb = s;
      mb += d;
    }
  }
  // dL/dC_in: one atomic per segment and wavefront (every lane must call)
  __device__ __forceinline__ void flush_cin(double *dcin) {
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      const int seg = slot ? sb : sa;
      const double v = slot ? mb : ma;
      unsigned long long pend = __ballot(seg >= 0);
      while (pend) {
        const int lead = __ffsll(pend) - 1;
        const int sg = __shfl(seg, lead);
        const bool mine = seg == sg;
        const double a = wsum(mine ? v : 0.0);
        if ((int)__lane_id() == lead) atomicAdd(dcin + sg, a);
        pend &= ~__ballot(mine);
      }
    }
    sa = sb = -1;
    ma = mb = 0.0;
  }
};

// The adjoint of step t at fluid node (x, y): from lam = dL/dG(t+1) at the
// node (lx) and at its four axis neighbours (ln[j] = lam_j(x + e_j), j =
// 1..4; any value where x + e_j is not fluid), with the taped state (g, u)
// of step t, the node's dL/dg(t) in lo. Gathers lam* = dL/dg* over every
// use of the node's post-collision populations (fluid neighbour, bounce-back,
// anti-bounce-back at an open inlet, re-emission by an open outlet behind),
// then applies the transposed collision. Returns the node's dL/dR; adds
// dL/domega_g and dL/dC_in to acc where count.
template <class TT>
__device__ __forceinline__ double adj_node(CDesc &L, int x, int y, uint8_t lc, bool seg_tile,
                                           const Ph &ph, const double *lx, const double *ln,
                                           const double *g, double ux, double uy, double *lo,
                                           AdjAcc &acc, bool count) {
  using T = double;
  const T wga = (T)(TT)L.wg_axis;  // the forward step's weights
  const T wg[5] = {(T)(TT(1) - TT(4) * (TT)L.wg_axis), wga, wga, wga, wga};
  T ls[5];
  ls[0] = lx[0];
#pragma unroll
  for (int j = 1; j < 5; ++j)  // x + e_j fluid: g*_j(x) streams there
    ls[j] = ((lc >> (j - 1)) & 1) ? T(0) : ln[j];
  if (lc != 0) {
#pragma unroll
    for (int j = 1; j < 5; ++j) {
      // link toward x + e_j when that cell is not fluid
      if ((lc >> (j - 1)) & 1) {
        int code = GG_MASK_WALL;
        if (seg_tile) {
          int sx = x + EX[j], sy = y + EY[j];
          bool inside = true;
          if (sx < 0 || sx >= L.nx) {
            if (L.periodic_x) sx = (sx + L.nx) % L.nx; else inside = false;
          }
          if (sy < 0 || sy >= L.ny) {
            if (L.periodic_y) sy = (sy + L.ny) % L.ny; else inside = false;
          }
          if (inside) code = ((const GG_GLOBAL uint8_t *)L.mask)[L.node0 + sy * L.pitch + sx];
        }
        const int s = code - GG_FIRST_SEGMENT;
        const bool open = code >= GG_FIRST_SEGMENT && ((ph.open >> s) & 1u);
        if (!open) {
          ls[j] += lx[OPP[j]];  // bounce-back returns g*_j as G(x, opp j)
        } else if (L.seg_kind[s] == GG_SEG_INLET) {
          ls[j] -= lx[OPP[j]];  // anti-bounce-back
          if (count) acc.add_cin(s, 2.0 * (double)wg[OPP[j]] * (double)lx[OPP[j]]);
        }  // open outlet ahead: g*_j leaves the lattice
      }
      // an open outlet behind x re-emits g*_j(x) into x
      if (seg_tile && ((lc >> (OPP[j] - 1)) & 1)) {
        int sx = x - EX[j], sy = y - EY[j];
        bool inside = true;
        if (sx < 0 || sx >= L.nx) {
          if (L.periodic_x) sx = (sx + L.nx) % L.nx; else inside = false;
        }
        if (sy < 0 || sy >= L.ny) {
          if (L.periodic_y) sy = (sy + L.ny) % L.ny; else inside = false;
        }
        const int code = inside ? (int)((const GG_GLOBAL uint8_t *)L.mask)[L.node0 + sy * L.pitch + sx]
                                : GG_MASK_WALL;
        const int s = code - GG_FIRST_SEGMENT;
        if (code >= GG_FIRST_SEGMENT && ((ph.open >> s) & 1u) && L.seg_kind[s] == GG_SEG_OUTLET)
          ls[j] += lx[j];
      }
    }
  }
  // transposed collision with the taped state of step t
  const T dC = g[0] + g[1] + g[2] + g[3] + g[4];  // taped deviations
  const T C = (T)L.c_shift + dC;
  const T om = (T)L.omega_g, kd = (T)L.k_decay, ics = (T)L.inv_cs2g;
  T s = T(0), dr = T(0), dwl = T(0);
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const T eu = ((T)EX[j] * ux + (T)EY[j] * uy) * ics;
    const T Wj = wg[j] * (T(1) + eu);
    s += (om * Wj - kd * wg[j]) * ls[j];
    dr += wg[j] * ls[j];
    // g_j - g^eq_j from the deviations: dg_j - w_j (dC + C e.u / cs2)
    dwl -= ls[j] * (g[j] - wg[j] * (dC + C * eu));
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) lo[i] = (T(1) - om) * ls[i] + s;
  if (count) acc.dw += (double)dwl;
  return (double)dr;
}

// The taped state of step t at a node: dg_0..4, u_x, u_y (planes of TT).
template <class TT>
__device__ __forceinline__ void tape_at(const void *tape, int64_t plane, uint32_t node, double *g,
                                        double &ux, double &uy) {
#pragma unroll
  for (int i = 0; i < 5; ++i) g[i] = (double)*at<TT>(tape, plane, i, node);
  ux = (double)*at<TT>(tape, plane, 5, node);
  uy = (double)*at<TT>(tape, plane, 6, node);
}

// One adjoint step (pull over the links, then the transposed collision).
// The adjoint field is FP64 for every storage type: the tape (type TT) holds
// the forward state in its compute type; lam has no rest part to subtract,
// and an FP32 lam drifts by about 1e-7 relative per step.
template <class TT>
__global__ void __launch_bounds__(256)
    k_adjoint(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles, int n_tiles,
              int tx_shift, int64_t t, const void *__restrict__ lam_in, void *__restrict__ lam_out,
              const void *__restrict__ tape, double *__restrict__ dR, int32_t rx0, int32_t ry0,
              int32_t rw, int32_t rh, double *__restrict__ dcin, double *__restrict__ partial) {
  __shared__ double lds[4];
  const int tile = blockIdx.x;
  if (tile >= n_tiles) return;
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int x = tl.x0 + (int)(threadIdx.x & ((1 << tx_shift) - 1));
  const int y = tl.y0 + (int)(threadIdx.x >> tx_shift);
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  const uint8_t lc = (x < L.nx && y < L.ny) ? ((const GG_GLOBAL uint8_t *)L.link)[node] : NOT_FLUID;
  const bool seg_tile = (tl.flags & TILE_TOUCHES_SEGMENT) != 0;
  Ph ph{0u, nullptr};
  if (seg_tile) ph = phase_of(L, t);
  AdjAcc acc;

  if (lc != NOT_FLUID) {
    // every load is issued up front: the tape, lambda here, and lambda of
    // the four neighbours (addressable in the padded planes whatever they
    // hold; only the fluid ones are used)
    double g[5], ux, uy;
    tape_at<TT>(tape, L.plane, node, g, ux, uy);
    double lx[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) lx[i] = *at<double>(lam_in, L.plane, i, node);
    const int xm = (x == 0 && L.periodic_x) ? L.nx - 1 : x - 1;
    const int xp = (x == L.nx - 1 && L.periodic_x) ? 0 : x + 1;
    const int ym = (y == 0 && L.periodic_y) ? L.ny - 1 : y - 1;
    const int yp = (y == L.ny - 1 && L.periodic_y) ? 0 : y + 1;
    double ln[5];
    ln[0] = 0.0;
#pragma unroll
    for (int j = 1; j < 5; ++j) {
      const int xx = EX[j] > 0 ? xp : (EX[j] < 0 ? xm : x);
      const int yy = EY[j] > 0 ? yp : (EY[j] < 0 ? ym : y);
      ln[j] = *at<double>(lam_in, L.plane, j, (uint32_t)(L.node0 + yy * L.pitch + xx));
    }
    double lo[5];
    const double dr = adj_node<TT>(L, x, y, lc, seg_tile, ph, lx, ln, g, ux, uy, lo, acc, true);
#pragma unroll
    for (int i = 0; i < 5; ++i) *atw<double>(lam_out, L.plane, i, node) = lo[i];
    if (dR) {
      const int px = x - rx0, py = y - ry0;
      if (px >= 0 && px < rw && py >= 0 && py < rh) dR[py * rw + px] += dr;
    }
  }

  if (seg_tile) acc.flush_cin(dcin);
  const double bs = block_sum<256>(acc.dw, lds);
  if (threadIdx.x == 0) partial[tile] += bs;
}

// Two adjoint steps in one pass, the adjoint of the forward two-step pass:
// lam = dL/dG(t+1) in, dL/dg(t-1) out, for a tile of 62 columns x R rows
// (tiles of the forward pass's layout with their one-node halo: R + 2
// wavefronts, wavefront w on row y0 - 1 + w, lanes on the columns x0 - 1 ..
// x0 + 62). Every wavefront takes the adjoint of step t on its row (lam of
// step t + 1 read around each node), the components that the owned rows
// pull from the rows above and below go through LDS, and after one barrier
// the owned rows take the adjoint of step t - 1 and store it. Each node goes
// through adj_node with the same inputs as in two single adjoint steps (the
// same lam; the gradients of dL/dR add in the same order).
template <class TT, int R>
__global__ void __launch_bounds__((R + 2) * 64)
    k_adjoint2(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles, int n_tiles,
               int per_xcd, int64_t t, const void *__restrict__ lam_in, void *__restrict__ lam_out,
               const void *__restrict__ tape_t, const void *__restrict__ tape_tm1,
               double *__restrict__ dR, int32_t rx0, int32_t ry0, int32_t rw, int32_t rh,
               double *__restrict__ dcin, double *__restrict__ partial) {
  __shared__ double lds_up[R + 2][64];  // lam_4 of step t: pulled by the row above
  __shared__ double lds_dn[R + 2][64];  // lam_2 of step t: pulled by the row below
  __shared__ double lds_sum[R + 2];
  const int lane = (int)(threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int b = (int)blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  if (tile >= n_tiles) return;  // the same for the whole work-group
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int nx = L.nx, ny = L.ny, pitch = L.pitch;
  const int rows = tl.flags >> 8;
  const bool seg = (tl.flags & TILE_TOUCHES_SEGMENT) != 0;
  Ph ph1{0u, nullptr}, ph2{0u, nullptr};
  if (seg) {
    ph1 = phase_of(L, t);
    ph2 = phase_of(L, t - 1);
  }
  const int xr = tl.x0 - 1 + lane;
  int x = xr;
  if (L.periodic_x) x = xr < 0 ? xr + nx : (xr >= nx ? xr - nx : xr);
  const int yr = tl.y0 - 1 + w;
  int y = yr;
  if (L.periodic_y) y = yr < 0 ? yr + ny : (yr >= ny ? yr - ny : yr);
  const bool live = xr >= -1 && xr <= nx && yr >= -1 && yr <= ny && w <= rows + 1;
  const bool own = lane >= 1 && lane <= 62 && xr >= 0 && xr < nx && w >= 1 && w <= rows && yr < ny;
  const uint32_t node = (uint32_t)(L.node0 + y * pitch + x);
  const uint8_t lc = live ? ((const GG_GLOBAL uint8_t *)L.link)[live ? node : (uint32_t)L.node0]
                          : NOT_FLUID;
  AdjAcc acc;
  double dr1 = 0.0, dr2 = 0.0;
  // the tape of step t - 1 of the owned nodes, loaded up front (raw words;
  // taken to FP64 where step t - 1 is taken)
  const bool own_fluid = own && lc != NOT_FLUID;
  TT tr[7];
  if (own_fluid) {
#pragma unroll
    for (int i = 0; i < 7; ++i) tr[i] = *at<TT>(tape_tm1, L.plane, i, node);
  }

  // adjoint of step t on every fluid node of the row (halo included)
  double lt[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (lc != NOT_FLUID) {
    double g[5], ux, uy;
    tape_at<TT>(tape_t, L.plane, node, g, ux, uy);
    double lx[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) lx[i] = *at<double>(lam_in, L.plane, i, node);
    const int xm = (x == 0 && L.periodic_x) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1 && L.periodic_x) ? 0 : x + 1;
    const int ym = (y == 0 && L.periodic_y) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1 && L.periodic_y) ? 0 : y + 1;
    double ln[5];
    ln[0] = 0.0;
#pragma unroll
    for (int j = 1; j < 5; ++j) {
      const int xx = EX[j] > 0 ? xp : (EX[j] < 0 ? xm : x);
      const int yy = EY[j] > 0 ? yp : (EY[j] < 0 ? ym : y);
      ln[j] = *at<double>(lam_in, L.plane, j, (uint32_t)(L.node0 + yy * pitch + xx));
    }
    dr1 = adj_node<TT>(L, x, y, lc, seg, ph1, lx, ln, g, ux, uy, lt, acc, own);
  }
  // lam of step t that neighbours pull: lam_1 from the right, lam_3 from
  // the left (lane shifts), lam_2 from the row above, lam_4 from below
  const double p1 = __shfl_down(lt[1], 1), p3 = __shfl_up(lt[3], 1);
  lds_dn[w][lane] = lt[2];
  lds_up[w][lane] = lt[4];
  __syncthreads();

  // adjoint of step t - 1 on the owned fluid nodes
  if (own_fluid) {
    double g[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = (double)tr[i];
    const double ux = (double)tr[5], uy = (double)tr[6];
    double ln[5];
    ln[0] = 0.0;
    ln[1] = p1;
    ln[2] = lds_dn[w + 1][lane];
    ln[3] = p3;
    ln[4] = lds_up[w - 1][lane];
    double lo[5];
    dr2 = adj_node<TT>(L, x, y, lc, seg, ph2, lt, ln, g, ux, uy, lo, acc, true);
#pragma unroll
    for (int i = 0; i < 5; ++i) *atw<double>(lam_out, L.plane, i, node) = lo[i];
    if (dR) {
      const int px = x - rx0, py = y - ry0;
      if (px >= 0 && px < rw && py >= 0 && py < rh) {
        double *d = dR + py * rw + px;
        *d += dr1;  // the two steps in the order two single steps add them
        *d += dr2;
      }
    }
  }
  if (seg) acc.flush_cin(dcin);
  // dL/domega_g: one partial sum per tile
  const double v = wsum(acc.dw);
  if (lane == 0) lds_sum[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int k = 0; k < R + 2; ++k) sum += lds_sum[k];
    partial[tile] += sum;
  }
}

}  // namespace

hipError_t launch_seed(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                       int tx_shift, const double *weight, const double *target, void *lam,
                       double *partial, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  switch (s) {
    case GG_F64: k_seed<double><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, weight, target, lam, partial); break;
    case GG_F32: k_seed<float><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, weight, target, lam, partial); break;
    case GG_F16_SHIFTED: k_seed<__half><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, weight, target, lam, partial); break;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint2(gg_storage s, int rows, const LatDesc *d, const Tile *tiles, int n_tiles,
                           int64_t t, const void *lam_in, void *lam_out, const void *tape_t,
                           const void *tape_tm1, double *dR, const int32_t box[4], double *dcin,
                           double *partial, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  const int per_xcd = (n_tiles + 7) / 8;
  const int grid = 8 * per_xcd;
#define GG_LAUNCHA2(TT, RV)                                                                    \
  k_adjoint2<TT, RV><<<grid, ((RV) + 2) * 64, 0, st>>>(d, tiles, n_tiles, per_xcd, t, lam_in,  \
                                                        lam_out, tape_t, tape_tm1, dR, box[0], \
                                                        box[1], box[2], box[3], dcin, partial)
  if (s == GG_F64) {
    if (rows <= 6) GG_LAUNCHA2(double, 6); else GG_LAUNCHA2(double, 14);
  } else {
    if (rows <= 6) GG_LAUNCHA2(float, 6); else GG_LAUNCHA2(float, 14);
  }
#undef GG_LAUNCHA2
  return hipGetLastError();
}

hipError_t launch_adjoint(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                          int tx_shift, int64_t t, const void *lam_in, void *lam_out,
                          const void *tape, double *dR, const int32_t box[4], double *dcin,
                          double *partial, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (s == GG_F64)
    k_adjoint<double><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, t, lam_in, lam_out, tape,
                                              dR, box[0], box[1], box[2], box[3], dcin, partial);
  else
    k_adjoint<float><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, t, lam_in, lam_out, tape,
                                             dR, box[0], box[1], box[2], box[3], dcin, partial);
  return hipGetLastError();
}

}  // namespace gg
