// gfx950 kernels of the coupled D2Q9 + D2Q5 lattice Boltzmann step.
//
// In-place AA streaming over structure-of-arrays planes. With A[x][i] the
// slot of population i at node x, a time step t does, for every fluid node:
//   even t: read A[x][i] = f_i(x,t); collide; write the value that must
//           arrive at x along direction j into A[x][j] (the post-collision
//           population of the opposite direction, or a boundary value).
//   odd t : read f_i(x,t) from A[x - e_i][opp i] (or from A[x][i] where
//           x - e_i is not fluid); collide; write f*_i into A[x + e_i][i]
//           (or a boundary value into A[x][opp i] where x + e_i is not fluid).
// Each slot is read and written by one node only within a step, so no
// synchronisation between work-groups is needed, and every boundary rule
// (paper Boundary Conditions section, read as bounce-back variants) uses
// only the node's own post-collision populations and velocity.
//
// Memory access shape: every plane is addressed as a uniform base pointer
// (scalar registers) plus a 32-bit per-lane element offset; consecutive
// lanes hold consecutive x, so each wavefront touches whole cache lines
// (shifted by one element for the x-neighbours of the odd step).
#include <algorithm>

#include "gg_device.h"
#include "gg_kernels.h"
#include "gg_node.h"

namespace gg {

// ---------------------------------------------------------------------------
// The fused coupled step.
// ---------------------------------------------------------------------------
// ODD is the parity of the step, known to the host (the layout of the state
// alternates between the two forms above).
// One tile of the fused step (every lane of the work-group calls it). TAPE:
// also write the node's state before the step to `tape` for the adjoint,
// planes of the compute type with the populations' plane stride: dg_0..4,
// then u_x, u_y (from the same moments as the collision).
template <class S, bool ODD, bool PAIRS, bool TAPE = false>
__device__ __forceinline__ void step_tile(const LatDesc *__restrict__ descs,
                                          const Tile *__restrict__ tiles, int tile,
                                          int tx_shift, int dt, void *tape = nullptr) {
  using P = Pop<S>;
  using T = typename P::T;
  using W = typename P::W;
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = ((CDesc *)descs)[tl.inst];
  const int tmask = (1 << tx_shift) - 1;
  const int x = tl.x0 + (int)(threadIdx.x & tmask);
  const int y = tl.y0 + (int)(threadIdx.x >> tx_shift);
  const int nx = L.nx, ny = L.ny, pitch = L.pitch;
  const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
  const bool seg_tile = (tl.flags & TILE_TOUCHES_SEGMENT) != 0;
  PhaseNow ph{0u, nullptr};
  if (seg_tile) ph = phase_at(L, t);

  const uint32_t node = (uint32_t)(L.node0 + y * pitch + x);
  const uint8_t lc = (x < nx && y < ny) ? ((const GG_GLOBAL uint8_t *)L.link)[node] : NOT_FLUID;

  // boundary fluxes: the lane's terms of this step summed in the compute
  // type (as every form of the step sums them), then in FP64
  FluxT<T> fx;

  if (lc != NOT_FLUID) {
    const Planes<W> pl(L.pop, L.plane, PAIRS);  // (the lattice's layout)
    const Neigh nb(L, x, y);
    T f[9], g[5];  // deviations from rest, df_i and dg_i
    load_state<S, ODD>(pl, node, lc, nb, f, g);
    if (TAPE) {
      T rho, drho, ux, uy;
      node_velocity<T>(L, f, rho, drho, ux, uy);
      const TapePlanes<T> tp(tape, L.plane);
#pragma unroll
      for (int i = 0; i < 5; ++i) *tp.at(i, node) = g[i];
      *tp.at(5, node) = ux;
      *tp.at(6, node) = uy;
    }

    T pf[9], pg[5], in_f[9], in_g[5];
    collide_node<T, true, FluxT<T>>(L, x, y, lc, seg_tile, ph, f, g, pf, pg, in_f, in_g, fx, true);

    if (!ODD && PAIRS) {  // (f_j, g_j) side by side: one access each
#pragma unroll
      for (int j = 0; j < 5; ++j) P::st_pair(pl.at(j, node), in_f[j], in_g[j]);
#pragma unroll
      for (int j = 5; j < 9; ++j) P::st(pl.at(j, node), in_f[j]);
    } else if (!ODD) {
#pragma unroll
      for (int j = 0; j < 9; ++j) P::st(pl.at(j, node), in_f[j]);
#pragma unroll
      for (int j = 0; j < 5; ++j) P::st(pl.at(9 + j, node), in_g[j]);
    } else {
      // free flight to x + e_i; where that cell is not fluid the value lands
      // in a slot nobody reads
      if (PAIRS) {
        P::st_pair(pl.at(0, node), pf[0], pg[0]);
#pragma unroll
        for (int i = 1; i < 5; ++i) P::st_pair(pl.at(i, nb.idx[i]), pf[i], pg[i]);
#pragma unroll
        for (int i = 5; i < 9; ++i) P::st(pl.at(i, nb.idx[i]), pf[i]);
      } else {
        P::st(pl.at(0, node), pf[0]);
        P::st(pl.at(9, node), pg[0]);
#pragma unroll
        for (int i = 1; i < 9; ++i) P::st(pl.at(i, nb.idx[i]), pf[i]);
#pragma unroll
        for (int i = 1; i < 5; ++i) P::st(pl.at(9 + i, nb.idx[i]), pg[i]);
      }
      if (lc != 0) {
        // x + e_i not fluid: the value arriving here along opp(i) goes to
        // this node's own slot opp(i)
#pragma unroll
        for (int i = 1; i < 9; ++i)
          if ((lc >> (i - 1)) & 1) P::st(pl.at(OPP[i], node), in_f[OPP[i]]);
#pragma unroll
        for (int i = 1; i < 5; ++i)
          if ((lc >> (i - 1)) & 1) P::st(pl.at(9 + OPP[i], node), in_g[OPP[i]]);
      }
    }
  }

  if (seg_tile) fx.flush((double *)L.flux);
}

// The fused step over a tile list. Work-groups are dealt to the 8 XCDs
// round-robin; block b handles tile (b mod 8) * per_xcd + b / 8, so each XCD
// processes a contiguous run of tiles (neighbouring tiles share an L2). With
// a grid smaller than 8 * per_xcd (a multiple of 8), blocks stride through
// the list and stay on their XCD's run (persistent launch).
template <class S, int BS, bool ODD, bool PAIRS>
__global__ void __launch_bounds__(BS)
    k_step(const LatDesc *__restrict__ descs, const Tile *__restrict__ tiles,
           int n_tiles, int per_xcd, int tx_shift, int dt) {
  const int nb = 8 * per_xcd;
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile < n_tiles) step_tile<S, ODD, PAIRS>(descs, tiles, tile, tx_shift, dt);
  }
}

// The fused step that also writes the tape of the adjoint (see step_tile).
template <class S, int BS, bool ODD, bool PAIRS>
__global__ void __launch_bounds__(BS)
    k_step_tape(const LatDesc *__restrict__ descs, const Tile *__restrict__ tiles, int n_tiles,
                int per_xcd, int tx_shift, int dt, void *__restrict__ tape) {
  const int nb = 8 * per_xcd;
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile < n_tiles) step_tile<S, ODD, PAIRS, true>(descs, tiles, tile, tx_shift, dt, tape);
  }
}

// ---------------------------------------------------------------------------
// Equilibrium initialisation (natural order, t = 0).
// ---------------------------------------------------------------------------
template <class S>
__global__ void __launch_bounds__(256)
    k_init(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles,
           int n_tiles, int tx_shift, const double *__restrict__ rho_in,
           const double *__restrict__ ux_in, const double *__restrict__ uy_in,
           const double *__restrict__ c_in) {
  using P = Pop<S>;
  using T = typename P::T;
  using W = typename P::W;
  const int tile = blockIdx.x;
  if (tile >= n_tiles) return;
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int tmask = (1 << tx_shift) - 1;
  const int x = tl.x0 + (int)(threadIdx.x & tmask);
  const int y = tl.y0 + (int)(threadIdx.x >> tx_shift);
  if (x >= L.nx || y >= L.ny) return;
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  const Planes<W> pl(L);
  if (((const GG_GLOBAL uint8_t *)L.link)[node] == NOT_FLUID) {
    // never read; stored as the rest state
    for (int i = 0; i < 14; ++i) P::st(pl.at(i, node), T(0));
    return;
  }
  // deviations from rest, differences taken in FP64
  const int k = y * L.nx + x;
  const T drho = rho_in ? (T)(rho_in[k] - L.rho0) : T(0);
  const T rho = rho_in ? (T)rho_in[k] : (T)L.rho0;
  const T ux = ux_in ? (T)ux_in[k] : T(0);
  const T uy = uy_in ? (T)uy_in[k] : T(0);
  const T C = c_in ? (T)c_in[k] : T(0);
  const T dC = (T)((c_in ? c_in[k] : 0.0) - L.c_shift);
  const T usq = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    const T eu = (T)EX[i] * ux + (T)EY[i] * uy;
    P::st(pl.at(i, node), (T)WF[i] * (drho + rho * (T(3) * eu + T(4.5) * eu * eu - T(1.5) * usq)));
  }
  const T ics = (T)L.inv_cs2g;
  const T wga = (T)L.wg_axis;
  for (int i = 0; i < 5; ++i) {
    const T w = i == 0 ? T(1) - T(4) * wga : wga;  // weights summing to one exactly
    const T eu = (T)EX[i] * ux + (T)EY[i] * uy;
    P::st(pl.at(9 + i, node), w * (dC + C * eu * ics));
  }
}

// Gathers the deviations df(x,t), dg(x,t) of the current parity for the
// auxiliary kernels.
template <class S>
__device__ __forceinline__ void gather(CDesc &L, uint32_t node, uint8_t lc, int x, int y,
                                       typename Pop<S>::T *f, typename Pop<S>::T *g) {
  const Planes<typename Pop<S>::W> pl(L);
  const Neigh nb(L, x, y);
  if (*(const GG_CONST int64_t *)L.t & 1)
    load_state<S, true>(pl, node, lc, nb, f, g);
  else
    load_state<S, false>(pl, node, lc, nb, f, g);
}

// ---------------------------------------------------------------------------
// Read-back: macroscopic fields and natural-order populations (FP64 out).
// ---------------------------------------------------------------------------
template <class S>
__global__ void __launch_bounds__(256)
    k_read(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles,
           int n_tiles, int tx_shift, double *__restrict__ rho_out,
           double *__restrict__ ux_out, double *__restrict__ uy_out,
           double *__restrict__ c_out, double *__restrict__ f_out,
           double *__restrict__ g_out) {
  using T = typename Pop<S>::T;
  const int tile = blockIdx.x;
  if (tile >= n_tiles) return;
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int tmask = (1 << tx_shift) - 1;
  const int x = tl.x0 + (int)(threadIdx.x & tmask);
  const int y = tl.y0 + (int)(threadIdx.x >> tx_shift);
  if (x >= L.nx || y >= L.ny) return;
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  const uint8_t lc = ((const GG_GLOBAL uint8_t *)L.link)[node];
  if (lc == NOT_FLUID) return;
  T fT[9], gT[5];
  gather<S>(L, node, lc, x, y, fT, gT);
  const int64_t n = (int64_t)L.nx * L.ny;
  const int k = y * L.nx + x;
  double f[9], g[5];  // deviations, FP64
  for (int i = 0; i < 9; ++i) f[i] = (double)fT[i];
  for (int i = 0; i < 5; ++i) g[i] = (double)gT[i];
  if (f_out)
    for (int i = 0; i < 9; ++i) f_out[i * n + k] = f[i] + WF[i] * L.rho0;
  if (g_out)
    for (int i = 0; i < 5; ++i) {
      // the weights of the step, in its compute type
      const T wga = (T)L.wg_axis;
      const double w = (double)(i == 0 ? T(1) - T(4) * wga : wga);
      g_out[i * n + k] = g[i] + w * L.c_shift;
    }
  const double rho = L.rho0 + (f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8]);
  const double jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const double jy = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
  if (rho_out) rho_out[k] = rho;
  if (ux_out) ux_out[k] = jx / rho;
  if (uy_out) uy_out[k] = jy / rho;
  if (c_out) c_out[k] = L.c_shift + (g[0] + g[1] + g[2] + g[3] + g[4]);
}

// Fills nx*ny doubles with a value (marks non-fluid nodes before k_read).
__global__ void k_fill(double *__restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// FP64 diagnostics: wavefront reductions, then one partial per work-group
// (no atomics, so the totals do not depend on the order of the work-groups),
// then one work-group folds the partials.
// partial[6 * tile + k] / acc[k]: [0] mass, [1] solute, [2] max|u|,
// [3] max|u| in the region, [4] non-finite count, [5] fluid count
// ---------------------------------------------------------------------------
template <class S>
__global__ void __launch_bounds__(256)
    k_reduce(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles,
             int n_tiles, int tx_shift, double *__restrict__ partial) {
  // Work-group b folds tiles b, b + gridDim.x, ... (one tile each when the
  // grid has a work-group per tile) into partial[6 * b .. 6 * b + 5].
  using T = typename Pop<S>::T;
  __shared__ double lds[4][6];
  CDesc &L = *(CDesc *)desc;
  const int tmask = (1 << tx_shift) - 1;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int tile = (int)blockIdx.x; tile < n_tiles; tile += (int)gridDim.x) {
    const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
    const int x = tl.x0 + (int)(threadIdx.x & tmask);
    const int y = tl.y0 + (int)(threadIdx.x >> tx_shift);
    const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
    const uint8_t lc = (x < L.nx && y < L.ny) ? ((const GG_GLOBAL uint8_t *)L.link)[node] : NOT_FLUID;
    if (lc == NOT_FLUID) continue;
    T fT[9], gT[5];
    gather<S>(L, node, lc, x, y, fT, gT);
    double rho = 0.0, jx = 0.0, jy = 0.0, C = 0.0;  // deviations first
    bool finite = true;
    for (int i = 0; i < 9; ++i) {
      const double q = (double)fT[i];
      finite = finite && isfinite(q);
      rho += q;
      jx += EX[i] * q;
      jy += EY[i] * q;
    }
    for (int i = 0; i < 5; ++i) {
      const double q = (double)gT[i];
      finite = finite && isfinite(q);
      C += q;
    }
    rho += L.rho0;
    C += L.c_shift;
    v[5] += 1.0;
    if (finite) {
      v[0] += rho;
      v[1] += C;
      const double um = sqrt(jx * jx + jy * jy) / rho;
      v[2] = fmax(v[2], um);
      if (L.has_region && ((const GG_GLOBAL uint8_t *)L.region)[node]) v[3] = fmax(v[3], um);
    } else {
      v[4] += 1.0;
    }
  }
  const int w = (int)(threadIdx.x >> 6);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double r = (k == 2 || k == 3) ? wave_max(v[k]) : wave_sum(v[k]);
    if (__lane_id() == 0) lds[w][k] = r;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = (int)threadIdx.x;
    double r = lds[0][k];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
      r = (k == 2 || k == 3) ? fmax(r, lds[q][k]) : r + lds[q][k];
    partial[6 * blockIdx.x + k] = r;
  }
}

// Folds the per-work-group partials into acc[0..5] (one work-group).
__global__ void __launch_bounds__(256)
    k_reduce_final(const double *__restrict__ partial, int n_tiles, double *__restrict__ acc) {
  __shared__ double lds[4][6];
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = (int)threadIdx.x; t < n_tiles; t += (int)blockDim.x)
#pragma unroll
    for (int k = 0; k < 6; ++k)
      v[k] = (k == 2 || k == 3) ? fmax(v[k], partial[6 * t + k]) : v[k] + partial[6 * t + k];
  const int w = (int)(threadIdx.x >> 6);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double r = (k == 2 || k == 3) ? wave_max(v[k]) : wave_sum(v[k]);
    if (__lane_id() == 0) lds[w][k] = r;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = (int)threadIdx.x;
    double r = lds[0][k];
    for (int q = 1; q < 4; ++q) r = (k == 2 || k == 3) ? fmax(r, lds[q][k]) : r + lds[q][k];
    acc[k] = r;
  }
}

// Plain streaming copy: one 16-byte word per lane, one lane per word (the
// fastest plain copy shape on this GPU).
__global__ void __launch_bounds__(256) k_copy(int4 *__restrict__ dst, const int4 *__restrict__ src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Set a step counter to v (the adjoint's recomputation copy, without a
// host round trip).
__global__ void k_set_counter(int64_t *__restrict__ t, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *(GG_GLOBAL int64_t *)t = v;
}

// Advance the step counters of n lattices by k (after k step launches).
__global__ void k_advance(const LatDesc *__restrict__ descs, int n, int64_t k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *(GG_GLOBAL int64_t *)descs[i].t += k;
}

// ---------------------------------------------------------------------------
// Host-side launch wrappers.
// ---------------------------------------------------------------------------
template <class S, bool ODD, bool PAIRS>
static hipError_t launch_step_p(int bs, const LatDesc *d, const Tile *tiles, int n_tiles,
                                int tx_shift, int dt, int persist, hipStream_t st) {
  const int per_xcd = (n_tiles + 7) / 8;
  const int full = 8 * per_xcd;
  const dim3 grid(persist > 0 ? std::min(full, (persist + 7) / 8 * 8) : full);
  switch (bs) {
    case 64: k_step<S, 64, ODD, PAIRS><<<grid, 64, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt); break;
    case 128: k_step<S, 128, ODD, PAIRS><<<grid, 128, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt); break;
    case 256: k_step<S, 256, ODD, PAIRS><<<grid, 256, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt); break;
    case 512: k_step<S, 512, ODD, PAIRS><<<grid, 512, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class S>
static hipError_t launch_step_s(int bs, bool odd, bool pairs, const LatDesc *d, const Tile *tiles,
                                int n_tiles, int tx_shift, int dt, int persist, hipStream_t st) {
  if (pairs)
    return odd ? launch_step_p<S, true, true>(bs, d, tiles, n_tiles, tx_shift, dt, persist, st)
               : launch_step_p<S, false, true>(bs, d, tiles, n_tiles, tx_shift, dt, persist, st);
  return odd ? launch_step_p<S, true, false>(bs, d, tiles, n_tiles, tx_shift, dt, persist, st)
             : launch_step_p<S, false, false>(bs, d, tiles, n_tiles, tx_shift, dt, persist, st);
}

hipError_t launch_step(gg_storage s, bool pairs, int block, bool odd, const LatDesc *d,
                       const Tile *tiles, int n_tiles, int tx_shift, int dt, hipStream_t st,
                       int persist) {
  if (n_tiles <= 0) return hipSuccess;
  switch (s) {
    case GG_F64:
      return launch_step_s<double>(block, odd, pairs, d, tiles, n_tiles, tx_shift, dt, persist, st);
    case GG_F32:
      return launch_step_s<float>(block, odd, pairs, d, tiles, n_tiles, tx_shift, dt, persist, st);
    case GG_F16_SHIFTED:
      return launch_step_s<__half>(block, odd, pairs, d, tiles, n_tiles, tx_shift, dt, persist, st);
  }
  return hipErrorInvalidValue;
}

template <class S, bool ODD, bool PAIRS>
static hipError_t launch_step_tape_p(int bs, const LatDesc *d, const Tile *tiles, int n_tiles,
                                     int tx_shift, int dt, void *tape, hipStream_t st) {
  const int per_xcd = (n_tiles + 7) / 8;
  const dim3 grid(8 * per_xcd);
  switch (bs) {
    case 64: k_step_tape<S, 64, ODD, PAIRS><<<grid, 64, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt, tape); break;
    case 128: k_step_tape<S, 128, ODD, PAIRS><<<grid, 128, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt, tape); break;
    case 256: k_step_tape<S, 256, ODD, PAIRS><<<grid, 256, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt, tape); break;
    case 512: k_step_tape<S, 512, ODD, PAIRS><<<grid, 512, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt, tape); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step_tape(gg_storage s, bool pairs, int block, bool odd, const LatDesc *d,
                            const Tile *tiles, int n_tiles, int tx_shift, int dt, void *tape,
                            hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
#define GG_TAPE_P(TYPE, PV)                                                                  \
  (odd ? launch_step_tape_p<TYPE, true, PV>(block, d, tiles, n_tiles, tx_shift, dt, tape, st) \
       : launch_step_tape_p<TYPE, false, PV>(block, d, tiles, n_tiles, tx_shift, dt, tape, st))
#define GG_TAPE_S(TYPE) return pairs ? GG_TAPE_P(TYPE, true) : GG_TAPE_P(TYPE, false)
  switch (s) {
    case GG_F64: GG_TAPE_S(double);
    case GG_F32: GG_TAPE_S(float);
    case GG_F16_SHIFTED: GG_TAPE_S(__half);
  }
#undef GG_TAPE_S
#undef GG_TAPE_P
  return hipErrorInvalidValue;
}

// The auxiliary kernels run 256-thread work-groups over 256-node tiles.
hipError_t launch_init(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                       int tx_shift, const double *rho, const double *ux,
                       const double *uy, const double *c, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  switch (s) {
    case GG_F64: k_init<double><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, rho, ux, uy, c); break;
    case GG_F32: k_init<float><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, rho, ux, uy, c); break;
    case GG_F16_SHIFTED: k_init<__half><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, rho, ux, uy, c); break;
  }
  return hipGetLastError();
}

hipError_t launch_read(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                       int tx_shift, double *rho, double *ux, double *uy, double *c,
                       double *f, double *g, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  switch (s) {
    case GG_F64: k_read<double><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, rho, ux, uy, c, f, g); break;
    case GG_F32: k_read<float><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, rho, ux, uy, c, f, g); break;
    case GG_F16_SHIFTED: k_read<__half><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, rho, ux, uy, c, f, g); break;
  }
  return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_reduce(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                         int tx_shift, double *partial, double *acc, hipStream_t st,
                         int max_groups) {
  if (n_tiles <= 0) return hipSuccess;
  const int groups = max_groups > 0 ? std::min(n_tiles, max_groups) : n_tiles;
  switch (s) {
    case GG_F64: k_reduce<double><<<groups, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, partial); break;
    case GG_F32: k_reduce<float><<<groups, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, partial); break;
    case GG_F16_SHIFTED: k_reduce<__half><<<groups, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, partial); break;
  }
  k_reduce_final<<<1, 256, 0, st>>>(partial, groups, acc);
  return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / 16);
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (n > 0)
    k_copy<<<(unsigned)blocks, 256, 0, st>>>(static_cast<int4 *>(dst), static_cast<const int4 *>(src), n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pressure boundary: rescaling after a step (paper Eq. 10).
// ---------------------------------------------------------------------------
// Writes the deviations df, dg of node x at a step of parity ODD back into
// the slots load_state reads them from.
template <class S, bool ODD>
__device__ __forceinline__ void store_state(const Planes<typename Pop<S>::W> &pl, uint32_t node,
                                            uint8_t lc, const Neigh &nb,
                                            const typename Pop<S>::T *f,
                                            const typename Pop<S>::T *g) {
  using P = Pop<S>;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const bool own = !ODD || i == 0 || ((lc >> (OPP[i] - 1)) & 1);
    P::st(own ? pl.at(i, node) : pl.at(OPP[i], nb.idx[OPP[i]]), f[i]);
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const bool own = !ODD || i == 0 || ((lc >> (OPP[i] - 1)) & 1);
    P::st(own ? pl.at(9 + i, node) : pl.at(9 + OPP[i], nb.idx[OPP[i]]), g[i]);
  }
}

// After step t (device counter + dt): every listed node with a link from a
// ghost cell of a pressure segment open at step t has its state at t + 1
// multiplied through so that rho = rho_s (velocity unchanged), and, where
// the segment holds the compound, C = C_in (the equilibrium at rest of
// C_in where C <= 0); the mass and compound added count as the segment's
// boundary flux. fluid = 0 leaves f alone (compound-only steps). In the
// deviation form: gamma (w rho0 + df) - w rho0 = gamma df + (gamma - 1) w rho0.
template <class S>
__global__ void __launch_bounds__(64)
    k_rescale(const LatDesc *__restrict__ desc, const int32_t *__restrict__ list, int n, int dt,
              int fluid, int other) {
  using P = Pop<S>;
  using T = typename P::T;
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  CDesc &L = *(CDesc *)desc;
  const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
  const PhaseNow ph = phase_at(L, t);
  Flux flux;
  // entry: x, y, and the pressure segments among the node's source cells,
  // one byte each (index + 1), in order of first appearance in direction
  // order 1..8: the node follows the first of them open at this step
  int s = -1, x = 0, y = 0;
  if (k < n) {
    x = list[3 * k];
    y = list[3 * k + 1];
    const uint32_t cand = (uint32_t)list[3 * k + 2];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int q = (int)((cand >> (8 * b)) & 0xFFu) - 1;
      if (s < 0 && q >= 0 && ((ph.open >> q) & 1u)) s = q;
    }
  }
  if (s >= 0) {
    const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
    const uint8_t lc = ((const GG_GLOBAL uint8_t *)L.link)[node];
    const Planes<typename P::W> pl(other ? L.pop_b : L.pop, L.plane, L.pairs != 0);
    const Neigh nb(L, x, y);
    T f[9], g[5];
    const bool odd = ((t + 1) & 1) != 0;  // parity of the state at t + 1
    if (odd)
      load_state<S, true>(pl, node, lc, nb, f, g);
    else
      load_state<S, false>(pl, node, lc, nb, f, g);
    double dm, dc;
    rescale_node<T>(L, s, ph, fluid != 0, f, g, dm, dc);
    if (odd)
      store_state<S, true>(pl, node, lc, nb, f, g);
    else
      store_state<S, false>(pl, node, lc, nb, f, g);
    flux.add(s, dm, dc);
  }
  flux.flush((double *)L.flux);  // every lane of the wavefront
}

hipError_t launch_rescale(gg_storage s, const LatDesc *d, const int32_t *xy, int n, int dt,
                          bool fluid, hipStream_t st, bool other) {
  if (n <= 0) return hipSuccess;
  const int grid = (n + 63) / 64;
  switch (s) {
    case GG_F64: k_rescale<double><<<grid, 64, 0, st>>>(d, xy, n, dt, fluid, other); break;
    case GG_F32: k_rescale<float><<<grid, 64, 0, st>>>(d, xy, n, dt, fluid, other); break;
    case GG_F16_SHIFTED: k_rescale<__half><<<grid, 64, 0, st>>>(d, xy, n, dt, fluid, other); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The paper's walls: ghost cells in place of bounce-back (fix-up kernels).
// ---------------------------------------------------------------------------
// For a fluid node z and a link i whose source s = z - e_i is a wall or a
// closed valve, s acts as a ghost node that emits, along e_i, at step t:
//   f_i^eq(rho_s, u_s), rho_s = 2 rho(z) - rho(z + e_i) (rho(z) where
//   z + e_i is not fluid), u_s = -j(z) / rho_s (momentum through zero at
//   the halfway wall), and
//   g_i^eq(C(z), u_s) + (1 - omega_g) (g_i(z) - g_i^eq(C(z), u(z)))
//   (Guo's non-equilibrium extrapolation, zero normal gradient of C),
// all of step t. k_wall_save stores, before the step, what these need of
// step t (it is overwritten in place by the step); k_wall_apply writes the
// values, after the step, into z's own slots i, where the step left the
// bounce-back value (a link from a non-fluid cell arrives in the node's own
// slot in both parities). In the compound-only step u(z) is the frozen
// field's and u_s = -u(z).
constexpr int WALL_SAVE = 16;  // d rho, j_x, j_y, dC, d rho(z + e_k) k = 1..8, dg_1..4

// Mask value of the source cell x - e_j (j = 1..8), wrapped on periodic
// axes; a wall outside the lattice otherwise.
__device__ __forceinline__ int source_code(CDesc &L, int x, int y, int j) {
  int sx = x - EX[j], sy = y - EY[j];
  if (sx < 0 || sx >= L.nx) {
    if (!L.periodic_x) return GG_MASK_WALL;
    sx = (sx + L.nx) % L.nx;
  }
  if (sy < 0 || sy >= L.ny) {
    if (!L.periodic_y) return GG_MASK_WALL;
    sy = (sy + L.ny) % L.ny;
  }
  return ((const GG_GLOBAL uint8_t *)L.mask)[L.node0 + sy * L.pitch + sx];
}

// A link from source code `code` takes the wall rule at a step in phase ph.
__device__ __forceinline__ bool wall_link(CDesc &L, int code, const PhaseNow &ph) {
  if (code == GG_MASK_WALL) return true;
  if (code < GG_FIRST_SEGMENT) return false;
  const int q = code - GG_FIRST_SEGMENT;
  return L.seg_kind[q] == 0 || !((ph.open >> q) & 1u);
}

// Deviation of the density of the fluid node at element offset `node`
// (link code lc) at a step of parity `odd`, summed in direction order.
template <class S>
__device__ __forceinline__ typename Pop<S>::T node_drho(CDesc &L,
                                                        const Planes<typename Pop<S>::W> &pl,
                                                        int x, int y, uint32_t node, uint8_t lc,
                                                        bool odd) {
#pragma clang fp contract(off)
  typename Pop<S>::T f[9], g[5];
  const Neigh nb(L, x, y);
  if (odd) load_state<S, true>(pl, node, lc, nb, f, g);
  else load_state<S, false>(pl, node, lc, nb, f, g);
  return f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
}

// Before step t (device counter + dt). Threads 0 .. n - 1: the moments of
// listed node k (d rho, j, dC) and its dg_1..4 into save[k]; threads n ..
// n + n_links - 1 (fluid steps only): for the link entry (x, y, k * 8 +
// (i - 1)) of node k at (x, y),
// the density deviation of z + e_i into save[k][3 + i], or that of z
// itself where z + e_i is not fluid (then 2 d rho - d rho = d rho exactly:
// rho_s = rho(z)). One thread per link keeps the loads of a node's
// extrapolation partners in parallel.
template <class S>
__global__ void __launch_bounds__(64)
    k_wall_save(const LatDesc *__restrict__ desc, const int32_t *__restrict__ xy, int n,
                const int32_t *__restrict__ links, int n_links, int dt, int fluid,
                typename Pop<S>::T *__restrict__ save) {
#pragma clang fp contract(off)
  using P = Pop<S>;
  using T = typename P::T;
  const int tid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (tid >= n + (fluid ? n_links : 0)) return;
  CDesc &L = *(CDesc *)desc;
  const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
  const bool odd = (t & 1) != 0;
  const Planes<typename P::W> pl(L);
  if (tid < n) {
    const int x = xy[2 * tid], y = xy[2 * tid + 1];
    const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
    const uint8_t lc = ((const GG_GLOBAL uint8_t *)L.link)[node];
    T f[9], g[5];
    const Neigh nb(L, x, y);
    if (odd) load_state<S, true>(pl, node, lc, nb, f, g);
    else load_state<S, false>(pl, node, lc, nb, f, g);
    T *o = save + (size_t)tid * WALL_SAVE;
    o[0] = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    o[1] = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    o[2] = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
    o[3] = g[0] + g[1] + g[2] + g[3] + g[4];
#pragma unroll
    for (int i = 1; i < 5; ++i) o[11 + i] = g[i];
    return;
  }
  const int32_t *le = links + 3 * (tid - n);
  int x = le[0], y = le[1];
  const int k = le[2] >> 3, i = (le[2] & 7) + 1;
  int ax = x + EX[i], ay = y + EY[i];
  bool inside = true;
  if (ax < 0 || ax >= L.nx) {
    if (L.periodic_x) ax = (ax + L.nx) % L.nx; else inside = false;
  }
  if (ay < 0 || ay >= L.ny) {
    if (L.periodic_y) ay = (ay + L.ny) % L.ny; else inside = false;
  }
  uint8_t alc = NOT_FLUID;
  if (inside) alc = ((const GG_GLOBAL uint8_t *)L.link)[L.node0 + ay * L.pitch + ax];
  if (alc != NOT_FLUID) {
    x = ax;
    y = ay;
  } else {
    alc = ((const GG_GLOBAL uint8_t *)L.link)[L.node0 + y * L.pitch + x];
  }
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  save[(size_t)k * WALL_SAVE + 3 + i] = node_drho<S>(L, pl, x, y, node, alc, odd);
}

// After step t, before a pressure rescaling: one thread per link entry
// (x, y, k * 8 + (i - 1)) whose source is, at step t's phase, a wall, a closed
// valve or an unconfigured segment cell; writes the ghost's populations
// into node k's own slots i (f, fluid steps only) and 9 + i (g, i <= 4).
template <class S>
__global__ void __launch_bounds__(64)
    k_wall_apply(const LatDesc *__restrict__ desc, const int32_t *__restrict__ links,
                 int n_links, int dt,
                 const typename Pop<S>::T *__restrict__ save, int fluid) {
#pragma clang fp contract(off)
  using P = Pop<S>;
  using T = typename P::T;
  const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= n_links) return;
  CDesc &L = *(CDesc *)desc;
  const int32_t *le = links + 3 * j;
  const int k = le[2] >> 3, i = (le[2] & 7) + 1;
  if (!fluid && i > 4) return;
  const int x = le[0], y = le[1];
  const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
  const PhaseNow ph = phase_at(L, t);
  if (!wall_link(L, source_code(L, x, y, i), ph)) return;
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  const Planes<typename P::W> pl(L);
  const T *o = save + (size_t)k * WALL_SAVE;
  const T rho0 = (T)L.rho0;
  T usx, usy, ux = T(0), uy = T(0);
  if (fluid) {
    const T drs = T(2) * o[0] - o[3 + i];
    const T rs = rho0 + drs;
    usx = -o[1] / rs;
    usy = -o[2] / rs;
    const T eu = (T)EX[i] * usx + (T)EY[i] * usy;
    const T usq = usx * usx + usy * usy;
    const T poly = T(3) * eu + T(4.5) * eu * eu - T(1.5) * usq;
    P::st(pl.at(i, node), (T)WF[i] * (drs + rs * poly));
    if (i > 4) return;
    const T rho = rho0 + o[0];
    ux = o[1] / rho;
    uy = o[2] / rho;
  } else {
    const int slot = L.phase_field[ph.index];
    ux = ((const GG_GLOBAL T *)L.ufield)[(int64_t)(2 * slot) * L.plane + node];
    uy = ((const GG_GLOBAL T *)L.ufield)[(int64_t)(2 * slot + 1) * L.plane + node];
    usx = -ux;
    usy = -uy;
  }
  const T cs = (T)L.c_shift, ics = (T)L.inv_cs2g;
  const T dC = o[3];
  const T C = cs + dC;
  const T w = (T)L.wg_axis;  // i = 1..4
  const T eus = (T)EX[i] * usx + (T)EY[i] * usy;
  const T euz = (T)EX[i] * ux + (T)EY[i] * uy;
  const T eq_s = w * (dC + C * eus * ics);  // g^eq(C, u_s) - w C_s
  const T eq_z = w * (dC + C * euz * ics);  // g^eq(C, u(z)) - w C_s
  P::st(pl.at(9 + i, node), eq_s + (T(1) - (T)L.omega_g) * (o[11 + i] - eq_z));
}

hipError_t launch_wall_save(gg_storage s, const LatDesc *d, const int32_t *xy, int n,
                            const int32_t *links, int n_links, int dt, bool fluid, void *save,
                            hipStream_t st) {
  const int m = n + (fluid ? n_links : 0);
  if (m <= 0) return hipSuccess;
  const int grid = (m + 63) / 64;
  switch (s) {
    case GG_F64:
      k_wall_save<double><<<grid, 64, 0, st>>>(d, xy, n, links, n_links, dt, fluid, (double *)save);
      break;
    case GG_F32:
      k_wall_save<float><<<grid, 64, 0, st>>>(d, xy, n, links, n_links, dt, fluid, (float *)save);
      break;
    case GG_F16_SHIFTED:
      k_wall_save<__half><<<grid, 64, 0, st>>>(d, xy, n, links, n_links, dt, fluid, (float *)save);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_wall_apply(gg_storage s, const LatDesc *d, const int32_t *links, int n_links,
                             int dt, const void *save,
                             bool fluid, hipStream_t st) {
  if (n_links <= 0) return hipSuccess;
  const int grid = (n_links + 63) / 64;
  switch (s) {
    case GG_F64:
      k_wall_apply<double><<<grid, 64, 0, st>>>(d, links, n_links, dt, (const double *)save, fluid);
      break;
    case GG_F32:
      k_wall_apply<float><<<grid, 64, 0, st>>>(d, links, n_links, dt, (const float *)save, fluid);
      break;
    case GG_F16_SHIFTED:
      k_wall_apply<__half><<<grid, 64, 0, st>>>(d, links, n_links, dt, (const float *)save, fluid);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_set_counter(int64_t *t, int64_t v, hipStream_t st) {
  k_set_counter<<<1, 64, 0, st>>>(t, v);
  return hipGetLastError();
}

hipError_t launch_advance(const LatDesc *descs, int n, int64_t k, hipStream_t st) {
  k_advance<<<(n + 63) / 64, 64, 0, st>>>(descs, n, k);
  return hipGetLastError();
}

// Every element of every population plane (padding included) from the
// layout of src into that of dst.
template <class W>
__global__ void __launch_bounds__(256)
    k_relayout(void *src, void *dst, int64_t plane, int64_t n, int from_pairs, int to_pairs) {
  const Planes<W> a(src, plane, from_pairs != 0), b(dst, plane, to_pairs != 0);
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    const uint32_t idx = (uint32_t)k;
#pragma unroll
    for (int i = 0; i < NPOP; ++i) gstore(b.at(i, idx), gload((const GG_GLOBAL W *)a.at(i, idx)));
  }
}

hipError_t launch_relayout(gg_storage s, void *src, void *dst, int64_t plane, int64_t n,
                           bool from_pairs, bool to_pairs, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  switch (s) {
    case GG_F64:
      k_relayout<double><<<grid, 256, 0, st>>>(src, dst, plane, n, from_pairs, to_pairs);
      break;
    case GG_F32:
      k_relayout<float><<<grid, 256, 0, st>>>(src, dst, plane, n, from_pairs, to_pairs);
      break;
    case GG_F16_SHIFTED:
      k_relayout<unsigned short><<<grid, 256, 0, st>>>(src, dst, plane, n, from_pairs, to_pairs);
      break;
  }
  return hipGetLastError();
}

}  // namespace gg
