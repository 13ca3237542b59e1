// gfx950 kernels of the compound lattice alone on frozen velocity fields.
//
// The paper computes the flow of each valve configuration once (it reaches
// its steady state long before the compound does) and then advances the
// advection-diffusion lattice on its own, driven by that fixed velocity
// field (Results section). Here a field is a pair of planes in the compute
// type, one slot per valve configuration, and each schedule phase names the
// slot it uses. A step reads the 5 compound populations (AA pattern, as in
// the coupled step), the 2 velocity components and the link code, and
// writes the 5 populations: per node FP32 5 x 4 x 2 + 2 x 4 + 1 = 49 bytes
// against 113 for the coupled step. The fluid populations are left alone.
// The compound arithmetic is the coupled step's (compound_collide and the
// same link rules), so with the velocity the coupled step's fluid has the
// result is the coupled step's compound.
#include "gg_device.h"
#include "gg_kernels.h"
#include "gg_node.h"

namespace gg {

namespace {

template <class T>
__device__ __forceinline__ const GG_GLOBAL T *field_plane(CDesc &L, int slot, int c) {
  return (const GG_GLOBAL T *)L.ufield + (int64_t)(2 * slot + c) * L.plane;
}

// One compound-only step over a tile list (one node per lane); ODD is the
// parity of the step. Block b takes tile (b mod 8) * per_xcd + b / 8, so
// each XCD does a contiguous run of tiles (work-groups are dealt to the 8
// XCDs round-robin), and neighbouring tiles, which store into each other's
// edge lines on odd steps, share an L2.
template <class S, bool ODD, bool PAIRS>
__global__ void __launch_bounds__(256)
    k_cde(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles, int n_tiles,
          int per_xcd, int tx_shift, int dt) {
  using P = Pop<S>;
  using T = typename P::T;
  using W = typename P::W;
  const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (tile >= n_tiles) return;
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int tmask = (1 << tx_shift) - 1;
  const int x = tl.x0 + (int)(threadIdx.x & tmask);
  const int y = tl.y0 + (int)(threadIdx.x >> tx_shift);
  const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
  const bool seg_tile = (tl.flags & TILE_TOUCHES_SEGMENT) != 0;
  const PhaseNow ph = phase_at(L, t);
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  const uint8_t lc = (x < L.nx && y < L.ny) ? ((const GG_GLOBAL uint8_t *)L.link)[node] : NOT_FLUID;
  Flux fx;
  if (lc != NOT_FLUID) {
    const Planes<W> pl(L.pop, L.plane, PAIRS);  // (the lattice's layout)
    const Neigh nb(L, x, y);
    T g[5];
    if (!ODD) {
#pragma unroll
      for (int i = 0; i < 5; ++i) g[i] = P::ld(pl.at(9 + i, node));
    } else {
      g[0] = P::ld(pl.at(9, node));
#pragma unroll
      for (int i = 1; i < 5; ++i)
        g[i] = ((lc >> (OPP[i] - 1)) & 1) ? P::ld(pl.at(9 + i, node))
                                         : P::ld(pl.at(9 + OPP[i], nb.idx[OPP[i]]));
    }
    const int slot = L.phase_field[ph.index];
    const T ux = field_plane<T>(L, slot, 0)[node];
    const T uy = field_plane<T>(L, slot, 1)[node];
    T pg[5], in_g[5];
    compound_collide<T>(L, x, y, g, ux, uy, pg);
    compound_links<T>(L, x, y, lc, seg_tile, ph, g, pg, in_g, fx, true);
    if (!ODD) {
#pragma unroll
      for (int j = 0; j < 5; ++j) P::st(pl.at(9 + j, node), in_g[j]);
    } else {
      P::st(pl.at(9, node), pg[0]);
#pragma unroll
      for (int i = 1; i < 5; ++i) P::st(pl.at(9 + i, nb.idx[i]), pg[i]);
      if (lc != 0) {
#pragma unroll
        for (int i = 1; i < 5; ++i)
          if ((lc >> (i - 1)) & 1) P::st(pl.at(9 + OPP[i], node), in_g[OPP[i]]);
      }
    }
  }
  if (seg_tile) fx.flush((double *)L.flux);
}

// Two compound-only steps in one pass (t even, natural order in): one
// work-group of R + 2 wavefronts per tile of 62 columns x (flags >> 8) rows,
// wavefront w on lattice row y0 - 1 + w, lanes on the columns x0 - 1 ..
// x0 + 62. Every wavefront does step t on its row (the halo once more for
// the populations it sends into the tile); g1 and g3 cross columns through
// lane shifts, g2 and g4 cross rows through LDS; after one barrier the
// owned rows do step t + 1 and store the state at t + 2 in natural order
// into the other plane set. The velocity is read once for both steps
// (again only when the phase of step t + 1 uses another field). The values
// between the steps are rounded to the storage type, as a store and load
// would round them, so the result is the single steps' bit for bit. Per
// node and pass (FP32): 5 populations read and written, 2 field values and
// the link code read, 49 bytes for two steps. PRESS (lattices with pressure
// segments): the pressure rule at the links, and the compound's rescaling
// (Eq. 10) of a node next to an open pressure segment between the two
// steps, in registers, as the rescaling kernel does it after a single step;
// with bit 1 of dir set, also of the state at t as loaded, in every row of
// the tile, halo included (the caller then marks as segment tiles all tiles
// whose rows or halo hold a node next to a segment), else that kernel
// follows the pass.
template <class S, int R, bool PRESS, bool PAIRS>
__global__ void __launch_bounds__((R + 2) * 64)
    k_cde_tile2(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles, int n_tiles,
                int per_xcd, int dir, int dt) {
  using P = Pop<S>;
  using T = typename P::T;
  using W = typename P::W;
  __shared__ T lds_up[R + 2][64];
  __shared__ T lds_dn[R + 2][64];
  const int lane = (int)(threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (tile >= n_tiles) return;  // the whole work-group
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int nx = L.nx, ny = L.ny;
  const int rows = strip_rows(tl.flags);
  const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
  const bool seg = (tl.flags & TILE_TOUCHES_SEGMENT) != 0;
  const PhaseNow ph1 = phase_at(L, t);
  const PhaseNow ph2 = phase_at(L, t + 1);
  const int s1 = L.phase_field[ph1.index];
  const int s2 = L.phase_field[ph2.index];
  const int dsel = PRESS ? (dir & 1) : dir;
  const Planes<W> src(dsel ? L.pop_b : L.pop, L.plane, PAIRS);  // (the lattice's layout)
  const Planes<W> dst(dsel ? L.pop : L.pop_b, L.plane, PAIRS);

  const int xr = tl.x0 - 1 + lane;
  int x = xr;
  if (L.periodic_x) x = xr < 0 ? xr + nx : (xr >= nx ? xr - nx : xr);
  const bool col = xr >= -1 && xr <= nx;
  const bool own_col = lane >= 1 && lane <= STRIP_W && xr >= 0 && xr < nx;
  const int yr = tl.y0 - 1 + w;
  int y = yr;
  if (L.periodic_y) y = yr < 0 ? yr + ny : (yr >= ny ? yr - ny : yr);
  const bool row = yr >= -1 && yr <= ny && w <= rows + 1;
  const bool own = own_col && w >= 1 && w <= rows && yr < ny;
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  uint8_t lc = NOT_FLUID;
  T g[5], ux = T(0), uy = T(0);
  uint32_t nbr[2] = {0u, 0u};
  if (row && col) {
    lc = ((const GG_GLOBAL uint8_t *)L.link)[node];
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = P::ld(src.at(9 + i, node));
    ux = field_plane<T>(L, s1, 0)[node];
    uy = field_plane<T>(L, s1, 1)[node];
    // the neighbours' mask values, for the rescaling (cells inside the
    // lattice only: their neighbours all lie in the padded planes)
    if (PRESS && seg && x >= 0 && x < nx && y >= 0 && y < ny) {
      const Neigh nb(L, x, y);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        nbr[k >> 2] |= (uint32_t)((const GG_GLOBAL uint8_t *)L.mask)[nb.idx[k + 1]] << (8 * (k & 3));
    }
  }

  // step t on this row
  Flux fx;
  if (PRESS && seg && (dir & 2) && lc != NOT_FLUID && lc != 0) {
    // the compound's rescaling after step t - 1 (flux counted by the owner)
    const PhaseNow ph0 = phase_at(L, t - 1);
    const int ps = pressure_source(L, lc, ph0, nbr);
    if (ps >= 0) {
      T unused[9];
      double dm, dc;
      rescale_node<T>(L, ps, ph0, false, unused, g, dm, dc);
#pragma unroll
      for (int i = 0; i < 5; ++i) g[i] = P::rt(g[i]);
      if (own) fx.add(ps, dm, dc);
    }
  }
  T pg[5], ing[5];
  if (lc != NOT_FLUID) {
    compound_collide<T>(L, x, y, g, ux, uy, pg);
    compound_links<T, PRESS>(L, x, y, lc, seg, ph1, g, pg, ing, fx, own);
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) pg[i] = ing[i] = T(0);
  }
  const T z1 = from_left(pg[1]), z3 = from_right(pg[3]);
  lds_up[w][lane] = pg[2];
  lds_dn[w][lane] = pg[4];
  __syncthreads();

  // step t + 1 on the owned rows
  if (own && lc != NOT_FLUID) {
    T sg[5];
    sg[0] = P::rt(pg[0]);
    sg[1] = P::rt(src_solid(lc, 1) ? ing[1] : z1);
    sg[3] = P::rt(src_solid(lc, 3) ? ing[3] : z3);
    sg[2] = P::rt(src_solid(lc, 2) ? ing[2] : lds_up[w - 1][lane]);
    sg[4] = P::rt(src_solid(lc, 4) ? ing[4] : lds_dn[w + 1][lane]);
    if (PRESS && seg) {
      const int ps = pressure_source(L, lc, ph1, nbr);
      if (ps >= 0) {
        T unused[9];
        double dm, dc;
        rescale_node<T>(L, ps, ph1, false, unused, sg, dm, dc);
#pragma unroll
        for (int i = 0; i < 5; ++i) sg[i] = P::rt(sg[i]);
        fx.add(ps, dm, dc);
      }
    }
    if (s2 != s1) {
      ux = field_plane<T>(L, s2, 0)[node];
      uy = field_plane<T>(L, s2, 1)[node];
    }
    T qg[5], jg[5];
    compound_collide<T>(L, x, y, sg, ux, uy, qg);
    compound_links<T, PRESS>(L, x, y, lc, seg, ph2, sg, qg, jg, fx, true);
    const Neigh nb(L, x, y);
    P::st(dst.at(9, node), qg[0]);
#pragma unroll
    for (int i = 1; i < 5; ++i) P::st(dst.at(9 + i, nb.idx[i]), qg[i]);
    if (lc != 0) {
      // x + e_i not fluid: the value arriving along opp(i) stays here
#pragma unroll
      for (int i = 1; i < 5; ++i)
        if ((lc >> (i - 1)) & 1) P::st(dst.at(9 + OPP[i], node), jg[OPP[i]]);
    }
  }
  if (seg) fx.flush((double *)L.flux);
}

// Velocity of the current fluid state times scale into field slot `slot`
// (compute type; the product rounded once).
template <class S>
__global__ void __launch_bounds__(256)
    k_capture(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles, int n_tiles,
              int tx_shift, int slot, double scale) {
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
  GG_GLOBAL T *ux = (GG_GLOBAL T *)field_plane<T>(L, slot, 0);
  GG_GLOBAL T *uy = (GG_GLOBAL T *)field_plane<T>(L, slot, 1);
  if (lc == NOT_FLUID) {
    ux[node] = T(0);
    uy[node] = T(0);
    return;
  }
  const Planes<typename Pop<S>::W> pl(L);
  const Neigh nb(L, x, y);
  T f[9], g[5];
  if (*(const GG_CONST int64_t *)L.t & 1)
    load_state<S, true>(pl, node, lc, nb, f, g);
  else
    load_state<S, false>(pl, node, lc, nb, f, g);
  T rho, drho, vx, vy;
  node_velocity<T>(L, f, rho, drho, vx, vy);
  ux[node] = vx * (T)scale;
  uy[node] = vy * (T)scale;
}

// A given field (host order y * nx + x, FP64) times scale into slot `slot`
// (the product in FP64, then rounded to the compute type).
template <class T>
__global__ void __launch_bounds__(256)
    k_put_field(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles, int n_tiles,
                int tx_shift, int slot, const double *__restrict__ ux_in,
                const double *__restrict__ uy_in, double scale) {
  const int tile = blockIdx.x;
  if (tile >= n_tiles) return;
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int tmask = (1 << tx_shift) - 1;
  const int x = tl.x0 + (int)(threadIdx.x & tmask);
  const int y = tl.y0 + (int)(threadIdx.x >> tx_shift);
  if (x >= L.nx || y >= L.ny) return;
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  const int k = y * L.nx + x;
  ((GG_GLOBAL T *)field_plane<T>(L, slot, 0))[node] = (T)(scale * ux_in[k]);
  ((GG_GLOBAL T *)field_plane<T>(L, slot, 1))[node] = (T)(scale * uy_in[k]);
}

// Four compound-only steps per pass over memory (no pressure segments):
// tiles of 58 columns x R rows, R + 6 wavefronts (wavefront w on row
// y0 - 3 + w, its lanes on the columns x0 - 3 .. x0 + 60), as the coupled
// four-step pass: step t on every row and column of the tile and its
// three-node halo, g1/g3 to the next column by lane shifts, g2/g4 to the
// next row through LDS (two buffers, alternating), steps t + 1 and t + 2 on
// the rows and columns whose state they can complete, step t + 3 on the
// owned nodes, pushed into the neighbours' slots of the other plane set. The
// field is read once, again only when a later step's phase uses another
// slot. The state between steps is rounded to the storage type, so the
// pass leaves what four single steps leave. Segment links are taken per
// tile (flag), for tiles with one within two nodes of their own.
template <class S, int R, bool PAIRS>
__global__ void __launch_bounds__((R + 6) * 64)
    k_cde_tile4(const LatDesc *__restrict__ desc, const Tile *__restrict__ tiles, int n_tiles,
                int per_xcd, int dir, int dt) {
  using P = Pop<S>;
  using T = typename P::T;
  using W = typename P::W;
  constexpr int NW = R + 6;
  __shared__ T lds_up[2][NW][64];
  __shared__ T lds_dn[2][NW][64];
  const int lane = (int)(threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (tile >= n_tiles) return;  // the whole work-group
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
  CDesc &L = *(CDesc *)desc;
  const int nx = L.nx, ny = L.ny;
  const int rows = strip_rows(tl.flags);
  const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
  const bool seg = (tl.flags & TILE_TOUCHES_SEGMENT) != 0;
  PhaseNow ph[4];
  int sl[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ph[k] = phase_at(L, t + k);
    sl[k] = L.phase_field[ph[k].index];
  }
  const Planes<W> src(dir ? L.pop_b : L.pop, L.plane, PAIRS);
  const Planes<W> dst(dir ? L.pop : L.pop_b, L.plane, PAIRS);

  const int xr = tl.x0 - 3 + lane;
  // addressable: the padding column on each side, or on a periodic axis
  // the three-node halo wrapped once
  const bool col = L.periodic_x ? xr >= -3 && xr <= nx + 2 : xr >= -1 && xr <= nx;
  int x = xr;
  if (L.periodic_x) x = xr < 0 ? xr + nx : (xr >= nx ? xr - nx : xr);
  const bool own_col = lane >= 3 && lane < 3 + STRIP4_W && xr >= 0 && xr < nx;
  const int yr = tl.y0 - 3 + w;
  int y = yr;
  if (L.periodic_y) y = yr < 0 ? yr + ny : (yr >= ny ? yr - ny : yr);
  const bool row =
      (L.periodic_y ? yr >= -3 && yr <= ny + 2 : yr >= -1 && yr <= ny) && w <= rows + 5;
  const bool own = own_col && w >= 3 && w < 3 + rows && yr < ny;
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  uint8_t lc = NOT_FLUID;
  T g[5], ux = T(0), uy = T(0);
  if (row && col) {
    lc = ((const GG_GLOBAL uint8_t *)L.link)[node];
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = P::ld(src.at(9 + i, node));
    ux = field_plane<T>(L, sl[0], 0)[node];
    uy = field_plane<T>(L, sl[0], 1)[node];
  }

  // step t on every row
  Flux fx;
  T pg[5], ing[5];
  if (lc != NOT_FLUID) {
    compound_collide<T>(L, x, y, g, ux, uy, pg);
    compound_links<T, false>(L, x, y, lc, seg, ph[0], g, pg, ing, fx, own);
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) pg[i] = ing[i] = T(0);
  }
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    const int q = (k - 1) & 1;
    const T z1 = from_left(pg[1]), z3 = from_right(pg[3]);
    lds_up[q][w][lane] = pg[2];
    lds_dn[q][w][lane] = pg[4];
    __syncthreads();
    // rows whose state at t + k is needed (wave-uniform)
    const bool act = w >= k && w < NW - k;
    const bool run = (k < 3 ? act : own) && lc != NOT_FLUID;
    if (run) {
      T sg[5];
      sg[0] = P::rt(pg[0]);
      sg[1] = P::rt(src_solid(lc, 1) ? ing[1] : z1);
      sg[3] = P::rt(src_solid(lc, 3) ? ing[3] : z3);
      sg[2] = P::rt(src_solid(lc, 2) ? ing[2] : lds_up[q][w - 1][lane]);
      sg[4] = P::rt(src_solid(lc, 4) ? ing[4] : lds_dn[q][w + 1][lane]);
      if (sl[k] != sl[k - 1]) {  // (uniform) the phase of this step uses another field
        ux = field_plane<T>(L, sl[k], 0)[node];
        uy = field_plane<T>(L, sl[k], 1)[node];
      }
      if (k < 3) {
        compound_collide<T>(L, x, y, sg, ux, uy, pg);
        compound_links<T, false>(L, x, y, lc, seg, ph[k], sg, pg, ing, fx, own);
      } else {
        T qg[5], jg[5];
        compound_collide<T>(L, x, y, sg, ux, uy, qg);
        compound_links<T, false>(L, x, y, lc, seg, ph[3], sg, qg, jg, fx, true);
        const Neigh nb(L, x, y);
        P::st(dst.at(9, node), qg[0]);
#pragma unroll
        for (int i = 1; i < 5; ++i) P::st(dst.at(9 + i, nb.idx[i]), qg[i]);
        if (lc != 0) {
          // x + e_i not fluid: the value arriving along opp(i) stays here
#pragma unroll
          for (int i = 1; i < 5; ++i)
            if ((lc >> (i - 1)) & 1) P::st(dst.at(9 + OPP[i], node), jg[OPP[i]]);
        }
      }
    }
  }
  if (seg) fx.flush((double *)L.flux);
}

}  // namespace

hipError_t launch_cde(gg_storage s, bool pairs, bool odd, const LatDesc *d, const Tile *tiles,
                      int n_tiles, int tx_shift, int dt, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  const int per_xcd = (n_tiles + 7) / 8;
  const int grid = 8 * per_xcd;
#define GG_CDE_P(TYPE, PV)                                                                    \
  (odd ? k_cde<TYPE, true, PV><<<grid, 256, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt) \
       : k_cde<TYPE, false, PV><<<grid, 256, 0, st>>>(d, tiles, n_tiles, per_xcd, tx_shift, dt))
#define GG_CDE(TYPE) (pairs ? GG_CDE_P(TYPE, true) : GG_CDE_P(TYPE, false))
  switch (s) {
    case GG_F64: GG_CDE(double); break;
    case GG_F32: GG_CDE(float); break;
    case GG_F16_SHIFTED: GG_CDE(__half); break;
  }
#undef GG_CDE
#undef GG_CDE_P
  return hipGetLastError();
}

hipError_t launch_cde_tile2(gg_storage s, bool pairs, int rows, const LatDesc *d,
                            const Tile *tiles, int n_tiles, int dir, int dt, hipStream_t st,
                            bool press) {
  if (n_tiles <= 0) return hipSuccess;
  const int per_xcd = (n_tiles + 7) / 8;
  const int grid = 8 * per_xcd;
#define GG_CDE2(TYPE, RV, PV)                                                                \
  (pairs ? k_cde_tile2<TYPE, RV, PV, true><<<grid, ((RV) + 2) * 64, 0, st>>>(d, tiles, n_tiles, \
                                                                           per_xcd, dir, dt)   \
         : k_cde_tile2<TYPE, RV, PV, false><<<grid, ((RV) + 2) * 64, 0, st>>>(d, tiles, n_tiles, \
                                                                            per_xcd, dir, dt))
#define GG_CDE2_R(TYPE)                                  \
  do {                                                   \
    if (press && rows <= 6) GG_CDE2(TYPE, 6, true);      \
    else if (press) GG_CDE2(TYPE, 14, true);             \
    else if (rows <= 6) GG_CDE2(TYPE, 6, false);         \
    else GG_CDE2(TYPE, 14, false);                       \
  } while (0)
  switch (s) {
    case GG_F64: GG_CDE2_R(double); break;
    case GG_F32: GG_CDE2_R(float); break;
    case GG_F16_SHIFTED: GG_CDE2_R(__half); break;
  }
#undef GG_CDE2_R
#undef GG_CDE2
  return hipGetLastError();
}

hipError_t launch_cde_tile4(gg_storage s, bool pairs, int rows, const LatDesc *d,
                            const Tile *tiles, int n_tiles, int dir, int dt, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  const int per_xcd = (n_tiles + 7) / 8;
  const int grid = 8 * per_xcd;
#define GG_CDE4_R(TYPE, RV)                                                                    \
  (pairs ? k_cde_tile4<TYPE, RV, true><<<grid, ((RV) + 6) * 64, 0, st>>>(d, tiles, n_tiles,     \
                                                                         per_xcd, dir, dt)      \
         : k_cde_tile4<TYPE, RV, false><<<grid, ((RV) + 6) * 64, 0, st>>>(d, tiles, n_tiles,    \
                                                                          per_xcd, dir, dt))
#define GG_CDE4(TYPE) (rows <= 6 ? GG_CDE4_R(TYPE, 6) : GG_CDE4_R(TYPE, 10))
  switch (s) {
    case GG_F64: GG_CDE4(double); break;
    case GG_F32: GG_CDE4(float); break;
    case GG_F16_SHIFTED: GG_CDE4(__half); break;
  }
#undef GG_CDE4
#undef GG_CDE4_R
  return hipGetLastError();
}

hipError_t launch_capture(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                          int tx_shift, int slot, double scale, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  switch (s) {
    case GG_F64:
      k_capture<double><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, slot, scale);
      break;
    case GG_F32:
      k_capture<float><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, slot, scale);
      break;
    case GG_F16_SHIFTED:
      k_capture<__half><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, slot, scale);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_put_field(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                            int tx_shift, int slot, const double *ux, const double *uy,
                            double scale, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (s == GG_F64)
    k_put_field<double><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, slot, ux, uy, scale);
  else
    k_put_field<float><<<n_tiles, 256, 0, st>>>(d, tiles, n_tiles, tx_shift, slot, ux, uy, scale);
  return hipGetLastError();
}

}  // namespace gg
