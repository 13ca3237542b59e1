// Two coupled time steps in one pass over memory.
//
// The lattice state at an even step t is in natural order in one plane set
// (slot i of node x holds df_i(x,t)); the pass reads it once and writes the
// state at t + 2, in natural order, into the other plane set. One wavefront
// owns a strip of 62 columns and H rows. Its 64 lanes hold the columns
// x0 - 1 .. x0 + 62 and it walks the rows y0 - 1 .. y0 + H, so the strip
// plus a one-node halo is collided once for step t:
//
//   row y:   load df, dg (natural order) -> collide (step t) -> post1(y)
//            the populations post1 sends to its own row and to the rows
//            y - 1 and y + 1 reach the right columns through lane shifts;
//   row y-1: its state at t + 1 is now complete (the populations it pulls
//            from rows y - 2, y - 1 and y, or its own boundary values where
//            the source is not fluid) -> collide (step t + 1) -> store the
//            post-collision populations into the neighbours' slots of the
//            other plane set (or boundary values into its own slots).
//
// This is the same data flow as an even AA step followed by an odd one,
// with the intermediate state kept in registers instead of memory: each node
// goes through collide_node with the same inputs (the intermediate values
// are rounded to the storage type, as a store and load would round them),
// so the result is the one the single-step kernels give. The halo lanes and
// rows are collided for step t only, for the populations they send into
// the strip; they are owned by the neighbouring strips, which collide and
// store them themselves.
#include "gg_device.h"
#include "gg_kernels.h"
#include "gg_node.h"

namespace gg {

namespace {

// Step t + 1 at node (x, y) from its state sf, sg at t + 1 (natural order),
// with the post-collision populations pushed into the neighbours' slots of
// the destination planes (or, toward a non-fluid neighbour, the value that
// arrives here along the opposite direction into this node's own slot).
template <class S, bool SEG, bool PRESS = false, class FX = Flux>
__device__ __forceinline__ void second_step(CDesc &L, const Planes<typename Pop<S>::W> &dst,
                                            int x, int y, uint8_t lc, const PhaseNow &ph,
                                            const typename Pop<S>::T *sf,
                                            const typename Pop<S>::T *sg, FX &fx,
                                            const uint32_t *nbr = nullptr) {
  using P = Pop<S>;
  using T = typename P::T;
  T qf[9], qg[5], jf[9], jg[5];
  collide_node<T, PRESS, FX>(L, x, y, lc, SEG, ph, sf, sg, qf, qg, jf, jg, fx, true, nbr);
  const uint32_t node = (uint32_t)(L.node0 + y * L.pitch + x);
  // slot i of neighbour x + e_i as nbp(i) gives it
  auto push = [&](auto nbp) {
    // (stores in pairs: one conversion for two values where FP16 is stored)
    if (dst.pairs) {  // (uniform) f_i and g_i to x + e_i in one access
      P::st_pair(dst.at(0, node), qf[0], qg[0]);
#pragma unroll
      for (int i = 1; i < 5; ++i) P::st_pair(nbp(i), qf[i], qg[i]);
#pragma unroll
      for (int i = 5; i < 9; i += 2) P::st2(nbp(i), nbp(i + 1), qf[i], qf[i + 1]);
    } else {
      P::st2(dst.at(0, node), dst.at(9, node), qf[0], qg[0]);
#pragma unroll
      for (int i = 1; i < 9; i += 2) P::st2(nbp(i), nbp(i + 1), qf[i], qf[i + 1]);
#pragma unroll
      for (int i = 1; i < 5; i += 2) P::st2(nbp(9 + i), nbp(10 + i), qg[i], qg[i + 1]);
    }
  };
  if (!L.periodic_x && !L.periodic_y) {
    // (uniform) the neighbours are node + e_x + e_y pitch, padding included:
    // the row offset goes into the scalar base, the column offset into the
    // store's immediate
    const int pitch = L.pitch;
    push([&](int k) { return dst.at_nb(k, node, EY[k > 8 ? k - 9 : k] * pitch, EX[k > 8 ? k - 9 : k]); });
  } else {
    const Neigh n(L, x, y);
    push([&](int k) { return dst.at(k, n.idx[k > 8 ? k - 9 : k]); });
  }
  if (lc != 0) {
    // x + e_i not fluid: the value arriving along opp(i) stays here
#pragma unroll
    for (int i = 1; i < 9; ++i)
      if ((lc >> (i - 1)) & 1) P::st(dst.at(OPP[i], node), jf[OPP[i]]);
#pragma unroll
    for (int i = 1; i < 5; ++i)
      if ((lc >> (i - 1)) & 1) P::st(dst.at(9 + OPP[i], node), jg[OPP[i]]);
  }
}

template <class S, bool SEG, bool PAIRS>
__device__ __forceinline__ void strip_two_steps(const LatDesc *__restrict__ descs,
                                                const Tile *__restrict__ strips, int s, int dir,
                                                int dt) {
  using P = Pop<S>;
  using T = typename P::T;
  using W = typename P::W;
  const int lane = (int)(threadIdx.x & 63);
  const GG_CONST Tile &tl = ((const GG_CONST Tile *)strips)[s];
  CDesc &L = ((CDesc *)descs)[tl.inst];
  const int nx = L.nx, ny = L.ny, pitch = L.pitch;
  const int H = strip_rows(tl.flags);
  const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
  PhaseNow ph1{0u, nullptr}, ph2{0u, nullptr};
  if (SEG) {
    ph1 = phase_at(L, t);
    ph2 = phase_at(L, t + 1);
  }
  const Planes<W> src(dir ? L.pop_b : L.pop, L.plane, PAIRS);  // (the lattice's layout)
  const Planes<W> dst(dir ? L.pop : L.pop_b, L.plane, PAIRS);
  const GG_GLOBAL uint8_t *link = (const GG_GLOBAL uint8_t *)L.link;

  // this lane's column: addressable for -1 <= x <= nx (wrapped if periodic)
  const int xr = tl.x0 - 1 + lane;
  const bool col = xr >= -1 && xr <= nx;
  int x = xr;
  if (L.periodic_x) x = xr < 0 ? xr + nx : (xr >= nx ? xr - nx : xr);
  const bool own_col = lane >= 1 && lane <= STRIP_W && xr >= 0 && xr < nx;

  // row r of the strip is lattice row y0 + r, addressable for -1 <= y <= ny
  // (wrapped if periodic)
  auto row_y = [&](int r) -> int {
    const int yr = tl.y0 + r;
    return L.periodic_y ? (yr < 0 ? yr + ny : (yr >= ny ? yr - ny : yr)) : yr;
  };
  auto node_of = [&](int r, bool &ok) -> uint32_t {
    const int yr = tl.y0 + r;
    ok = col && yr >= -1 && yr <= ny;
    return (uint32_t)(L.node0 + row_y(r) * pitch + x);
  };

  T sf[9], sg[5];  // state at t + 1 of the previous row (this column)
  T uf2 = T(0), uf5 = T(0), uf6 = T(0), ug2 = T(0);  // pulls it passes up
  uint8_t lcp = NOT_FLUID;
  int yprev = 0;
  bool own_prev = false;
#pragma unroll
  for (int i = 0; i < 9; ++i) sf[i] = T(0);
#pragma unroll
  for (int i = 0; i < 5; ++i) sg[i] = T(0);
  FluxT<T> fx;

  // Software pipeline: the link codes run two rows ahead and the
  // populations one row ahead of the row being computed, so both are in
  // flight while the current row is collided, and only fluid cells load.
  T nf[9], ng[5];
  uint8_t nlc, nnlc = NOT_FLUID;
  {
    bool ok;
    const uint32_t node = node_of(-1, ok);
    nlc = ok ? link[node] : NOT_FLUID;
    if (nlc != NOT_FLUID) {
#pragma unroll
      for (int i = 0; i < 9; ++i) nf[i] = P::ld(src.at(i, node));
#pragma unroll
      for (int i = 0; i < 5; ++i) ng[i] = P::ld(src.at(9 + i, node));
    }
    const uint32_t node2 = node_of(0, ok);
    if (ok) nnlc = link[node2];
  }

  for (int r = -1; r <= H; ++r) {
    bool ok;
    const int y = row_y(r);
    const bool own = own_col && r >= 0 && r < H && tl.y0 + r < ny;
    const uint8_t lc = nlc;
    T f[9], g[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = nf[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = ng[i];
    // loads of row r + 1 (populations) and r + 2 (link codes)
    nlc = nnlc;
    nnlc = NOT_FLUID;
    if (r < H) {
      const uint32_t node1 = node_of(r + 1, ok);
      if (nlc != NOT_FLUID) {
#pragma unroll
        for (int i = 0; i < 9; ++i) nf[i] = P::ld(src.at(i, node1));
#pragma unroll
        for (int i = 0; i < 5; ++i) ng[i] = P::ld(src.at(9 + i, node1));
      }
      if (r + 1 < H) {
        const uint32_t node2 = node_of(r + 2, ok);
        if (ok) nnlc = link[node2];
      }
    }

    // step t at (x, y)
    T pf[9], pg[5], inf[9], ing[5];
    if (lc != NOT_FLUID) {
      collide_node<T, false, FluxT<T>>(L, x, y, lc, SEG, ph1, f, g, pf, pg, inf, ing, fx, own);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) pf[i] = inf[i] = T(0);
#pragma unroll
      for (int i = 0; i < 5; ++i) pg[i] = ing[i] = T(0);
    }
    // populations that change column on their way (every lane takes part)
    const T zf1 = from_left(pf[1]), zf3 = from_right(pf[3]);
    const T zg1 = from_left(pg[1]), zg3 = from_right(pg[3]);
    const T vf5 = from_left(pf[5]), vf6 = from_right(pf[6]);
    const T df7 = from_right(pf[7]), df8 = from_left(pf[8]);

    // (each collision's fluxes leave on their own, as a single step's do;
    // every lane of the wavefront takes part)
    if (SEG) fx.flush((double *)L.flux);
    // the previous row pulls f4, f7, f8, g4 from this row: step t + 1 there
    if (own_prev && lcp != NOT_FLUID) {
      if (!src_solid(lcp, 4)) sf[4] = P::rt(pf[4]);
      if (!src_solid(lcp, 7)) sf[7] = P::rt(df7);
      if (!src_solid(lcp, 8)) sf[8] = P::rt(df8);
      if (!src_solid(lcp, 4)) sg[4] = P::rt(pg[4]);
      second_step<S, SEG, false, FluxT<T>>(L, dst, x, yprev, lcp, ph2, sf, sg, fx);
    }

    // state at t + 1 of this row, without the pulls from the row below
    if (lc != NOT_FLUID) {
      sf[0] = P::rt(pf[0]);
      sg[0] = P::rt(pg[0]);
      sf[1] = P::rt(src_solid(lc, 1) ? inf[1] : zf1);
      sf[3] = P::rt(src_solid(lc, 3) ? inf[3] : zf3);
      sg[1] = P::rt(src_solid(lc, 1) ? ing[1] : zg1);
      sg[3] = P::rt(src_solid(lc, 3) ? ing[3] : zg3);
      sf[2] = P::rt(src_solid(lc, 2) ? inf[2] : uf2);
      sf[5] = P::rt(src_solid(lc, 5) ? inf[5] : uf5);
      sf[6] = P::rt(src_solid(lc, 6) ? inf[6] : uf6);
      sg[2] = P::rt(src_solid(lc, 2) ? ing[2] : ug2);
      sf[4] = P::rt(inf[4]);
      sf[7] = P::rt(inf[7]);
      sf[8] = P::rt(inf[8]);
      sg[4] = P::rt(ing[4]);
    }
    uf2 = pf[2];
    uf5 = vf5;
    uf6 = vf6;
    ug2 = pg[2];
    lcp = lc;
    yprev = y;
    own_prev = own;
    if (SEG) fx.flush((double *)L.flux);
  }
}


// Two steps over a strip list: 256-thread work-groups, one strip per
// wavefront. Work-groups are dealt to the 8 XCDs so that each XCD walks a
// contiguous run of strips (the list runs along each band of rows, so
// neighbouring strips, which share cache lines at their edges, share an L2).
// SEG: strips with links to boundary segments (their own kernel, so that
// the boundary rules do not set the register budget of the others).
template <class S, bool SEG, bool PAIRS>
__global__ void __launch_bounds__(256)
    k_step2(const LatDesc *__restrict__ descs, const Tile *__restrict__ strips, int n_strips,
            int per_xcd, int dir, int dt) {
  const int nb = 8 * per_xcd;
  // the wavefront index, marked uniform so that the strip, the descriptor
  // and the plane bases are read with scalar loads
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int s = ((b & 7) * per_xcd + (b >> 3)) * 4 + w;
    if (s < n_strips) strip_two_steps<S, SEG, PAIRS>(descs, strips, s, dir, dt);
  }
}

// Row-parallel form of the same two steps, for lattices too small to keep
// the GPU busy with walking strips: one work-group per tile of 62 columns x
// R rows (at most; the row count is in the tile flags), R + 2 wavefronts,
// wavefront w on lattice row y0 - 1 + w. Every wavefront does step t on its
// row; the populations that cross rows (f2, f5, f6, g2 up; f4, f7, f8, g4
// down) go through LDS; after one barrier the owned rows do step t + 1.
// PRESS (segment tiles of lattices with pressure segments): the pressure
// rule at the links, and the rescaling (Eq. 10) of the state at t + 1 of a
// node next to an open pressure segment, in registers between the two
// steps, as the rescaling kernel does it in memory after a single step.
// With bit 1 of dir set, the state at t as loaded is taken as not yet
// rescaled after step t - 1 and every row of the tile, halo included,
// rescales it first in the same way; the caller then marks as segment tiles
// all tiles whose rows or halo hold a node next to a segment. Otherwise the
// rescaling kernel runs after the pass.
// TAPE (the adjoint's recomputation): also write each owned node's state
// before each of the two steps, dg_0..4 then u_x, u_y (from the same
// moments as the collision), to the planes of the compute type at tape0
// (step t) and tape1 (step t + 1), as the single step's tape does.
template <class S, bool SEG, int R, bool PRESS, bool TAPE, bool PAIRS>
__global__ void __launch_bounds__((R + 2) * 64)
    k_tile2(const LatDesc *__restrict__ descs, const Tile *__restrict__ tiles, int n_tiles,
            int per_xcd, int dir, int dt, void *__restrict__ tape0, void *__restrict__ tape1) {
  using P = Pop<S>;
  using T = typename P::T;
  using W = typename P::W;
  __shared__ T lds_up[R + 2][4][64];
  __shared__ T lds_dn[R + 2][4][64];
  const int lane = (int)(threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nb = 8 * per_xcd;
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile >= n_tiles) continue;  // the same for the whole work-group
    const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
    CDesc &L = ((CDesc *)descs)[tl.inst];
    const int nx = L.nx, ny = L.ny, pitch = L.pitch;
    const int rows = strip_rows(tl.flags);
    const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
    // with SEG, the tiles without segment links skip the boundary rules
    const bool seg = SEG && (tl.flags & TILE_TOUCHES_SEGMENT) != 0;
    PhaseNow ph1{0u, nullptr}, ph2{0u, nullptr};
    if (seg) {
      ph1 = phase_at(L, t);
      ph2 = phase_at(L, t + 1);
    }
    const int dsel = PRESS ? (dir & 1) : dir;
    // (the layout is the lattice's, PAIRS: known at compile time)
    const Planes<W> src(dsel ? L.pop_b : L.pop, L.plane, PAIRS);
    const Planes<W> dst(dsel ? L.pop : L.pop_b, L.plane, PAIRS);

    const int xr = tl.x0 - 1 + lane;
    const bool col = xr >= -1 && xr <= nx;
    int x = xr;
    if (L.periodic_x) x = xr < 0 ? xr + nx : (xr >= nx ? xr - nx : xr);
    const bool own_col = lane >= 1 && lane <= STRIP_W && xr >= 0 && xr < nx;
    const int yr = tl.y0 - 1 + w;
    int y = yr;
    if (L.periodic_y) y = yr < 0 ? yr + ny : (yr >= ny ? yr - ny : yr);
    const bool row = yr >= -1 && yr <= ny && w <= rows + 1;
    const bool own = own_col && w >= 1 && w <= rows && yr < ny;
    const uint32_t node = (uint32_t)(L.node0 + y * pitch + x);
    // every load of the row is issued at once, by every lane: the link code
    // and the populations of any addressable cell (non-fluid cells hold
    // finite values nobody uses; lanes off the addressable cells read node
    // (0, 0) and take the link code of a non-fluid cell), and on segment
    // tiles the neighbours' mask values
    const bool live = row && col;
    const uint32_t lnode = live ? node : (uint32_t)L.node0;
    const uint8_t lc = live ? ((const GG_GLOBAL uint8_t *)L.link)[lnode] : NOT_FLUID;
    T f[9], g[5];
    if (src.pairs) {  // (uniform) f_i and g_i in one access
#pragma unroll
      for (int i = 0; i < 5; ++i) P::ld_pair(src.at(i, lnode), f[i], g[i]);
#pragma unroll
      for (int i = 5; i < 9; ++i) f[i] = P::ld(src.at(i, lnode));
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = P::ld(src.at(i, lnode));
#pragma unroll
      for (int i = 0; i < 5; ++i) g[i] = P::ld(src.at(9 + i, lnode));
    }
    uint32_t nbr[2] = {0u, 0u};
    // (only for cells inside the lattice, whose neighbours all lie in the
    // padded planes; the halo cells outside are not fluid)
    if (seg && live && x >= 0 && x < nx && y >= 0 && y < ny) {
      const Neigh nb(L, x, y);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        nbr[k >> 2] |= (uint32_t)((const GG_GLOBAL uint8_t *)L.mask)[nb.idx[k + 1]] << (8 * (k & 3));
    }

    // step t on this row (the boundary fluxes of the tile's two steps summed
    // per lane in the compute type)
    // Boundary fluxes: each collision's terms summed per lane in the compute
    // type (fx) and each rescaling's term in FP64 (fr), as the single steps
    // and the rescaling kernel sum them
    FluxT<T> fx;
    Flux fr;
    if (PRESS && seg && (dir & 2) && lc != NOT_FLUID && lc != 0) {
      // the rescaling after step t - 1 (the flux counted once, by the owner)
      const PhaseNow ph0 = phase_at(L, t - 1);
      const int ps = pressure_source(L, lc, ph0, nbr);
      if (ps >= 0) {
        double dm, dc;
        rescale_node<T>(L, ps, ph0, true, f, g, dm, dc);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = P::rt(f[i]);
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = P::rt(g[i]);
        if (own) fr.add(ps, dm, dc);
      }
    }
    if (TAPE && own && lc != NOT_FLUID) {
      T rho, drho, ux, uy;
      node_velocity<T>(L, f, rho, drho, ux, uy);
      const TapePlanes<T> tp(tape0, L.plane);
#pragma unroll
      for (int i = 0; i < 5; ++i) *tp.at(i, node) = g[i];
      *tp.at(5, node) = ux;
      *tp.at(6, node) = uy;
    }
    // step t on every lane of the interior tiles (what a non-fluid lane
    // computes is never taken: its neighbours take their link rule's value
    // instead), on the fluid lanes of the segment tiles
    T pf[9], pg[5], inf[9], ing[5];
    if (!SEG || lc != NOT_FLUID) {
      collide_node<T, PRESS, FluxT<T>>(L, x, y, lc, seg, ph1, f, g, pf, pg, inf, ing, fx, own,
                                       SEG ? nbr : nullptr);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) pf[i] = inf[i] = T(0);
#pragma unroll
      for (int i = 0; i < 5; ++i) pg[i] = ing[i] = T(0);
    }
    const T zf1 = from_left(pf[1]), zf3 = from_right(pf[3]);
    const T zg1 = from_left(pg[1]), zg3 = from_right(pg[3]);
    lds_up[w][0][lane] = pf[2];
    lds_up[w][1][lane] = from_left(pf[5]);
    lds_up[w][2][lane] = from_right(pf[6]);
    lds_up[w][3][lane] = pg[2];
    lds_dn[w][0][lane] = pf[4];
    lds_dn[w][1][lane] = from_right(pf[7]);
    lds_dn[w][2][lane] = from_left(pf[8]);
    lds_dn[w][3][lane] = pg[4];
    // (the first step's fluxes leave before the barrier: the accumulators
    // are not held across it)
    if (seg) {
      fx.flush((double *)L.flux);
      if (PRESS) fr.flush((double *)L.flux);
    }
    __syncthreads();

    // step t + 1 on the owned rows
    if (own && lc != NOT_FLUID) {
      T sf[9], sg[5];
      // the pulled values (read unconditionally, so that the LDS reads are
      // issued together rather than one by one behind the selects below)
      sf[0] = pf[0];
      sg[0] = pg[0];
      sf[1] = zf1;
      sf[3] = zf3;
      sg[1] = zg1;
      sg[3] = zg3;
      sf[2] = lds_up[w - 1][0][lane];
      sf[5] = lds_up[w - 1][1][lane];
      sf[6] = lds_up[w - 1][2][lane];
      sg[2] = lds_up[w - 1][3][lane];
      sf[4] = lds_dn[w + 1][0][lane];
      sf[7] = lds_dn[w + 1][1][lane];
      sf[8] = lds_dn[w + 1][2][lane];
      sg[4] = lds_dn[w + 1][3][lane];
      // where x - e_j is not fluid, the value from the link rule instead
      // (skipped when no lane of the wavefront has such a link)
      if (__any(lc != 0)) {
#pragma unroll
        for (int j = 1; j < 9; ++j)
          if (src_solid(lc, j)) sf[j] = inf[j];
#pragma unroll
        for (int j = 1; j < 5; ++j)
          if (src_solid(lc, j)) sg[j] = ing[j];
      }
      // rounded to the storage type (in pairs)
      P::rt2(sf[0], sg[0]);
#pragma unroll
      for (int j = 1; j < 9; j += 2) P::rt2(sf[j], sf[j + 1]);
#pragma unroll
      for (int j = 1; j < 5; j += 2) P::rt2(sg[j], sg[j + 1]);
      if (PRESS && seg) {
        const int ps = pressure_source(L, lc, ph1, nbr);
        if (ps >= 0) {
          double dm, dc;
          rescale_node<T>(L, ps, ph1, true, sf, sg, dm, dc);
#pragma unroll
          for (int i = 0; i < 9; ++i) sf[i] = P::rt(sf[i]);
#pragma unroll
          for (int i = 0; i < 5; ++i) sg[i] = P::rt(sg[i]);
          fr.add(ps, dm, dc);
        }
      }
      if (TAPE) {
        T rho, drho, ux, uy;
        node_velocity<T>(L, sf, rho, drho, ux, uy);
        const TapePlanes<T> tp(tape1, L.plane);
#pragma unroll
        for (int i = 0; i < 5; ++i) *tp.at(i, node) = sg[i];
        *tp.at(5, node) = ux;
        *tp.at(6, node) = uy;
      }
      if (seg)
        second_step<S, true, PRESS, FluxT<T>>(L, dst, x, y, lc, ph2, sf, sg, fx, nbr);
      else
        second_step<S, false, false, FluxT<T>>(L, dst, x, y, lc, ph2, sf, sg, fx);
    }
    if (seg) {
      fx.flush((double *)L.flux);
      if (PRESS) fr.flush((double *)L.flux);
    }
    __syncthreads();  // the LDS rows are reused by the next tile
  }
}

// Four coupled steps in one pass over memory: tiles of 58 columns x R rows,
// R + 6 wavefronts (wavefront w on lattice row y0 - 3 + w, its 64 lanes on
// the columns x0 - 3 .. x0 + 60). Step t runs on every row and column of
// the tile and its three-node halo; the populations of each step's result
// that cross columns go through lane shifts, those that cross rows through
// LDS (two buffers, alternating), so that steps t + 1 and t + 2 run on the
// rows and columns whose state they can complete (a node fewer on each side
// per step), and step t + 3 on the owned nodes, stored into the
// neighbours' slots of the other plane set as the two-step pass stores its
// second step. Each collision goes through collide_node with the inputs the
// single steps give it (the state between steps rounded to the storage
// type), so the pass leaves what four single steps leave. SEG: the tiles
// with a segment link among the nodes whose state at t + 1 or t + 2 they
// complete; the others skip the boundary rules.
template <class S, bool SEG, int R, bool PAIRS>
__global__ void __launch_bounds__((R + 6) * 64)
    k_tile4(const LatDesc *__restrict__ descs, const Tile *__restrict__ tiles, int n_tiles,
            int per_xcd, int dir, int dt) {
  using P = Pop<S>;
  using T = typename P::T;
  using W = typename P::W;
  constexpr int NW = R + 6;
  __shared__ T lds_up[2][NW][4][64];
  __shared__ T lds_dn[2][NW][4][64];
  const int lane = (int)(threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nb = 8 * per_xcd;
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile >= n_tiles) continue;  // the same for the whole work-group
    const GG_CONST Tile &tl = ((const GG_CONST Tile *)tiles)[tile];
    CDesc &L = ((CDesc *)descs)[tl.inst];
    const int nx = L.nx, ny = L.ny, pitch = L.pitch;
    const int rows = strip_rows(tl.flags);
    const int64_t t = *(const GG_CONST int64_t *)L.t + dt;
    const bool seg = SEG && (tl.flags & TILE_TOUCHES_SEGMENT) != 0;
    PhaseNow ph[4] = {{0u, nullptr}, {0u, nullptr}, {0u, nullptr}, {0u, nullptr}};
    if (seg) {
#pragma unroll
      for (int k = 0; k < 4; ++k) ph[k] = phase_at(L, t + k);
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
    const uint32_t node = (uint32_t)(L.node0 + y * pitch + x);
    const bool live = row && col;
    const uint32_t lnode = live ? node : (uint32_t)L.node0;
    const uint8_t lc = live ? ((const GG_GLOBAL uint8_t *)L.link)[lnode] : NOT_FLUID;
    T f[9], g[5];
    if (src.pairs) {
#pragma unroll
      for (int i = 0; i < 5; ++i) P::ld_pair(src.at(i, lnode), f[i], g[i]);
#pragma unroll
      for (int i = 5; i < 9; ++i) f[i] = P::ld(src.at(i, lnode));
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = P::ld(src.at(i, lnode));
#pragma unroll
      for (int i = 0; i < 5; ++i) g[i] = P::ld(src.at(9 + i, lnode));
    }
    uint32_t nbr[2] = {0u, 0u};
    if (seg && live && x >= 0 && x < nx && y >= 0 && y < ny) {
      const Neigh nb(L, x, y);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        nbr[k >> 2] |= (uint32_t)((const GG_GLOBAL uint8_t *)L.mask)[nb.idx[k + 1]] << (8 * (k & 3));
    }
    FluxT<T> fx;
    T pf[9], pg[5], inf[9], ing[5];
    if (!SEG || lc != NOT_FLUID) {
      collide_node<T, false, FluxT<T>>(L, x, y, lc, seg, ph[0], f, g, pf, pg, inf, ing, fx, own,
                                       SEG ? nbr : nullptr);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) pf[i] = inf[i] = T(0);
#pragma unroll
      for (int i = 0; i < 5; ++i) pg[i] = ing[i] = T(0);
    }
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      const int q = (k - 1) & 1;
      const T zf1 = from_left(pf[1]), zf3 = from_right(pf[3]);
      const T zg1 = from_left(pg[1]), zg3 = from_right(pg[3]);
      lds_up[q][w][0][lane] = pf[2];
      lds_up[q][w][1][lane] = from_left(pf[5]);
      lds_up[q][w][2][lane] = from_right(pf[6]);
      lds_up[q][w][3][lane] = pg[2];
      lds_dn[q][w][0][lane] = pf[4];
      lds_dn[q][w][1][lane] = from_right(pf[7]);
      lds_dn[q][w][2][lane] = from_left(pf[8]);
      lds_dn[q][w][3][lane] = pg[4];
      if (seg) fx.flush((double *)L.flux);
      __syncthreads();
      // rows whose state at t + k is needed (wave-uniform)
      const bool act = w >= k && w < NW - k;
      const bool run = k < 3 ? act && (!SEG || lc != NOT_FLUID) : own && lc != NOT_FLUID;
      if (run) {
        T sf[9], sg[5];
        sf[0] = pf[0];
        sg[0] = pg[0];
        sf[1] = zf1;
        sf[3] = zf3;
        sg[1] = zg1;
        sg[3] = zg3;
        sf[2] = lds_up[q][w - 1][0][lane];
        sf[5] = lds_up[q][w - 1][1][lane];
        sf[6] = lds_up[q][w - 1][2][lane];
        sg[2] = lds_up[q][w - 1][3][lane];
        sf[4] = lds_dn[q][w + 1][0][lane];
        sf[7] = lds_dn[q][w + 1][1][lane];
        sf[8] = lds_dn[q][w + 1][2][lane];
        sg[4] = lds_dn[q][w + 1][3][lane];
        if (__any(lc != 0)) {
#pragma unroll
          for (int j = 1; j < 9; ++j)
            if (src_solid(lc, j)) sf[j] = inf[j];
#pragma unroll
          for (int j = 1; j < 5; ++j)
            if (src_solid(lc, j)) sg[j] = ing[j];
        }
        P::rt2(sf[0], sg[0]);
#pragma unroll
        for (int j = 1; j < 9; j += 2) P::rt2(sf[j], sf[j + 1]);
#pragma unroll
        for (int j = 1; j < 5; j += 2) P::rt2(sg[j], sg[j + 1]);
        if (k < 3) {
          collide_node<T, false, FluxT<T>>(L, x, y, lc, seg, ph[k], sf, sg, pf, pg, inf, ing, fx,
                                           own, SEG ? nbr : nullptr);
        } else if (seg) {
          second_step<S, true, false, FluxT<T>>(L, dst, x, y, lc, ph[3], sf, sg, fx, nbr);
        } else {
          second_step<S, false, false, FluxT<T>>(L, dst, x, y, lc, ph[3], sf, sg, fx);
        }
      }
    }
    if (seg) fx.flush((double *)L.flux);
    __syncthreads();  // the LDS rows are reused by the next tile
  }
}

template <class S, bool PAIRS>
static void tile4_launch(bool seg, int grid, hipStream_t st, const LatDesc *d, const Tile *tiles,
                         int n_tiles, int per_xcd, int dir, int dt) {
  if (seg)
    k_tile4<S, true, 2, PAIRS><<<grid, 8 * 64, 0, st>>>(d, tiles, n_tiles, per_xcd, dir, dt);
  else
    k_tile4<S, false, 6, PAIRS><<<grid, 12 * 64, 0, st>>>(d, tiles, n_tiles, per_xcd, dir, dt);
}

}  // namespace

hipError_t launch_step2(gg_storage s, bool pairs, bool seg, const LatDesc *d, const Tile *strips,
                        int n_strips, int dir, int dt, hipStream_t st, int persist) {
  if (n_strips <= 0) return hipSuccess;
  const int nblk = (n_strips + 3) / 4;
  const int per_xcd = (nblk + 7) / 8;
  int grid = 8 * per_xcd;
  if (persist > 0) grid = std::min(grid, (persist + 7) / 8 * 8);
#define GG_LAUNCH2(TYPE, SEGV)                                                              \
  (pairs ? k_step2<TYPE, SEGV, true><<<grid, 256, 0, st>>>(d, strips, n_strips, per_xcd, dir, dt) \
         : k_step2<TYPE, SEGV, false><<<grid, 256, 0, st>>>(d, strips, n_strips, per_xcd, dir, dt))
  switch (s) {
    case GG_F64: if (seg) GG_LAUNCH2(double, true); else GG_LAUNCH2(double, false); break;
    case GG_F32: if (seg) GG_LAUNCH2(float, true); else GG_LAUNCH2(float, false); break;
    case GG_F16_SHIFTED: if (seg) GG_LAUNCH2(__half, true); else GG_LAUNCH2(__half, false); break;
  }
#undef GG_LAUNCH2
  return hipGetLastError();
}

template <class S, bool PAIRS>
static void tile2_launch(bool seg, int rows, bool press, bool tape, int grid, hipStream_t st,
                         const LatDesc *d, const Tile *tiles, int n_tiles, int per_xcd, int dir,
                         int dt, void *tape0, void *tape1) {
#define GG_T2(SEGV, RV, PV, TV)                                                              \
  k_tile2<S, SEGV, RV, PV, TV, PAIRS><<<grid, ((RV) + 2) * 64, 0, st>>>(d, tiles, n_tiles,   \
                                                                     per_xcd, dir, dt, tape0, \
                                                                     tape1)
  if (tape) {  // the adjoint's recomputation (no pressure segments)
    if (seg && rows <= 2) GG_T2(true, 2, false, true);
    else if (seg && rows <= 6) GG_T2(true, 6, false, true);
    else if (seg) GG_T2(true, 14, false, true);
    else if (rows <= 6) GG_T2(false, 6, false, true);
    else GG_T2(false, 14, false, true);
  } else if (seg && press) {
    if (rows <= 2) GG_T2(true, 2, true, false);
    else if (rows <= 6) GG_T2(true, 6, true, false);
    else GG_T2(true, 14, true, false);
  } else if (seg) {
    if (rows <= 2) GG_T2(true, 2, false, false);
    else if (rows <= 6) GG_T2(true, 6, false, false);
    else GG_T2(true, 14, false, false);
  } else {
    if (rows <= 6) GG_T2(false, 6, false, false);
    else GG_T2(false, 14, false, false);
  }
#undef GG_T2
}

hipError_t launch_tile2(gg_storage s, bool pairs, bool seg, int rows, const LatDesc *d,
                        const Tile *tiles, int n_tiles, int dir, int dt, hipStream_t st, bool press,
                        void *tape0, void *tape1) {
  if (n_tiles <= 0) return hipSuccess;
  const int per_xcd = (n_tiles + 7) / 8;
  const int grid = 8 * per_xcd;
  const bool tape = tape0 != nullptr;
#define GG_T2S(TYPE)                                                                        \
  (pairs ? tile2_launch<TYPE, true>(seg, rows, press, tape, grid, st, d, tiles, n_tiles,    \
                                     per_xcd, dir, dt, tape0, tape1)                        \
         : tile2_launch<TYPE, false>(seg, rows, press, tape, grid, st, d, tiles, n_tiles,   \
                                      per_xcd, dir, dt, tape0, tape1))
  switch (s) {
    case GG_F64: GG_T2S(double); break;
    case GG_F32: GG_T2S(float); break;
    case GG_F16_SHIFTED: GG_T2S(__half); break;
  }
#undef GG_T2S
  return hipGetLastError();
}

hipError_t launch_tile4(gg_storage s, bool pairs, bool seg, const LatDesc *d, const Tile *tiles,
                        int n_tiles, int dir, int dt, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  const int per_xcd = (n_tiles + 7) / 8;
  const int grid = 8 * per_xcd;
  switch (s) {
    case GG_F64:
      if (pairs) tile4_launch<double, true>(seg, grid, st, d, tiles, n_tiles, per_xcd, dir, dt);
      else tile4_launch<double, false>(seg, grid, st, d, tiles, n_tiles, per_xcd, dir, dt);
      break;
    case GG_F32:
      if (pairs) tile4_launch<float, true>(seg, grid, st, d, tiles, n_tiles, per_xcd, dir, dt);
      else tile4_launch<float, false>(seg, grid, st, d, tiles, n_tiles, per_xcd, dir, dt);
      break;
    case GG_F16_SHIFTED:
      if (pairs) tile4_launch<__half, true>(seg, grid, st, d, tiles, n_tiles, per_xcd, dir, dt);
      else tile4_launch<__half, false>(seg, grid, st, d, tiles, n_tiles, per_xcd, dir, dt);
      break;
  }
  return hipGetLastError();
}

}  // namespace gg
