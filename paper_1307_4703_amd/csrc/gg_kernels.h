// Launch wrappers of the gfx950 kernels, called by the host runtime.
#pragma once

#include "gg_device.h"

namespace gg {

// Fused coupled step over a tile list; block = threads per work-group
// (64, 128, 256 or 512), tile width 1 << tx_shift, odd = parity of the
// step, dt added to the device step counter of each lattice. persist > 0
// caps the grid at that many work-groups (rounded up to a multiple of 8),
// which then stride through the tiles.
hipError_t launch_step(gg_storage s, bool pairs, int block, bool odd, const LatDesc *d,
                       const Tile *tiles, int n_tiles, int tx_shift, int dt, hipStream_t st,
                       int persist = 0);
// launch_step that also writes, for each fluid node, the state before the
// step to `tape` (compute type, plane stride of the populations: dg_0..4,
// u_x, u_y), the adjoint's tape.
hipError_t launch_step_tape(gg_storage s, bool pairs, int block, bool odd, const LatDesc *d,
                            const Tile *tiles, int n_tiles, int tx_shift, int dt, void *tape,
                            hipStream_t st);

// Two steps in one pass (t even, natural order in): strips of 62 columns x
// (flags >> 8) rows, four per 256-thread work-group; seg selects the kernel
// for strips with segment links; dir 0 reads the plane set pop and writes
// pop_b, dir 1 the reverse; dt as for launch_step.
hipError_t launch_step2(gg_storage s, bool pairs, bool seg, const LatDesc *d, const Tile *strips,
                        int n_strips, int dir, int dt, hipStream_t st, int persist = 0);

// The same two steps row-parallel: one work-group of rows + 2 wavefronts
// per tile of 62 columns x (flags >> 8) rows, rows 2, 6 or 14; seg selects
// the kernel that also carries the boundary rules (applied to the tiles
// whose segment bit is set); press (with seg): the lattice has pressure
// segments, whose link rule and first rescaling the pass then applies (the
// rescaling of the state after the pass is launch_rescale's). tape0,
// tape1 (the adjoint's recomputation, no pressure segments): tape slots of
// the pass's two steps, written for the tiles' owned nodes.
// pairs: the tiles' lattices hold their populations in the paired layout
// (all of them, or none).
hipError_t launch_tile2(gg_storage s, bool pairs, bool seg, int rows, const LatDesc *d,
                        const Tile *tiles, int n_tiles, int dir, int dt, hipStream_t st,
                        bool press = false, void *tape0 = nullptr, void *tape1 = nullptr);

// Four steps in one pass (t even, natural order in and out): one work-group
// of rows + 6 wavefronts per tile of 58 columns x (flags >> 8) rows, rows 2
// (seg, the boundary kernel) or 6; no pressure segments; dir and dt as for
// launch_tile2.
hipError_t launch_tile4(gg_storage s, bool pairs, bool seg, const LatDesc *d, const Tile *tiles,
                        int n_tiles, int dir, int dt, hipStream_t st);

// Compound-only step on frozen velocity fields (64 x 4 tiles, 256-thread
// work-groups, XCD-aware tile order as launch_step); odd = parity of the
// step, dt as for launch_step.
hipError_t launch_cde(gg_storage s, bool pairs, bool odd, const LatDesc *d, const Tile *tiles,
                      int n_tiles, int tx_shift, int dt, hipStream_t st);
// Two compound-only steps in one pass (t even, natural order in): one
// work-group of rows + 2 wavefronts per tile of 62 columns x (flags >> 8)
// rows, rows 6 or 14; dir 0 reads the compound planes of pop and writes
// those of pop_b, dir 1 the reverse; dt as for launch_step; press: the
// lattice has pressure segments (their link rule and first rescaling in the
// pass; launch_rescale after it).
hipError_t launch_cde_tile2(gg_storage s, bool pairs, int rows, const LatDesc *d,
                            const Tile *tiles, int n_tiles, int dir, int dt, hipStream_t st,
                            bool press = false);
// Four compound-only steps per pass (t even, no pressure segments): one
// work-group of rows + 6 wavefronts per tile of 58 columns x (flags >> 8)
// rows, rows 6 or 10; dir and dt as for launch_tile2.
hipError_t launch_cde_tile4(gg_storage s, bool pairs, int rows, const LatDesc *d,
                            const Tile *tiles, int n_tiles, int dir, int dt, hipStream_t st);
// Velocity of the current fluid state times `scale` into field slot `slot`.
hipError_t launch_capture(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                          int tx_shift, int slot, double scale, hipStream_t st);
// FP64 fields scale * ux, scale * uy (device, y * nx + x) into slot `slot`.
hipError_t launch_put_field(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                            int tx_shift, int slot, const double *ux, const double *uy,
                            double scale, hipStream_t st);

// The paper's walls for the n nodes listed as (x, y) pairs and their
// n_links links from non-fluid cells, entries (x, y, k * 8 + (i - 1)) (node
// k of the list at (x, y), direction i): before step (device counter + dt), save what the
// rule needs of that step (16 values of the compute type per node) into
// `save`; after it, write the links' values where the source is a wall at
// the step's phase; fluid = false: the compound-only step (frozen field).
hipError_t launch_wall_save(gg_storage s, const LatDesc *d, const int32_t *xy, int n,
                            const int32_t *links, int n_links, int dt, bool fluid, void *save,
                            hipStream_t st);
hipError_t launch_wall_apply(gg_storage s, const LatDesc *d, const int32_t *links, int n_links,
                             int dt, const void *save, bool fluid, hipStream_t st);

// Auxiliary kernels: 256-thread work-groups over one lattice's tiles.
// Population planes (n elements per plane, plane elements apart) from one
// layout into the other (pairs: the paired layout of Planes), src into dst
// (distinct buffers).
hipError_t launch_relayout(gg_storage s, void *src, void *dst, int64_t plane, int64_t n,
                           bool from_pairs, bool to_pairs, hipStream_t st);

hipError_t launch_init(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                       int tx_shift, const double *rho, const double *ux,
                       const double *uy, const double *c, hipStream_t st);
hipError_t launch_read(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                       int tx_shift, double *rho, double *ux, double *uy, double *c,
                       double *f, double *g, hipStream_t st);
// FP64 diagnostics into acc[0..5] (mass, solute, max|u|, region max|u|,
// non-finite count, fluid count) through partial[6 * groups], groups =
// n_tiles (one work-group per tile) or, with max_groups > 0, at most
// max_groups work-groups that each fold every groups-th tile. Every partial
// and acc[0..5] are written, nothing needs clearing beforehand.
hipError_t launch_reduce(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                         int tx_shift, double *partial, double *acc, hipStream_t st,
                         int max_groups = 0);
// The work-groups of every diagnostics reduction (gg_diagnostics, the
// monitor and the allocation-free form alike, so that all three sum in the
// same order): enough to keep the GPU's memory busy, few enough that the
// final fold of the partial records takes one short work-group.
constexpr int REDUCE_GROUPS = 2048;
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st);
// Pressure boundary: after step (device counter + dt), rescale the state at
// t + 1 of the n nodes listed as (x, y, candidates) triples that take a
// boundary value from an open pressure segment (candidates: the pressure
// segments among the node's source cells, one byte each, index + 1, in
// order of first appearance in direction order); fluid = false rescales the
// compound only; other: the state is in the second plane set (after a
// two-step pass).
hipError_t launch_rescale(gg_storage s, const LatDesc *d, const int32_t *xy, int n, int dt,
                          bool fluid, hipStream_t st, bool other = false);
hipError_t launch_advance(const LatDesc *descs, int n, int64_t k, hipStream_t st);
// *t = v on the stream.
hipError_t launch_set_counter(int64_t *t, int64_t v, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st);

}  // namespace gg
