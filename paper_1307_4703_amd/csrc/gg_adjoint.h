// Launch wrappers of the adjoint kernels, called by the host runtime.
#pragma once

#include "gg_device.h"

namespace gg {

// lam = weight (C - target) at every fluid node; per-tile loss partials.
hipError_t launch_seed(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                       int tx_shift, const double *weight, const double *target, void *lam,
                       double *partial, hipStream_t st);

// One adjoint step for step t: lam_in = dL/dg(t+1) -> lam_out = dL/dg(t),
// with the tape of step t (written by launch_step_tape: 7 planes g0..g4,
// ux, uy in the compute type); accumulates dL/dR on the box, dL/dC_in per
// segment and per-tile dL/domega_g partials.
hipError_t launch_adjoint(gg_storage s, const LatDesc *d, const Tile *tiles, int n_tiles,
                          int tx_shift, int64_t t, const void *lam_in, void *lam_out,
                          const void *tape, double *dR, const int32_t box[4], double *dcin,
                          double *partial, hipStream_t st);

// Two adjoint steps in one pass (steps t and t - 1): lam_in = dL/dg(t+1)
// -> lam_out = dL/dg(t-1), with the tapes of both steps, over the tiles of
// the two-step pass (62 columns x rows, one-node halo; segment flag set
// where the tile or its halo touches a segment); partials per tile.
hipError_t launch_adjoint2(gg_storage s, int rows, const LatDesc *d, const Tile *tiles, int n_tiles,
                           int64_t t, const void *lam_in, void *lam_out, const void *tape_t,
                           const void *tape_tm1, double *dR, const int32_t box[4], double *dcin,
                           double *partial, hipStream_t st);

}  // namespace gg
