// Host-side lattice object shared by the runtime translation units.
#pragma once

#include <string>
#include <vector>

#include "gg_device.h"

struct SegHost {
  bool set = false;
  int kind = 0;
  int nrm_x = 0, nrm_y = 0;
  double u_max = 0.0, c_in = 0.0;
  double rho = 1.0;    // pressure segments: density held
  bool hold_c = false; // pressure segments: compound held at c_in
  double s0 = 0.0, s1 = 1.0;  // halfway-wall tangential coordinates
};

struct gg_lattice {
  gg_alloc alloc{};         // the caller's device allocator (has_alloc)
  bool has_alloc = false;
  int32_t nx = 0, ny = 0, pitch = 0, node0 = 0;
  int64_t plane_elems = 0;  // addressable elements of one plane (with padding)
  int64_t plane = 0;        // stride between planes
  size_t nid(int x, int y) const { return (size_t)node0 + (size_t)y * pitch + x; }
  gg_storage storage = GG_F32;
  size_t esize = 4;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int device = 0;  // the HIP device current at creation (owns every buffer)
  gg_params p{};
  double tau_g = 0.0, cs2g = 0.0;
  std::vector<uint8_t> mask;         // nx*ny
  std::vector<uint8_t> link;         // link codes, plane layout
  std::vector<uint8_t> touches_seg;  // nx*ny: fluid node next to a segment
  int64_t n_fluid = 0;
  SegHost seg[GG_MAX_SEGMENTS];
  bool seg_present[GG_MAX_SEGMENTS] = {};
  std::vector<gg_phase> phases;
  int64_t t_origin = 0;
  int64_t t = 0;  // host mirror of the device counter
  // configuration generation: bumped by every call that re-uploads the
  // descriptor or frees or reallocates a device buffer it points to
  // (batches copy the descriptor and refuse to run once it changed)
  uint64_t gen = 0;
  int r_box[4] = {0, 0, 0, 0};

  void *d_pop = nullptr;
  void *d_pop_b = nullptr;  // second plane set of the two-step pass
  uint8_t *d_link = nullptr, *d_mask = nullptr, *d_region = nullptr;
  double *d_R = nullptr;
  int64_t *d_t = nullptr;
  double *d_flux = nullptr, *d_acc = nullptr;
  double *d_partial = nullptr;  // per-tile partials of the diagnostics
  gg::LatDesc *d_desc = nullptr;
  gg::LatDesc h{};
  gg::Tile *d_tiles = nullptr;
  int n_tiles = 0, tile_x = 64, tile_y = 4;
  gg::Tile *d_aux_tiles = nullptr;
  int n_aux_tiles = 0;
  int graph_chunk = 64;
  // two-step pass: fuse = 2, 3, 4 advance pairs of steps in one pass over
  // memory (walking strips of 62 columns x strip_h rows, or row-parallel
  // tiles of strip_h rows with the boundary kernel apart or in one kernel);
  // fuse = 5 runs runs of eight steps in four-step passes (58 x 6 tiles,
  // the boundary kernel apart) and other runs as fuse = 3; fuse = 1 keeps
  // to single steps
  int fuse = 3, strip_h = 6;
  // population layout: paired (f_i, g_i side by side, i = 0..4) or
  // plane-major (gg_set_layout)
  bool pairs = true;
  // tile lists built with the halo-inclusive segment flag (pressure
  // segments: the passes rescale the boundary nodes as they load them)
  bool tiles_halo_seg = false, cde_halo_seg = false;
  bool strip_flux_ok = true;  // no vertical node pair links to > 2 segments
  gg::Tile *d_strips = nullptr;      // strips without segment links
  int n_strips = 0;
  gg::Tile *d_seg_strips = nullptr;  // strips with segment links (2 rows each)
  int n_seg_strips = 0;
  // the segment strips run beside the others: forked onto a side stream and
  // joined back every pass (also inside captured graphs)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // fluid nodes with a link from a pressure segment's ghost cell, as (x, y)
  // pairs, rescaled after every step; rebuilt when the segments change
  int32_t *d_press = nullptr;
  int n_press = 0;
  bool press_dirty = true;
  // the paper's walls (wall_scheme 1): fluid nodes with a link from a wall
  // or a segment's ghost cell, as (x, y) pairs, and the values of step t
  // their rule needs (saved before each step)
  int wall_scheme = 0;
  int32_t *d_wall = nullptr;
  int n_wall = 0;
  int32_t *d_wall_links = nullptr;  // (x, y, k * 8 + (i - 1)): node k, link from x - e_i
  int n_wall_links = 0;
  void *d_wall_save = nullptr;
  bool wall_dirty = true;
  // compound alone on frozen velocity fields: n_ufield slots of two planes
  // (u_x, u_y) in the compute type; bit k of ufield_set: slot k written;
  // phase_field[k]: slot used in schedule phase k; graphs of graph_chunk
  // compound-only steps from an even / odd t
  void *d_ufield = nullptr;
  int n_ufield = 0;
  uint32_t ufield_set = 0;
  int8_t phase_field[GG_MAX_PHASES] = {};
  // compound-only steps in two-step passes over tiles of cde_rows rows (6 or
  // 14; 0: single steps only), or in four-step passes over 58-column tiles
  // of -cde_rows rows (-6 or -10; other runs in two-step passes of 6-row
  // tiles); the tile lists are built on first use
  int cde_rows = 14;
  gg::Tile *d_cde_tiles = nullptr, *d_cde_tiles4 = nullptr;
  int n_cde_tiles = 0, n_cde_tiles4 = 0, cde_tiles_rows = 0;
  hipGraph_t cde_graph[2] = {nullptr, nullptr};
  hipGraphExec_t cde_exec[2] = {nullptr, nullptr};
  // fluid nodes owned by the tiles of the pass's two lists
  int64_t strips_fluid = 0, seg_strips_fluid = 0;
  // the four-step pass's lists (fuse = 5 where the lattice allows it: no
  // pressure segments, periodic axes of 4 nodes or more)
  gg::Tile *d_strips4 = nullptr, *d_seg_strips4 = nullptr;
  int n_strips4 = 0, n_seg_strips4 = 0;
  int64_t strips4_fluid = 0, seg_strips4_fluid = 0;
  bool tiles4 = false;  // the lists were built (pass4_ok held)
  // monitor: the FP64 reduction of gg_diagnostics launched after every
  // mon_every-th step (counted from mon_t0) into d_mon (8 totals, then the
  // 2 * GG_MAX_SEGMENTS flux accumulators copied at the same point)
  int64_t mon_every = 0, mon_t0 = 0, mon_last_t = -1, mon_count = 0;
  double *d_mon = nullptr;
  // profiling (gg_step_profile): plain launches with an event pair around
  // every launch of the dominant kernel; kind 0 pass, 1 even step, 2 odd
  // step, 3 graph replay, 4 two-step pass beside the four-step pass
  bool prof = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int8_t> prof_kind;
  size_t prof_used = 0;
};

gg_status gg_upload_desc(gg_lattice *L);
// Record msg as this thread's last error and return s.
gg_status gg_fail(gg_status s, const std::string &msg);
// gg_diag from the reduction totals acc[0..5] and the flux accumulators.
void gg_fill_diag(const gg_lattice *L, const double *acc, const double *flux, int64_t t,
                  gg_diag *out);
gg_status gg_rebuild_tiles(gg_lattice *L);
void gg_free_device(gg_lattice *L);
void gg_drop_cde_graphs(gg_lattice *L);
