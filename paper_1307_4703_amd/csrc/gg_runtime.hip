// Host runtime behind the C ABI of include/gg.h: geometry classification,
// boundary segments, valve schedule, device memory, launches and graphs.
#include <algorithm>
#include <random>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gg_adjoint.h"
#include "gg_device.h"
#include "gg_kernels.h"
#include "gg_runtime.h"

using namespace gg;

namespace {

thread_local std::string g_err;

gg_status fail(gg_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

#define GG_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(GG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t storage_bytes(gg_storage s) {
  switch (s) {
    case GG_F64: return 8;
    case GG_F32: return 4;
    case GG_F16_SHIFTED: return 2;
  }
  return 0;
}

int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

// Device memory of a lattice: from the caller's allocator when one was
// given to gg_create_ex, else hipMalloc / hipFree. Memory goes back to the
// caller's allocator only after the device is idle (as hipFree waits), so
// no queued kernel still uses it when the allocator hands it out again.
hipError_t dev_alloc(const gg_lattice *L, void **p, size_t bytes) {
  if (!L->has_alloc) return hipMalloc(p, bytes);
  *p = bytes ? L->alloc.alloc(bytes, L->alloc.ctx) : nullptr;
  return (*p || !bytes) ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t dev_free(const gg_lattice *L, void *p) {
  if (!p) return hipSuccess;
  if (!L->has_alloc) return hipFree(p);
  const hipError_t e = hipDeviceSynchronize();
  L->alloc.release(p, L->alloc.ctx);
  return e;
}

}  // namespace

gg_status gg_fail(gg_status s, const std::string &msg) { return fail(s, msg); }

void gg_fill_diag(const gg_lattice *L, const double *acc, const double *flux, int64_t t,
                  gg_diag *out) {
  std::memset(out, 0, sizeof(*out));
  out->t = t;
  out->n_fluid = L->n_fluid;
  out->n_nonfinite = (int64_t)acc[4];
  out->mass = acc[0];
  out->solute = acc[1];
  out->max_u = acc[2];
  out->max_u_region = acc[3];
  out->max_pe_region = acc[3] / L->p.D;
  for (int s = 0; s < GG_MAX_SEGMENTS; ++s) {
    out->seg_mass[s] = flux[2 * s];
    out->seg_solute[s] = flux[2 * s + 1];
    if (!L->seg[s].set) continue;
    if (L->seg[s].kind == GG_SEG_INLET) {
      out->mass_in += flux[2 * s];
      out->solute_in += flux[2 * s + 1];
    } else {
      out->mass_out += flux[2 * s];
      out->solute_out += flux[2 * s + 1];
    }
  }
}


// ---------------------------------------------------------------------------
// Lattice object
// ---------------------------------------------------------------------------

void gg_drop_cde_graphs(gg_lattice *L) {
  for (int p = 0; p < 2; ++p) {
    if (L->cde_exec[p]) (void)hipGraphExecDestroy(L->cde_exec[p]);
    if (L->cde_graph[p]) (void)hipGraphDestroy(L->cde_graph[p]);
    L->cde_exec[p] = nullptr;
    L->cde_graph[p] = nullptr;
  }
}

void gg_free_device(gg_lattice *L) {
  gg_drop_cde_graphs(L);
  if (L->graph_exec) (void)hipGraphExecDestroy(L->graph_exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->graph_exec = nullptr;
  L->graph = nullptr;
  void *ptrs[] = {L->d_pop, L->d_pop_b, L->d_link, L->d_mask, L->d_region, L->d_R, L->d_t,
                  L->d_flux, L->d_acc, L->d_desc, L->d_tiles, L->d_aux_tiles, L->d_strips,
                  L->d_seg_strips, L->d_strips4, L->d_seg_strips4, L->d_partial, L->d_ufield,
                  L->d_cde_tiles, L->d_cde_tiles4, L->d_press, L->d_wall, L->d_wall_links,
                  L->d_wall_save,
                  L->d_mon};
  for (void *p : ptrs)
    if (p) (void)dev_free(L, p);
  for (hipEvent_t ev : L->prof_ev)
    if (ev) (void)hipEventDestroy(ev);
  L->prof_ev.clear();
  if (L->cap_stream) (void)hipStreamDestroy(L->cap_stream);
  if (L->side) (void)hipStreamDestroy(L->side);
  if (L->ev_fork) (void)hipEventDestroy(L->ev_fork);
  if (L->ev_join) (void)hipEventDestroy(L->ev_join);
}

gg_status gg_upload_desc(gg_lattice *L) {
  ++L->gen;
  LatDesc &h = L->h;
  std::memset(&h, 0, sizeof(h));
  h.nx = L->nx;
  h.ny = L->ny;
  h.pitch = L->pitch;
  h.node0 = L->node0;
  h.pairs = L->pairs ? 1 : 0;
  h.periodic_x = L->p.periodic_x != 0;
  h.periodic_y = L->p.periodic_y != 0;
  h.plane = L->plane;
  h.pop = L->d_pop;
  h.pop_b = L->d_pop_b;
  h.link = L->d_link;
  h.mask = L->d_mask;
  h.region = L->d_region;
  h.has_region = L->d_region != nullptr;
  h.R = L->d_R;
  h.has_source = L->d_R != nullptr;
  h.r_x0 = L->r_box[0];
  h.r_y0 = L->r_box[1];
  h.r_w = L->r_box[2];
  h.r_h = L->r_box[3];
  h.t = L->d_t;
  h.flux = L->d_flux;
  h.omega_f = 1.0 / L->p.tau_f;
  h.omega_g = 1.0 / L->tau_g;
  h.w0 = L->p.w0;
  h.wg_axis = (1.0 - L->p.w0) / 4.0;
  h.inv_cs2g = 1.0 / L->cs2g;
  h.rho0 = L->p.rho0;
  h.k_decay = L->p.k_decay;
  h.c_shift = L->p.c_shift;
  h.rho0_f = (float)h.rho0;
  h.omega_f_f = (float)h.omega_f;
  h.omega_g_f = (float)h.omega_g;
  h.wg_axis_f = (float)h.wg_axis;
  h.inv_cs2g_f = (float)h.inv_cs2g;
  h.k_decay_f = (float)h.k_decay;
  h.c_shift_f = (float)h.c_shift;
  h.ck = make_collk<double>(h.omega_f, h.omega_g, h.wg_axis, h.inv_cs2g);
  h.ck_f = make_collk<float>(h.omega_f, h.omega_g, h.wg_axis, h.inv_cs2g);
  for (int s = 0; s < GG_MAX_SEGMENTS; ++s) {
    const SegHost &g = L->seg[s];
    h.seg_kind[s] = g.set ? g.kind : 0;
    h.seg_nx[s] = g.nrm_x;
    h.seg_ny[s] = g.nrm_y;
    h.seg_umax[s] = g.u_max;
    h.seg_s0[s] = g.s0;
    h.seg_s1[s] = g.s1;
    h.seg_inv_w2[s] = g.set ? 1.0 / ((g.s1 - g.s0) * (g.s1 - g.s0)) : 0.0;
    h.seg_cin[s] = g.c_in;
    h.seg_umax4_f[s] = (float)(4.0 * h.seg_umax[s]);
    h.seg_s0_f[s] = (float)h.seg_s0[s];
    h.seg_s1_f[s] = (float)h.seg_s1[s];
    h.seg_inv_w2_f[s] = (float)h.seg_inv_w2[s];
    h.seg_cin_f[s] = (float)h.seg_cin[s];
    h.seg_rho[s] = g.rho;
    h.seg_rho_f[s] = (float)g.rho;
    h.seg_holdc[s] = g.hold_c ? 1 : 0;
  }
  h.n_phases = (int32_t)L->phases.size();
  h.t_origin = L->t_origin;
  int64_t start = 0;
  for (size_t k = 0; k < L->phases.size(); ++k) {
    const gg_phase &ph = L->phases[k];
    h.phase_start[k] = start;
    start += ph.duration;
    h.phase_open[k] = ph.open_mask;
    for (int s = 0; s < GG_MAX_SEGMENTS; ++s)
      h.phase_cin[k][s] = ((ph.c_in_set >> s) & 1u) ? ph.c_in[s] : L->seg[s].c_in;
    for (int s = 0; s < GG_MAX_SEGMENTS; ++s) h.phase_cin_f[k][s] = (float)h.phase_cin[k][s];
  }
  h.period = start > 0 ? start : 1;
  h.ufield = L->d_ufield;
  h.n_ufield = L->n_ufield;
  for (int k = 0; k < GG_MAX_PHASES; ++k) h.phase_field[k] = L->phase_field[k];
  GG_HIP(hipMemcpyAsync(L->d_desc, &h, sizeof(h), hipMemcpyHostToDevice, L->stream));
  GG_HIP(hipStreamSynchronize(L->stream));
  return GG_OK;
}

// Tiles of tx*ty nodes holding at least one fluid node, row-major.
static void build_tiles(const gg_lattice *L, int tx, int ty, int inst,
                        std::vector<Tile> &out) {
  for (int y0 = 0; y0 < L->ny; y0 += ty)
    for (int x0 = 0; x0 < L->nx; x0 += tx) {
      bool any = false, seg = false;
      for (int y = y0; y < std::min(y0 + ty, L->ny); ++y)
        for (int x = x0; x < std::min(x0 + tx, L->nx); ++x) {
          if (L->link[L->nid(x, y)] == NOT_FLUID) continue;
          any = true;
          if (L->touches_seg[(size_t)y * L->nx + x]) seg = true;
        }
      if (any) out.push_back(Tile{inst, x0, y0, seg ? TILE_TOUCHES_SEGMENT : 0});
    }
}

// Strips of the two-step pass: width (62) owned columns x h rows holding at
// least one fluid node, laid from the first column of each run of fluid
// columns of a band (rows y0 .. y0 + h - 1), listed band by band from left
// to right: horizontally adjacent strips store into the same cache lines at
// their common edge every row, so they go to the same XCD (a contiguous run
// of the list) and run side by side in one work-group. With split, a band
// piece with a link to a boundary segment is cut into 2-row strips and
// those with segment links go to the second list; otherwise it stays whole
// in the first. Flags: strip height << 8 | segment bit. The four-step pass
// takes tiles of 58 columns the same way.
static void build_strips(const gg_lattice *L, int h, int inst, bool split, std::vector<Tile> &main,
                         std::vector<Tile> &seg, int halo = 0, int width = 62) {
  auto scan = [&](int x0, int y0, int rows, bool &any, bool &sg) {
    any = sg = false;
    for (int y = y0; y < std::min(y0 + rows, L->ny); ++y)
      for (int x = x0; x < std::min(x0 + width, L->nx); ++x) {
        if (L->link[L->nid(x, y)] == NOT_FLUID) continue;
        any = true;
        if (L->touches_seg[(size_t)y * L->nx + x]) sg = true;
      }
    // halo 1 (pressure segments, rescaled at load): also when a node of
    // the one-node halo the tile collides touches a segment; halo 2 (the
    // four-step pass): within two nodes of the tile, the nodes whose state
    // at t + 1 the tile completes (wrapped on periodic axes)
    for (int yr = y0 - halo; halo > 0 && !sg && yr <= y0 + rows - 1 + halo; ++yr)
      for (int xr = x0 - halo; !sg && xr <= x0 + width - 1 + halo; ++xr) {
        int x = xr, y = yr;
        if (x < 0 || x >= L->nx) {
          if (!L->p.periodic_x) continue;
          x = (x + L->nx) % L->nx;
        }
        if (y < 0 || y >= L->ny) {
          if (!L->p.periodic_y) continue;
          y = (y + L->ny) % L->ny;
        }
        if (L->link[L->nid(x, y)] != NOT_FLUID && L->touches_seg[(size_t)y * L->nx + x]) sg = true;
      }
  };
  std::vector<uint8_t> colany((size_t)L->nx);
  for (int y0 = 0; y0 < L->ny; y0 += h) {
    // columns holding fluid in this band, as runs; runs less than a strip
    // apart are merged, so the strips laid from the start of each run never
    // overlap the next run's strips
    std::fill(colany.begin(), colany.end(), 0);
    for (int y = y0; y < std::min(y0 + h, L->ny); ++y)
      for (int x = 0; x < L->nx; ++x)
        if (L->link[L->nid(x, y)] != NOT_FLUID) colany[x] = 1;
    std::vector<std::pair<int, int>> runs;
    for (int x = 0; x < L->nx;) {
      if (!colany[x]) {
        ++x;
        continue;
      }
      int e = x;
      while (e < L->nx && colany[e]) ++e;
      if (!runs.empty() && x - runs.back().second < width)
        runs.back().second = e;
      else
        runs.push_back({x, e});
      x = e;
    }
    for (const auto &run : runs)
      for (int x0 = run.first; x0 < run.second; x0 += width) {
        bool any, sg;
        scan(x0, y0, h, any, sg);
        if (!any) continue;
        if (!sg || !split) {
          main.push_back(Tile{inst, x0, y0, (h << 8) | (sg ? TILE_TOUCHES_SEGMENT : 0)});
          continue;
        }
        for (int yy = y0; yy < std::min(y0 + h, L->ny); yy += 2) {
          const int rows = std::min(2, y0 + h - yy);
          scan(x0, yy, rows, any, sg);
          if (!any) continue;
          if (sg)
            seg.push_back(Tile{inst, x0, yy, (rows << 8) | TILE_TOUCHES_SEGMENT});
          else
            main.push_back(Tile{inst, x0, yy, rows << 8});
        }
      }
  }
}

// Fluid nodes owned by a list of pass tiles (width columns x the rows in
// the flags of each).
static int64_t owned_fluid(const gg_lattice *L, const std::vector<Tile> &list, int width = 62) {
  int64_t n = 0;
  for (const Tile &t : list)
    for (int y = t.y0; y < std::min(t.y0 + (t.flags >> 8), L->ny); ++y)
      for (int x = t.x0; x < std::min(t.x0 + width, L->nx); ++x)
        n += L->link[L->nid(x, y)] != NOT_FLUID;
  return n;
}

static bool has_pressure(const gg_lattice *L);

// The four-step pass (fuse 5) covers this lattice: no pressure segments
// (their rescaling runs between steps) nor the paper's walls, and periodic
// axes of 4 nodes or more (the tiles' three-node halo wraps once).
static bool pass4_ok(const gg_lattice *L) {
  return L->fuse == 5 && !has_pressure(L) && L->wall_scheme == 0 &&
         (!L->p.periodic_x || L->nx >= 4) && (!L->p.periodic_y || L->ny >= 4);
}

gg_status gg_rebuild_tiles(gg_lattice *L) {
  std::vector<Tile> t;
  build_tiles(L, L->tile_x, L->tile_y, 0, t);
  if (L->d_tiles) (void)dev_free(L, L->d_tiles);
  L->d_tiles = nullptr;
  L->n_tiles = (int)t.size();
  if (!t.empty()) {
    GG_HIP(dev_alloc(L, (void **)&L->d_tiles, t.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(L->d_tiles, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  std::vector<Tile> sv, ss;
  // with pressure segments the one-kernel pass rescales the state it loads
  // in every tile that collides a boundary node, halo included
  L->tiles_halo_seg = L->fuse == 4 && has_pressure(L);
  build_strips(L, L->strip_h, 0, L->fuse != 4, sv, ss, L->tiles_halo_seg ? 1 : 0);
  if (L->d_strips) (void)dev_free(L, L->d_strips);
  if (L->d_seg_strips) (void)dev_free(L, L->d_seg_strips);
  L->d_strips = L->d_seg_strips = nullptr;
  L->n_strips = (int)sv.size();
  L->n_seg_strips = (int)ss.size();
  L->strips_fluid = owned_fluid(L, sv);
  L->seg_strips_fluid = owned_fluid(L, ss);
  if (!sv.empty()) {
    GG_HIP(dev_alloc(L, (void **)&L->d_strips, sv.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(L->d_strips, sv.data(), sv.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  if (!ss.empty()) {
    GG_HIP(dev_alloc(L, (void **)&L->d_seg_strips, ss.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(L->d_seg_strips, ss.data(), ss.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  // the four-step pass's lists (6-row tiles, 2-row boundary tiles)
  if (L->d_strips4) (void)dev_free(L, L->d_strips4);
  if (L->d_seg_strips4) (void)dev_free(L, L->d_seg_strips4);
  L->d_strips4 = L->d_seg_strips4 = nullptr;
  L->n_strips4 = L->n_seg_strips4 = 0;
  L->strips4_fluid = L->seg_strips4_fluid = 0;
  L->tiles4 = pass4_ok(L);
  if (L->tiles4) {
    std::vector<Tile> m4, s4;
    build_strips(L, 6, 0, true, m4, s4, 2, 58);
    // in eight vertical stripes, each walked band by band: an XCD takes a
    // contiguous run of the list, and the tiles above and below a tile
    // (which share its three halo rows, half of what it loads) then run
    // soon after it on the same L2; a whole band of the lattice with its
    // halo rows need not fit in one XCD's L2
    std::stable_sort(m4.begin(), m4.end(), [&](const Tile &a, const Tile &b) {
      const int sa = (int)((int64_t)a.x0 * 8 / L->nx), sb = (int)((int64_t)b.x0 * 8 / L->nx);
      return sa != sb ? sa < sb : (a.y0 != b.y0 ? a.y0 < b.y0 : a.x0 < b.x0);
    });
    L->n_strips4 = (int)m4.size();
    L->n_seg_strips4 = (int)s4.size();
    L->strips4_fluid = owned_fluid(L, m4, 58);
    L->seg_strips4_fluid = owned_fluid(L, s4, 58);
    if (!m4.empty()) {
      GG_HIP(dev_alloc(L, (void **)&L->d_strips4, m4.size() * sizeof(Tile)));
      GG_HIP(hipMemcpy(L->d_strips4, m4.data(), m4.size() * sizeof(Tile), hipMemcpyHostToDevice));
    }
    if (!s4.empty()) {
      GG_HIP(dev_alloc(L, (void **)&L->d_seg_strips4, s4.size() * sizeof(Tile)));
      GG_HIP(hipMemcpy(L->d_seg_strips4, s4.data(), s4.size() * sizeof(Tile), hipMemcpyHostToDevice));
    }
  }
  if (L->graph_exec) (void)hipGraphExecDestroy(L->graph_exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->graph_exec = nullptr;
  L->graph = nullptr;
  return GG_OK;
}

static gg_status check_params(const gg_params *p) {
  if (!p) return fail(GG_ERR_ARG, "params is NULL");
  if (!(p->tau_f > 0.5)) return fail(GG_ERR_ARG, "tau_f must exceed 1/2");
  if (!(p->D > 0.0)) return fail(GG_ERR_ARG, "D must be positive");
  if (!(p->w0 >= 0.0 && p->w0 < 1.0)) return fail(GG_ERR_ARG, "w0 must lie in [0, 1)");
  if (!(p->rho0 > 0.0)) return fail(GG_ERR_ARG, "rho0 must be positive");
  if (!(p->k_decay >= 0.0)) return fail(GG_ERR_ARG, "k_decay must be non-negative");
  if (!std::isfinite(p->c_shift)) return fail(GG_ERR_ARG, "c_shift must be finite");
  return GG_OK;
}

extern "C" {

const char *gg_last_error(void) { return g_err.c_str(); }

gg_status gg_create(const uint8_t *mask, int32_t nx, int32_t ny, const gg_params *params,
                    gg_storage storage, void *hip_stream, gg_lattice **out) {
  return gg_create_ex(mask, nx, ny, params, storage, hip_stream, nullptr, out);
}

gg_status gg_create_ex(const uint8_t *mask, int32_t nx, int32_t ny, const gg_params *params,
                       gg_storage storage, void *hip_stream, const gg_alloc *allocator,
                       gg_lattice **out) {
  if (!out) return fail(GG_ERR_ARG, "out is NULL");
  if (allocator && (!allocator->alloc || !allocator->release))
    return fail(GG_ERR_ARG, "an allocator needs both its alloc and its release function");
  *out = nullptr;
  if (!mask) return fail(GG_ERR_ARG, "mask is NULL");
  if (nx < 1 || ny < 1) return fail(GG_ERR_ARG, "lattice dimensions must be positive");
  const size_t esize = storage_bytes(storage);
  if (esize == 0) return fail(GG_ERR_ARG, "unknown storage");
  gg_status st = check_params(params);
  if (st != GG_OK) return st;
  // one padding column (x = nx, doubling as x = -1 of the next row) and one
  // padding row on each side; rows start on 64-element boundaries
  const int pitch = (nx + 1 + 63) / 64 * 64;
  const int64_t plane_elems = (int64_t)(ny + 2) * pitch + 128;
  // kernels address a plane pair (the paired layout) with a 32-bit byte offset
  if (2 * plane_elems * (int64_t)esize > ((int64_t)1 << 32) - 4096)
    return fail(GG_ERR_ARG, "lattice too large: two population planes must stay below 4 GiB");

  gg_lattice *L = new gg_lattice();
  if (allocator) {
    L->alloc = *allocator;
    L->has_alloc = true;
  }
  L->nx = nx;
  L->ny = ny;
  L->pitch = pitch;
  L->node0 = pitch + 64;
  L->plane_elems = plane_elems;
  // Plane stride: the padded plane plus a stagger so that the 14 planes do
  // not start on the same DRAM channel.
  L->plane = plane_elems + 320;
  L->storage = storage;
  L->esize = esize;
  L->stream = (hipStream_t)hip_stream;
  L->p = *params;
  L->cs2g = (1.0 - params->w0) / 2.0;
  L->tau_g = 0.5 + params->D / L->cs2g;
  L->mask.assign(mask, mask + (size_t)nx * ny);
  L->t_origin = 0;
  L->t = 0;

  // classify links
  L->link.assign((size_t)plane_elems, NOT_FLUID);
  L->touches_seg.assign((size_t)nx * ny, 0);
  // the segments each fluid node links to (up to two mask values, 0: none)
  std::vector<uint16_t> node_segs((size_t)nx * ny, 0);
  int64_t nf = 0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const uint8_t m = L->mask[(size_t)y * nx + x];
      if (m > GG_FIRST_SEGMENT + GG_MAX_SEGMENTS - 1) {
        gg_status s = fail(GG_ERR_MASK, "mask value " + std::to_string(m) + " at (" +
                                            std::to_string(x) + "," + std::to_string(y) +
                                            ") is not 0, 1 or a segment id 2..17");
        delete L;
        return s;
      }
      if (m >= GG_FIRST_SEGMENT) L->seg_present[m - GG_FIRST_SEGMENT] = true;
      if (m != GG_MASK_FLUID) continue;
      uint8_t code = 0;
      int segs[8], nseg = 0;
      for (int k = 1; k < 9; ++k) {
        int xx = x + EX[k], yy = y + EY[k];
        bool inside = true;
        if (xx < 0 || xx >= nx) {
          if (params->periodic_x) xx = (xx + nx) % nx; else inside = false;
        }
        if (yy < 0 || yy >= ny) {
          if (params->periodic_y) yy = (yy + ny) % ny; else inside = false;
        }
        const uint8_t mm = inside ? L->mask[(size_t)yy * nx + xx] : (uint8_t)GG_MASK_WALL;
        if (mm != GG_MASK_FLUID) code |= (uint8_t)(1u << (k - 1));
        if (mm >= GG_FIRST_SEGMENT) {
          bool seen = false;
          for (int q = 0; q < nseg; ++q) seen = seen || segs[q] == mm;
          if (!seen) segs[nseg++] = mm;
        }
      }
      if (code == NOT_FLUID) {
        gg_status s = fail(GG_ERR_MASK, "fluid node (" + std::to_string(x) + "," +
                                            std::to_string(y) + ") has no fluid neighbour");
        delete L;
        return s;
      }
      if (nseg > 2) {
        gg_status s = fail(GG_ERR_MASK, "fluid node (" + std::to_string(x) + "," +
                                            std::to_string(y) + ") touches more than two segments");
        delete L;
        return s;
      }
      L->touches_seg[(size_t)y * nx + x] = nseg > 0;
      node_segs[(size_t)y * nx + x] =
          (uint16_t)((nseg > 0 ? segs[0] : 0) | (nseg > 1 ? segs[1] << 8 : 0));
      L->link[L->nid(x, y)] = code;
      ++nf;
    }
  L->n_fluid = nf;
  // a walking strip sums the boundary fluxes of a node and of the node
  // below it in one per-lane record of two segments
  for (int y = 1; y < ny && L->strip_flux_ok; ++y)
    for (int x = 0; x < nx; ++x) {
      const uint16_t a = node_segs[(size_t)y * nx + x], b = node_segs[(size_t)(y - 1) * nx + x];
      int u[4], nu = 0;
      for (int v : {a & 0xFF, a >> 8, b & 0xFF, b >> 8}) {
        bool seen = v == 0;
        for (int q = 0; q < nu; ++q) seen = seen || u[q] == v;
        if (!seen) u[nu++] = v;
      }
      if (nu > 2) {
        L->strip_flux_ok = false;
        break;
      }
    }

  if (hipGetDevice(&L->device) != hipSuccess) {
    delete L;
    return fail(GG_ERR_HIP, "hipGetDevice failed");
  }
  auto alloc = [&](void **p, size_t bytes) -> gg_status {
    hipError_t e = dev_alloc(L, p, bytes);
    if (e != hipSuccess) return fail(GG_ERR_OOM, std::string("device allocation: ") + hipGetErrorString(e));
    return GG_OK;
  };
  const size_t pop_bytes = (size_t)NPOP * L->plane * esize;
  if ((st = alloc(&L->d_pop, pop_bytes)) != GG_OK || (st = alloc(&L->d_pop_b, pop_bytes)) != GG_OK ||
      (st = alloc((void **)&L->d_link, (size_t)plane_elems)) != GG_OK ||
      (st = alloc((void **)&L->d_mask, (size_t)plane_elems)) != GG_OK ||
      (st = alloc((void **)&L->d_t, sizeof(int64_t))) != GG_OK ||
      (st = alloc((void **)&L->d_flux, 2 * GG_MAX_SEGMENTS * sizeof(double))) != GG_OK ||
      (st = alloc((void **)&L->d_acc, 8 * sizeof(double))) != GG_OK ||
      (st = alloc((void **)&L->d_desc, sizeof(LatDesc))) != GG_OK) {
    gg_free_device(L);
    delete L;
    return st;
  }
  std::vector<uint8_t> mpitch((size_t)plane_elems, GG_MASK_WALL);
  for (int y = 0; y < ny; ++y)
    std::memcpy(&mpitch[L->nid(0, y)], &L->mask[(size_t)y * nx], nx);
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(L->d_link, L->link.data(), L->link.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(L->d_mask, mpitch.data(), mpitch.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(L->d_pop, 0, pop_bytes);
  if (e == hipSuccess) e = hipMemset(L->d_pop_b, 0, pop_bytes);
  if (e == hipSuccess) e = hipMemset(L->d_t, 0, sizeof(int64_t));
  if (e == hipSuccess) e = hipMemset(L->d_flux, 0, 2 * GG_MAX_SEGMENTS * sizeof(double));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&L->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&L->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&L->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&L->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    gg_status s = fail(GG_ERR_HIP, std::string("lattice set-up: ") + hipGetErrorString(e));
    gg_free_device(L);
    delete L;
    return s;
  }
  // auxiliary kernels always run 64 x 4 tiles
  std::vector<Tile> aux;
  build_tiles(L, 64, 4, 0, aux);
  L->n_aux_tiles = (int)aux.size();
  if (!aux.empty()) {
    if ((st = alloc((void **)&L->d_aux_tiles, aux.size() * sizeof(Tile))) != GG_OK) {
      gg_free_device(L);
      delete L;
      return st;
    }
    if (hipMemcpy(L->d_aux_tiles, aux.data(), aux.size() * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess) {
      gg_free_device(L);
      delete L;
      return fail(GG_ERR_HIP, "upload of the tile list failed");
    }
  }
  L->tile_x = 64;
  L->tile_y = 4;
  L->graph_chunk = 64;
  if ((st = gg_rebuild_tiles(L)) != GG_OK || (st = gg_upload_desc(L)) != GG_OK ||
      (st = gg_init(L, nullptr, nullptr, nullptr, nullptr, GG_HOST)) != GG_OK) {
    gg_free_device(L);
    delete L;
    return st;
  }
  *out = L;
  return GG_OK;
}

void gg_destroy(gg_lattice *L) {
  if (!L) return;
  (void)hipStreamSynchronize(L->stream);
  gg_free_device(L);
  delete L;
}

// Checks the geometry of segment id with outward normal (nrm_x, nrm_y) and
// returns the halfway-wall tangential coordinates of its ghost line.
static gg_status segment_geometry(gg_lattice *L, int32_t id, int32_t nrm_x, int32_t nrm_y,
                                  double *s0, double *s1) {
  if (id < GG_FIRST_SEGMENT || id >= GG_FIRST_SEGMENT + GG_MAX_SEGMENTS)
    return fail(GG_ERR_ARG, "segment id must lie in 2..17");
  if (std::abs(nrm_x) + std::abs(nrm_y) != 1) return fail(GG_ERR_ARG, "normal must be an axis unit vector");
  int smin = 1 << 30, smax = -(1 << 30);
  int64_t cells = 0;
  for (int y = 0; y < L->ny; ++y)
    for (int x = 0; x < L->nx; ++x) {
      if (L->mask[(size_t)y * L->nx + x] != id) continue;
      ++cells;
      int xi = x - nrm_x, yi = y - nrm_y;
      bool inside = true;
      if (xi < 0 || xi >= L->nx) {
        if (L->p.periodic_x) xi = (xi + L->nx) % L->nx; else inside = false;
      }
      if (yi < 0 || yi >= L->ny) {
        if (L->p.periodic_y) yi = (yi + L->ny) % L->ny; else inside = false;
      }
      if (!inside || L->mask[(size_t)yi * L->nx + xi] != GG_MASK_FLUID)
        return fail(GG_ERR_MASK, "segment " + std::to_string(id) + " ghost cell (" +
                                     std::to_string(x) + "," + std::to_string(y) +
                                     ") has no fluid cell against its normal");
      const int s = nrm_x != 0 ? y : x;
      smin = std::min(smin, s);
      smax = std::max(smax, s);
    }
  if (cells == 0) return fail(GG_ERR_MASK, "segment " + std::to_string(id) + " has no cells in the mask");
  *s0 = smin - 0.5;
  *s1 = smax + 0.5;
  return GG_OK;
}

gg_status gg_set_segment(gg_lattice *L, int32_t id, gg_seg_kind kind, int32_t nrm_x,
                         int32_t nrm_y, double u_max, double c_in) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (kind != GG_SEG_INLET && kind != GG_SEG_OUTLET)
    return fail(GG_ERR_ARG, "unknown segment kind (pressure segments: gg_set_pressure_segment)");
  if (!std::isfinite(u_max) || !std::isfinite(c_in)) return fail(GG_ERR_ARG, "u_max and c_in must be finite");
  double s0 = 0.0, s1 = 1.0;
  gg_status st = segment_geometry(L, id, nrm_x, nrm_y, &s0, &s1);
  if (st != GG_OK) return st;
  GG_HIP(hipStreamSynchronize(L->stream));
  SegHost &g = L->seg[id - GG_FIRST_SEGMENT];
  g.set = true;
  g.kind = kind;
  g.nrm_x = nrm_x;
  g.nrm_y = nrm_y;
  g.u_max = u_max;
  g.c_in = c_in;
  g.rho = L->p.rho0;
  g.hold_c = false;
  g.s0 = s0;
  g.s1 = s1;
  L->press_dirty = true;
  return gg_upload_desc(L);
}

gg_status gg_set_pressure_segment(gg_lattice *L, int32_t id, int32_t nrm_x, int32_t nrm_y,
                                  double rho, double c_in, int32_t hold_c) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (!(rho > 0.0) || !std::isfinite(rho) || !std::isfinite(c_in))
    return fail(GG_ERR_ARG, "rho must be positive and finite, c_in finite");
  double s0 = 0.0, s1 = 1.0;
  gg_status st = segment_geometry(L, id, nrm_x, nrm_y, &s0, &s1);
  if (st != GG_OK) return st;
  GG_HIP(hipStreamSynchronize(L->stream));
  SegHost &g = L->seg[id - GG_FIRST_SEGMENT];
  g.set = true;
  g.kind = GG_SEG_PRESSURE;
  g.nrm_x = nrm_x;
  g.nrm_y = nrm_y;
  g.u_max = 0.0;
  g.c_in = c_in;
  g.rho = rho;
  g.hold_c = hold_c != 0;
  g.s0 = s0;
  g.s1 = s1;
  L->press_dirty = true;
  return gg_upload_desc(L);
}

// True if a configured segment is a pressure boundary.
static bool has_pressure(const gg_lattice *L) {
  for (int s = 0; s < GG_MAX_SEGMENTS; ++s)
    if (L->seg[s].set && L->seg[s].kind == GG_SEG_PRESSURE) return true;
  return false;
}

// The fluid nodes that take a boundary value from a pressure segment's
// ghost cell (in any phase), uploaded as (x, y) pairs.
static gg_status pressure_nodes(gg_lattice *L) {
  if (!L->press_dirty) return GG_OK;
  // the tile lists mark the tiles that must rescale what they load
  if (L->tiles_halo_seg != (L->fuse == 4 && has_pressure(L)) || L->tiles4 != pass4_ok(L)) {
    gg_status st = gg_rebuild_tiles(L);
    if (st != GG_OK) return st;
  }
  if (L->cde_halo_seg != has_pressure(L)) L->cde_tiles_rows = 0;
  std::vector<int32_t> xy;
  if (has_pressure(L))
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        const uint8_t lc = L->link[L->nid(x, y)];
        if (lc == NOT_FLUID || lc == 0) continue;
        // the pressure segments among the source cells x - e_j, in order of
        // first appearance for j = 1..8 (the kernel takes the first open one)
        uint32_t cand = 0;
        int n_cand = 0;
        for (int j = 1; j < 9; ++j) {
          if (!((lc >> (OPP[j] - 1)) & 1)) continue;  // x - e_j is fluid
          int xx = x - EX[j], yy = y - EY[j];
          bool inside = true;
          if (xx < 0 || xx >= L->nx) {
            if (L->p.periodic_x) xx = (xx + L->nx) % L->nx; else inside = false;
          }
          if (yy < 0 || yy >= L->ny) {
            if (L->p.periodic_y) yy = (yy + L->ny) % L->ny; else inside = false;
          }
          if (!inside) continue;
          const int m = L->mask[(size_t)yy * L->nx + xx];
          if (m < GG_FIRST_SEGMENT || !L->seg[m - GG_FIRST_SEGMENT].set ||
              L->seg[m - GG_FIRST_SEGMENT].kind != GG_SEG_PRESSURE)
            continue;
          const uint32_t q1 = (uint32_t)(m - GG_FIRST_SEGMENT + 1);
          bool seen = false;
          for (int b = 0; b < n_cand; ++b) seen = seen || ((cand >> (8 * b)) & 0xFFu) == q1;
          if (seen) continue;
          if (n_cand == 4) return fail(GG_ERR_ARG, "a node touches more than four pressure segments");
          cand |= q1 << (8 * n_cand++);
        }
        if (n_cand > 0) {
          xy.push_back(x);
          xy.push_back(y);
          xy.push_back((int32_t)cand);
        }
      }
  if (L->d_press) GG_HIP(dev_free(L, L->d_press));
  L->d_press = nullptr;
  L->n_press = (int)(xy.size() / 3);
  if (!xy.empty()) {
    GG_HIP(dev_alloc(L, (void **)&L->d_press, xy.size() * sizeof(int32_t)));
    GG_HIP(hipMemcpy(L->d_press, xy.data(), xy.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  L->press_dirty = false;
  // captured graphs hold the old list and the old launch form
  if (L->graph_exec) (void)hipGraphExecDestroy(L->graph_exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->graph_exec = nullptr;
  L->graph = nullptr;
  gg_drop_cde_graphs(L);
  return GG_OK;
}

gg_status gg_set_schedule(gg_lattice *L, const gg_phase *phases, int32_t n, int64_t t_origin) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (n < 0 || n > GG_MAX_PHASES) return fail(GG_ERR_ARG, "n_phases must lie in 0..64");
  if (n > 0 && !phases) return fail(GG_ERR_ARG, "phases is NULL");
  int64_t period = 0;
  for (int k = 0; k < n; ++k) {
    if (phases[k].duration <= 0) return fail(GG_ERR_ARG, "phase durations must be positive");
    if (phases[k].open_mask >> GG_MAX_SEGMENTS) return fail(GG_ERR_ARG, "open_mask has bits beyond segment 17");
    period += phases[k].duration;
    if (period > ((int64_t)1 << 60)) return fail(GG_ERR_ARG, "schedule period too long");
  }
  L->phases.assign(phases, phases + n);
  L->t_origin = t_origin;
  return gg_upload_desc(L);
}

gg_status gg_set_source(gg_lattice *L, const double *R, gg_where where) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  ++L->gen;
  if (L->d_R) (void)dev_free(L, L->d_R);
  L->d_R = nullptr;
  L->r_box[0] = L->r_box[1] = L->r_box[2] = L->r_box[3] = 0;
  if (R) {
    const size_t n = (size_t)L->nx * L->ny;
    std::vector<double> h(n);
    if (where == GG_DEVICE) {
      GG_HIP(hipStreamSynchronize(L->stream));
      GG_HIP(hipMemcpy(h.data(), R, n * sizeof(double), hipMemcpyDeviceToHost));
    } else {
      std::memcpy(h.data(), R, n * sizeof(double));
    }
    int x0 = L->nx, y0 = L->ny, x1 = -1, y1 = -1;
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        const double v = h[(size_t)y * L->nx + x];
        if (!std::isfinite(v)) return fail(GG_ERR_ARG, "source has non-finite entries");
        if (v != 0.0 && L->mask[(size_t)y * L->nx + x] == GG_MASK_FLUID) {
          x0 = std::min(x0, x); x1 = std::max(x1, x);
          y0 = std::min(y0, y); y1 = std::max(y1, y);
        }
      }
    if (x1 >= 0) {
      const int w = x1 - x0 + 1, hh = y1 - y0 + 1;
      std::vector<double> patch((size_t)w * hh);
      for (int y = 0; y < hh; ++y)
        for (int x = 0; x < w; ++x) patch[(size_t)y * w + x] = h[(size_t)(y0 + y) * L->nx + x0 + x];
      GG_HIP(dev_alloc(L, (void **)&L->d_R, patch.size() * sizeof(double)));
      GG_HIP(hipMemcpy(L->d_R, patch.data(), patch.size() * sizeof(double), hipMemcpyHostToDevice));
      L->r_box[0] = x0; L->r_box[1] = y0; L->r_box[2] = w; L->r_box[3] = hh;
    }
  }
  return gg_upload_desc(L);
}

gg_status gg_set_region(gg_lattice *L, const uint8_t *region) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  ++L->gen;
  if (L->d_region) (void)dev_free(L, L->d_region);
  L->d_region = nullptr;
  if (region) {
    std::vector<uint8_t> r((size_t)L->plane_elems, 0);
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) r[L->nid(x, y)] = region[(size_t)y * L->nx + x] ? 1 : 0;
    GG_HIP(dev_alloc(L, (void **)&L->d_region, r.size()));
    GG_HIP(hipMemcpy(L->d_region, r.data(), r.size(), hipMemcpyHostToDevice));
  }
  return gg_upload_desc(L);
}

gg_status gg_init(gg_lattice *L, const double *rho, const double *ux, const double *uy,
                  const double *C, gg_where where) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  const size_t n = (size_t)L->nx * L->ny;
  const double *src[4] = {rho, ux, uy, C};
  double *dev[4] = {nullptr, nullptr, nullptr, nullptr};
  gg_status st = GG_OK;
  if (where == GG_HOST) {
    for (int q = 0; q < 4 && st == GG_OK; ++q) {
      if (!src[q]) continue;
      if (dev_alloc(L, (void **)&dev[q], n * sizeof(double)) != hipSuccess) {
        st = fail(GG_ERR_OOM, "hipMalloc of an initial field failed");
        break;
      }
      if (hipMemcpy(dev[q], src[q], n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        st = fail(GG_ERR_HIP, "copy of an initial field failed");
    }
  } else {
    for (int q = 0; q < 4; ++q) dev[q] = const_cast<double *>(src[q]);
  }
  if (st == GG_OK) {
    hipError_t e = launch_init(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6,
                               dev[0], dev[1], dev[2], dev[3], L->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L->d_t, 0, sizeof(int64_t), L->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L->d_flux, 0, 2 * GG_MAX_SEGMENTS * sizeof(double), L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) st = fail(GG_ERR_HIP, std::string("init: ") + hipGetErrorString(e));
  }
  if (where == GG_HOST)
    for (int q = 0; q < 4; ++q)
      if (dev[q]) (void)dev_free(L, dev[q]);
  if (st == GG_OK) L->t = 0;
  return st;
}

static gg_status check_segments(gg_lattice *L) {
  for (int s = 0; s < GG_MAX_SEGMENTS; ++s)
    if (L->seg_present[s] && !L->seg[s].set)
      return fail(GG_ERR_STATE, "segment " + std::to_string(s + GG_FIRST_SEGMENT) +
                                    " is in the mask but was not configured");
  return GG_OK;
}

// Launch `n` step kernels on `st` for a lattice whose device counter reads
// t0 (host mirror), then advance the counter. With the two-step pass on,
// t0 even and n a multiple of 4, the steps go in n/2 passes that alternate
// between the two plane sets and end in the first one.
// One two-step pass: the segment strips on the side stream, forked from and
// joined back to st (inside a capture this becomes two graph branches).
// Lattices whose steps must run with fix-ups around them.
static bool special_boundaries(const gg_lattice *L) { return has_pressure(L) || L->wall_scheme != 0; }

// The two-step pass is on and covers the lattice's boundaries: the paper's
// walls need single steps, pressure segments the row-parallel tiles.
static bool pass_ok(const gg_lattice *L) {
  return L->fuse >= 2 && L->wall_scheme == 0 && (L->n_press == 0 || L->fuse >= 3);
}

// The fluid nodes with a link from a wall or from a segment's ghost cell
// (a valve that may close), for the paper's walls.
static gg_status wall_nodes(gg_lattice *L) {
  if (!L->wall_dirty) return GG_OK;
  std::vector<int32_t> xy, links;
  if (L->wall_scheme != 0)
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        const uint8_t lc = L->link[L->nid(x, y)];
        if (lc == NOT_FLUID || lc == 0) continue;
        const int k = (int)(xy.size() / 2);
        xy.push_back(x);
        xy.push_back(y);
        for (int i = 1; i < 9; ++i)  // bit opp(i) - 1: x - e_i is not fluid
          if ((lc >> (OPP[i] - 1)) & 1) {
            links.push_back(x);
            links.push_back(y);
            links.push_back(k * 8 + (i - 1));
          }
      }
  if (L->d_wall) GG_HIP(dev_free(L, L->d_wall));
  if (L->d_wall_links) GG_HIP(dev_free(L, L->d_wall_links));
  if (L->d_wall_save) GG_HIP(dev_free(L, L->d_wall_save));
  L->d_wall = nullptr;
  L->d_wall_links = nullptr;
  L->d_wall_save = nullptr;
  L->n_wall = (int)(xy.size() / 2);
  L->n_wall_links = (int)(links.size() / 3);
  if (!xy.empty()) {
    GG_HIP(dev_alloc(L, (void **)&L->d_wall, xy.size() * sizeof(int32_t)));
    GG_HIP(hipMemcpy(L->d_wall, xy.data(), xy.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    GG_HIP(dev_alloc(L, (void **)&L->d_wall_links, links.size() * sizeof(int32_t)));
    GG_HIP(hipMemcpy(L->d_wall_links, links.data(), links.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    const size_t tb = L->storage == GG_F64 ? 8 : 4;
    GG_HIP(dev_alloc(L, (void **)&L->d_wall_save, (size_t)L->n_wall * 16 * tb));
  }
  L->wall_dirty = false;
  if (L->graph_exec) (void)hipGraphExecDestroy(L->graph_exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->graph_exec = nullptr;
  L->graph = nullptr;
  gg_drop_cde_graphs(L);
  return GG_OK;
}

// Profiling (gg_step_profile): an event recorded on st before a launch of
// the dominant kernel (prof_begin returns its index, or -1 when profiling is
// off) and one after it (prof_end, tagged with the launch's kind).
static hipError_t prof_begin(gg_lattice *L, hipStream_t st, long &idx) {
  idx = -1;
  if (!L->prof) return hipSuccess;
  while (L->prof_ev.size() < L->prof_used + 2) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    L->prof_ev.push_back(ev);
  }
  idx = (long)L->prof_used;
  L->prof_used += 2;
  return hipEventRecord(L->prof_ev[idx], st);
}

static hipError_t prof_end(gg_lattice *L, hipStream_t st, long idx, int kind) {
  if (idx < 0) return hipSuccess;
  L->prof_kind.push_back((int8_t)kind);
  return hipEventRecord(L->prof_ev[idx + 1], st);
}

static hipError_t launch_pass(gg_lattice *L, int dir, int dt, hipStream_t st) {
  hipError_t e = hipSuccess;
  const bool fork = L->n_seg_strips > 0 && L->n_strips > 0;
  const bool press = L->n_press > 0;  // (fuse 3, 4 and 5 only)
  long pidx = -1;
  // (with the four-step pass on, the two-step passes of leftover steps are
  // not the dominant kernel: profiled apart, kind 4)
  const int kind = L->tiles4 && pass4_ok(L) ? 4 : 0;
  if (L->fuse == 4) {  // one kernel with the boundary rules for every tile
    e = prof_begin(L, st, pidx);
    if (e == hipSuccess)
      e = launch_tile2(L->storage, L->pairs, true, L->strip_h, L->d_desc, L->d_strips,
                       L->n_strips, dir, dt, st, press);
    if (e == hipSuccess) e = prof_end(L, st, pidx, 0);
    return e;
  }
  auto run = [&](bool seg, const Tile *list, int n, hipStream_t s) {
    // the segment list holds 2-row tiles
    return L->fuse >= 3 ? launch_tile2(L->storage, L->pairs, seg, seg ? 2 : L->strip_h, L->d_desc,
                                       list, n, dir, dt, s, press)
                        : launch_step2(L->storage, L->pairs, seg, L->d_desc, list, n, dir, dt, s);
  };
  if (fork) {
    e = hipEventRecord(L->ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(L->side, L->ev_fork, 0);
    if (e == hipSuccess) e = run(true, L->d_seg_strips, L->n_seg_strips, L->side);
    if (e == hipSuccess) e = hipEventRecord(L->ev_join, L->side);
  } else if (L->n_seg_strips > 0) {
    e = run(true, L->d_seg_strips, L->n_seg_strips, st);
  }
  if (e == hipSuccess) e = prof_begin(L, st, pidx);
  if (e == hipSuccess) e = run(false, L->d_strips, L->n_strips, st);
  if (e == hipSuccess) e = prof_end(L, st, pidx, kind);
  if (fork && e == hipSuccess) e = hipStreamWaitEvent(st, L->ev_join, 0);
  return e;
}

// One four-step pass: the boundary tiles on the side stream as in
// launch_pass.
static hipError_t launch_pass4(gg_lattice *L, int dir, int dt, hipStream_t st) {
  hipError_t e = hipSuccess;
  const bool fork = L->n_seg_strips4 > 0 && L->n_strips4 > 0;
  if (fork) {
    e = hipEventRecord(L->ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(L->side, L->ev_fork, 0);
    if (e == hipSuccess)
      e = launch_tile4(L->storage, L->pairs, true, L->d_desc, L->d_seg_strips4, L->n_seg_strips4,
                       dir, dt, L->side);
    if (e == hipSuccess) e = hipEventRecord(L->ev_join, L->side);
  } else if (L->n_seg_strips4 > 0) {
    e = launch_tile4(L->storage, L->pairs, true, L->d_desc, L->d_seg_strips4, L->n_seg_strips4, dir,
                     dt, st);
  }
  long pidx = -1;
  if (e == hipSuccess) e = prof_begin(L, st, pidx);
  if (e == hipSuccess)
    e = launch_tile4(L->storage, L->pairs, false, L->d_desc, L->d_strips4, L->n_strips4, dir, dt, st);
  if (e == hipSuccess) e = prof_end(L, st, pidx, 0);
  if (fork && e == hipSuccess) e = hipStreamWaitEvent(st, L->ev_join, 0);
  return e;
}

static hipError_t launch_steps(gg_lattice *L, int64_t t0, int64_t n, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (L->tiles4 && pass4_ok(L) && !(t0 & 1) && n % 4 == 0) {
    // four-step passes in pairs (ending in the first plane set), then the
    // last four steps of a run of 8k + 4 in two two-step passes
    const int64_t p4 = n / 8 * 2;
    for (int64_t k = 0; k < p4 && e == hipSuccess; ++k)
      e = launch_pass4(L, (int)(k & 1), (int)(4 * k), st);
    for (int64_t k = 0; k < (n % 8) / 2 && e == hipSuccess; ++k)
      e = launch_pass(L, (int)(k & 1), (int)(4 * p4 + 2 * k), st);
  } else if (pass_ok(L) && !(t0 & 1) && n % 4 == 0) {
    // with pressure segments the pass rescales the boundary nodes between
    // its two steps; the state it leaves is rescaled by the kernel after
    // it, or, in the one-kernel form, by the next pass as it loads it (bit
    // 1 of dir), so that only the last pass of the run needs the kernel
    const int64_t passes = n / 2;
    const bool at_load = L->n_press > 0 && L->fuse == 4 && L->tiles_halo_seg;
    for (int64_t k = 0; k < passes && e == hipSuccess; ++k) {
      e = launch_pass(L, (int)(k & 1) | (at_load && k > 0 ? 2 : 0), (int)(2 * k), st);
      if (e == hipSuccess && L->n_press > 0 && (!at_load || k == passes - 1))
        e = launch_rescale(L->storage, L->d_desc, L->d_press, L->n_press, (int)(2 * k + 1), true,
                           st, (k & 1) == 0);
    }
  } else {
    // single steps: with the paper's walls, the values of step t the wall
    // rule needs are saved before each step and the wall links written
    // after it; with pressure segments the boundary nodes are rescaled
    // after each step
    const int block = L->tile_x * L->tile_y;
    const int txs = ilog2(L->tile_x);
    for (int64_t dt = 0; dt < n && e == hipSuccess; ++dt) {
      if (L->n_wall > 0)
        e = launch_wall_save(L->storage, L->d_desc, L->d_wall, L->n_wall, L->d_wall_links,
                             L->n_wall_links, (int)dt, true, L->d_wall_save, st);
      long pidx = -1;
      if (e == hipSuccess) e = prof_begin(L, st, pidx);
      if (e == hipSuccess)
        e = launch_step(L->storage, L->pairs, block, ((t0 + dt) & 1) != 0, L->d_desc,
                        L->d_tiles, L->n_tiles, txs, (int)dt, st);
      if (e == hipSuccess) e = prof_end(L, st, pidx, 1 + (int)((t0 + dt) & 1));
      if (e == hipSuccess && L->n_wall > 0)
        e = launch_wall_apply(L->storage, L->d_desc, L->d_wall_links, L->n_wall_links,
                              (int)dt, L->d_wall_save, true, st);
      if (e == hipSuccess && L->n_press > 0)
        e = launch_rescale(L->storage, L->d_desc, L->d_press, L->n_press, (int)dt, true, st);
    }
  }
  if (e == hipSuccess) e = launch_advance(L->d_desc, 1, n, st);
  return e;
}

// n steps without monitor reductions: an odd-t step first, then graph
// replays (not while profiling), passes in groups of four, leftovers.
static gg_status step_run(gg_lattice *L, int64_t n) {
  int64_t left = n;
  // graph chunk: even (a multiple of 4 with the two-step pass), so every
  // replay starts on an even step and leaves the state in the first plane set
  const int K = L->graph_chunk;
  if ((L->t & 1) && left > 0) {
    GG_HIP(launch_steps(L, L->t, 1, L->stream));
    L->t += 1;
    left -= 1;
  }
  if (K > 0 && left >= K) {
    if (!L->graph_exec) {
      // (no profiling events inside the captured graph)
      const bool prof = L->prof;
      L->prof = false;
      GG_HIP(hipStreamBeginCapture(L->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = launch_steps(L, 0, K, L->cap_stream);
      L->prof = prof;
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(L->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(GG_ERR_HIP, std::string("graph capture: ") +
                                    hipGetErrorString(e != hipSuccess ? e : e2));
      }
      L->graph = g;
      GG_HIP(hipGraphInstantiate(&L->graph_exec, L->graph, nullptr, nullptr, 0));
    }
    while (left >= K) {
      // (profiling: one event pair around each replay, kind 3)
      long pidx = -1;
      GG_HIP(prof_begin(L, L->stream, pidx));
      GG_HIP(hipGraphLaunch(L->graph_exec, L->stream));
      GG_HIP(prof_end(L, L->stream, pidx, 3));
      left -= K;
      L->t += K;
    }
  }
  const int64_t quads = pass_ok(L) ? left / 4 * 4 : 0;
  if (quads > 0) {
    GG_HIP(launch_steps(L, L->t, quads, L->stream));
    L->t += quads;
    left -= quads;
  }
  if (left > 0) {
    GG_HIP(launch_steps(L, L->t, left, L->stream));
    L->t += left;
  }
  return GG_OK;
}

// The FP64 reduction of gg_diagnostics into the monitor record, launched
// on the lattice's stream at the current step; the flux accumulators are
// copied beside the totals at the same point.
static gg_status monitor_launch(gg_lattice *L) {
  GG_HIP(launch_fill(L->d_mon, 8, 0.0, L->stream));
  GG_HIP(launch_reduce(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6, L->d_partial,
                       L->d_mon, L->stream, REDUCE_GROUPS));
  GG_HIP(hipMemcpyAsync(L->d_mon + 8, L->d_flux, 2 * GG_MAX_SEGMENTS * sizeof(double),
                        hipMemcpyDeviceToDevice, L->stream));
  L->mon_last_t = L->t;
  L->mon_count += 1;
  return GG_OK;
}

static int64_t steps_to_monitor(const gg_lattice *L) {
  const int64_t k = L->mon_every;
  const int64_t r = ((L->t - L->mon_t0) % k + k) % k;
  return k - r;
}

gg_status gg_step(gg_lattice *L, int64_t n) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (n < 0) return fail(GG_ERR_ARG, "n must be non-negative");
  gg_status st = check_segments(L);
  if (st != GG_OK) return st;
  if ((st = pressure_nodes(L)) != GG_OK || (st = wall_nodes(L)) != GG_OK) return st;
  if (L->mon_every <= 0) return step_run(L, n);
  int64_t left = n;
  while (left > 0) {
    const int64_t run = std::min(left, steps_to_monitor(L));
    if ((st = step_run(L, run)) != GG_OK) return st;
    left -= run;
    if (steps_to_monitor(L) == L->mon_every && (st = monitor_launch(L)) != GG_OK) return st;
  }
  return GG_OK;
}

gg_status gg_set_monitor(gg_lattice *L, int64_t every) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (every < 0) return fail(GG_ERR_ARG, "every must be non-negative");
  if (every > 0) {
    if (!L->d_mon && dev_alloc(L, (void **)&L->d_mon, (8 + 2 * GG_MAX_SEGMENTS) * sizeof(double)) != hipSuccess) {
      L->d_mon = nullptr;
      return fail(GG_ERR_OOM, "monitor record");
    }
    if (!L->d_partial && L->n_aux_tiles > 0 &&
        dev_alloc(L, (void **)&L->d_partial, (size_t)6 * L->n_aux_tiles * sizeof(double)) != hipSuccess) {
      L->d_partial = nullptr;
      return fail(GG_ERR_OOM, "diagnostics partials");
    }
  }
  L->mon_every = every;
  L->mon_t0 = L->t;
  L->mon_last_t = -1;
  L->mon_count = 0;
  return GG_OK;
}

gg_status gg_monitor_read(gg_lattice *L, gg_diag *out, int64_t *count) {
  if (!L || !out) return fail(GG_ERR_ARG, "NULL argument");
  if (L->mon_count == 0 || !L->d_mon) return fail(GG_ERR_STATE, "no monitor reduction has run");
  double rec[8 + 2 * GG_MAX_SEGMENTS];
  GG_HIP(hipStreamSynchronize(L->stream));
  GG_HIP(hipMemcpy(rec, L->d_mon, sizeof(rec), hipMemcpyDeviceToHost));
  gg_fill_diag(L, rec, rec + 8, L->mon_last_t, out);
  if (count) *count = L->mon_count;
  if (out->n_nonfinite > 0)
    return fail(GG_ERR_NONFINITE, std::to_string(out->n_nonfinite) + " fluid nodes held non-finite populations at step " + std::to_string(out->t));
  return GG_OK;
}

gg_status gg_step_profile(gg_lattice *L, int64_t n, gg_profile *out) {
  if (!L || !out) return fail(GG_ERR_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  hipEvent_t a = nullptr, b = nullptr;
  GG_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(GG_ERR_HIP, "event creation");
  }
  const int64_t mon0 = L->mon_count;
  L->prof = true;
  L->prof_used = 0;
  L->prof_kind.clear();
  hipError_t e = hipEventRecord(a, L->stream);
  gg_status st = e == hipSuccess ? gg_step(L, n) : fail(GG_ERR_HIP, hipGetErrorString(e));
  L->prof = false;
  if (st == GG_OK && (e = hipEventRecord(b, L->stream)) == hipSuccess)
    e = hipStreamSynchronize(L->stream);
  if (st == GG_OK && e != hipSuccess) st = fail(GG_ERR_HIP, std::string("profile: ") + hipGetErrorString(e));
  float ms = 0.0f;
  if (st == GG_OK && (e = hipEventElapsedTime(&ms, a, b)) != hipSuccess)
    st = fail(GG_ERR_HIP, std::string("profile: ") + hipGetErrorString(e));
  out->ms_total = ms;
  for (size_t k = 0; k < L->prof_kind.size() && st == GG_OK; ++k) {
    float x = 0.0f;
    if ((e = hipEventElapsedTime(&x, L->prof_ev[2 * k], L->prof_ev[2 * k + 1])) != hipSuccess) {
      st = fail(GG_ERR_HIP, std::string("profile: ") + hipGetErrorString(e));
      break;
    }
    const int kind = L->prof_kind[k];
    if (kind == 0) {
      out->n_pass += 1;
      out->ms_pass += x;
    } else if (kind == 4) {
      out->n_pass2 += 1;
      out->ms_pass2 += x;
    } else if (kind == 3) {
      out->n_graph += 1;
      out->ms_graph += x;
      if (L->tiles4 && pass4_ok(L)) out->graph_passes += L->graph_chunk / 4;
      else if (pass_ok(L)) out->graph_passes += L->graph_chunk / 2;
      else out->graph_singles += L->graph_chunk;
    } else {
      out->n_single[kind - 1] += 1;
      out->ms_single[kind - 1] += x;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  out->n_monitor = L->mon_count - mon0;
  out->fuse = pass_ok(L) ? L->fuse : 1;
  out->rows = L->strip_h;
  out->steps_per_pass = 2;
  out->pass_fluid = L->fuse == 4 ? L->n_fluid : L->strips_fluid;
  out->pass_side_fluid = L->fuse == 4 ? 0 : L->seg_strips_fluid;
  out->pass_tiles = L->n_strips;
  out->pass_side_tiles = L->fuse == 4 ? 0 : L->n_seg_strips;
  if (L->tiles4 && pass4_ok(L)) {  // the four-step pass's interior kernel
    out->rows = 6;
    out->steps_per_pass = 4;
    out->pass_fluid = L->strips4_fluid;
    out->pass_side_fluid = L->seg_strips4_fluid;
    out->pass_tiles = L->n_strips4;
    out->pass_side_tiles = L->n_seg_strips4;
  }
  return st;
}

static gg_status gg_read_impl(gg_lattice *L, double *rho, double *ux, double *uy, double *C,
                       double *f, double *g, gg_where where) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  const int64_t n = (int64_t)L->nx * L->ny;
  double *user[6] = {rho, ux, uy, C, f, g};
  const int64_t len[6] = {n, n, n, n, 9 * n, 5 * n};
  const double fillv[6] = {NAN, NAN, NAN, NAN, 0.0, 0.0};
  double *dev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  gg_status st = GG_OK;
  for (int q = 0; q < 6; ++q) {
    if (!user[q]) continue;
    if (where == GG_HOST) {
      if (dev_alloc(L, (void **)&dev[q], len[q] * sizeof(double)) != hipSuccess) {
        st = fail(GG_ERR_OOM, "hipMalloc of a read-back buffer failed");
        break;
      }
    } else {
      dev[q] = user[q];
    }
    if (launch_fill(dev[q], len[q], fillv[q], L->stream) != hipSuccess) {
      st = fail(GG_ERR_HIP, "fill of a read-back buffer failed");
      break;
    }
  }
  if (st == GG_OK) {
    hipError_t e = launch_read(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6,
                               dev[0], dev[1], dev[2], dev[3], dev[4], dev[5], L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e == hipSuccess && where == GG_HOST)
      for (int q = 0; q < 6 && e == hipSuccess; ++q)
        if (user[q]) e = hipMemcpy(user[q], dev[q], len[q] * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = fail(GG_ERR_HIP, std::string("read: ") + hipGetErrorString(e));
  }
  if (where == GG_HOST)
    for (int q = 0; q < 6; ++q)
      if (dev[q]) (void)dev_free(L, dev[q]);
  return st;
}

gg_status gg_read(gg_lattice *L, double *rho, double *ux, double *uy, double *C, gg_where where) {
  return gg_read_impl(L, rho, ux, uy, C, nullptr, nullptr, where);
}

gg_status gg_read_populations(gg_lattice *L, double *f, double *g, gg_where where) {
  return gg_read_impl(L, nullptr, nullptr, nullptr, nullptr, f, g, where);
}

gg_status gg_diagnostics(gg_lattice *L, gg_diag *out) {
  if (!L || !out) return fail(GG_ERR_ARG, "NULL argument");
  if (!L->d_partial && L->n_aux_tiles > 0) {
    if (dev_alloc(L, (void **)&L->d_partial, (size_t)6 * L->n_aux_tiles * sizeof(double)) != hipSuccess) {
      L->d_partial = nullptr;
      return fail(GG_ERR_OOM, "diagnostics partials");
    }
  }
  GG_HIP(hipMemsetAsync(L->d_acc, 0, 8 * sizeof(double), L->stream));
  GG_HIP(launch_reduce(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6, L->d_partial,
                       L->d_acc, L->stream, REDUCE_GROUPS));
  double acc[8], flux[2 * GG_MAX_SEGMENTS];
  int64_t t = 0;
  GG_HIP(hipStreamSynchronize(L->stream));
  GG_HIP(hipMemcpy(acc, L->d_acc, sizeof(acc), hipMemcpyDeviceToHost));
  GG_HIP(hipMemcpy(flux, L->d_flux, sizeof(flux), hipMemcpyDeviceToHost));
  GG_HIP(hipMemcpy(&t, L->d_t, sizeof(t), hipMemcpyDeviceToHost));
  gg_fill_diag(L, acc, flux, t, out);
  if (out->n_nonfinite > 0)
    return fail(GG_ERR_NONFINITE, std::to_string(out->n_nonfinite) + " fluid nodes hold non-finite populations");
  return GG_OK;
}

// Snapshot layout: header, 14 population planes, fluxes.
struct SnapHeader {
  char magic[8];
  int32_t version, nx, ny, storage, pairs, pad;
  int64_t pitch, plane, t;
};

// The state from the current population layout into the other (pairs =
// the target), through the second plane set (free between calls) or a
// buffer of its size; the stream is idle.
static gg_status relayout(gg_lattice *L, bool pairs) {
  const size_t pop_bytes = (size_t)NPOP * L->plane * L->esize;
  void *dst = L->d_pop_b;
  if (!dst) {
    hipError_t e = dev_alloc(L, &dst, pop_bytes);
    if (e != hipSuccess) return fail(GG_ERR_OOM, std::string("relayout: ") + hipGetErrorString(e));
  }
  hipError_t e = launch_relayout(L->storage, L->d_pop, dst, L->plane, L->plane_elems, L->pairs,
                                 pairs, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) {  // the state stays where and as it was
    if (!L->d_pop_b) (void)dev_free(L, dst);
    return fail(GG_ERR_HIP, std::string("relayout: ") + hipGetErrorString(e));
  }
  if (L->d_pop_b) {
    std::swap(L->d_pop, L->d_pop_b);
  } else {
    GG_HIP(dev_free(L, L->d_pop));
    L->d_pop = dst;
  }
  L->pairs = pairs;
  // (captured graphs hold the old configuration)
  if (L->graph_exec) (void)hipGraphExecDestroy(L->graph_exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->graph_exec = nullptr;
  L->graph = nullptr;
  gg_drop_cde_graphs(L);
  return gg_upload_desc(L);
}

gg_status gg_set_layout(gg_lattice *L, int32_t layout) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (layout != GG_LAYOUT_PLANES && layout != GG_LAYOUT_PAIRED)
    return fail(GG_ERR_ARG, "layout must be GG_LAYOUT_PLANES or GG_LAYOUT_PAIRED");
  const bool pairs = layout == GG_LAYOUT_PAIRED;
  if (pairs == L->pairs) return GG_OK;
  GG_HIP(hipStreamSynchronize(L->stream));
  return relayout(L, pairs);
}

gg_status gg_get_layout(const gg_lattice *L, int32_t *layout) {
  if (!L || !layout) return fail(GG_ERR_ARG, "NULL argument");
  *layout = L->pairs ? GG_LAYOUT_PAIRED : GG_LAYOUT_PLANES;
  return GG_OK;
}

gg_status gg_save(gg_lattice *L, void *buf, size_t *nbytes) {
  if (!L || !nbytes) return fail(GG_ERR_ARG, "NULL argument");
  const size_t pop_bytes = (size_t)NPOP * L->plane * L->esize;
  const size_t need = sizeof(SnapHeader) + pop_bytes + 2 * GG_MAX_SEGMENTS * sizeof(double);
  if (!buf) {
    *nbytes = need;
    return GG_OK;
  }
  if (*nbytes < need) return fail(GG_ERR_ARG, "snapshot buffer too small");
  GG_HIP(hipStreamSynchronize(L->stream));
  SnapHeader h;
  std::memcpy(h.magic, "GGLBMSNP", 8);
  h.version = 2;
  h.nx = L->nx;
  h.ny = L->ny;
  h.storage = (int32_t)L->storage;
  h.pairs = L->pairs ? 1 : 0;
  h.pad = 0;
  h.pitch = L->pitch;
  h.plane = L->plane;
  GG_HIP(hipMemcpy(&h.t, L->d_t, sizeof(int64_t), hipMemcpyDeviceToHost));
  char *p = static_cast<char *>(buf);
  std::memcpy(p, &h, sizeof(h));
  GG_HIP(hipMemcpy(p + sizeof(h), L->d_pop, pop_bytes, hipMemcpyDeviceToHost));
  GG_HIP(hipMemcpy(p + sizeof(h) + pop_bytes, L->d_flux, 2 * GG_MAX_SEGMENTS * sizeof(double),
                   hipMemcpyDeviceToHost));
  *nbytes = need;
  return GG_OK;
}

gg_status gg_load(gg_lattice *L, const void *buf, size_t nbytes) {
  if (!L || !buf) return fail(GG_ERR_ARG, "NULL argument");
  const size_t pop_bytes = (size_t)NPOP * L->plane * L->esize;
  const size_t need = sizeof(SnapHeader) + pop_bytes + 2 * GG_MAX_SEGMENTS * sizeof(double);
  if (nbytes < need) return fail(GG_ERR_ARG, "snapshot too small");
  SnapHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, "GGLBMSNP", 8) != 0 || h.version != 2 || (h.pairs != 0 && h.pairs != 1))
    return fail(GG_ERR_ARG, "not a lattice snapshot");
  if (h.nx != L->nx || h.ny != L->ny || h.storage != (int32_t)L->storage ||
      h.pitch != L->pitch || h.plane != L->plane)
    return fail(GG_ERR_ARG, "snapshot belongs to a lattice of another shape or storage");
  const char *p = static_cast<const char *>(buf);
  GG_HIP(hipStreamSynchronize(L->stream));
  GG_HIP(hipMemcpy(L->d_pop, p + sizeof(h), pop_bytes, hipMemcpyHostToDevice));
  GG_HIP(hipMemcpy(L->d_flux, p + sizeof(h) + pop_bytes, 2 * GG_MAX_SEGMENTS * sizeof(double),
                   hipMemcpyHostToDevice));
  GG_HIP(hipMemcpy(L->d_t, &h.t, sizeof(int64_t), hipMemcpyHostToDevice));
  L->t = h.t;
  // a snapshot of the other population layout: into this lattice's (if
  // that fails, the lattice takes the snapshot's layout)
  if ((h.pairs != 0) != L->pairs) {
    const bool want = L->pairs;
    L->pairs = h.pairs != 0;
    gg_status st = relayout(L, want);
    if (st != GG_OK) (void)gg_upload_desc(L);
    return st;
  }
  return GG_OK;
}

gg_status gg_set_launch(gg_lattice *L, int32_t tile_x, int32_t tile_y, int32_t graph_chunk) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  const int bs = tile_x * tile_y;
  if (tile_x < 8 || (tile_x & (tile_x - 1)) || tile_y < 1 ||
      (bs != 64 && bs != 128 && bs != 256 && bs != 512))
    return fail(GG_ERR_ARG, "tile_x must be a power of two >= 8 and tile_x*tile_y one of 64, 128, 256, 512");
  if (graph_chunk < 0 || graph_chunk > 100000) return fail(GG_ERR_ARG, "graph_chunk must lie in 0..100000");
  GG_HIP(hipStreamSynchronize(L->stream));
  L->tile_x = tile_x;
  L->tile_y = tile_y;
  // even (a multiple of 4 with the two-step pass, of 8 with the four-step
  // pass): replays keep the parity and run whole passes
  const int q = L->fuse == 5 ? 8 : L->fuse >= 2 ? 4 : 2;
  L->graph_chunk = (graph_chunk + q - 1) / q * q;
  gg_drop_cde_graphs(L);
  return gg_rebuild_tiles(L);
}

gg_status gg_set_two_step(gg_lattice *L, int32_t fuse, int32_t strip_h) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (fuse < 1 || fuse > 5) return fail(GG_ERR_ARG, "fuse must be 1, 2, 3, 4 or 5");
  if (fuse == 2 && (strip_h < 1 || strip_h > 4096))
    return fail(GG_ERR_ARG, "strips walk 1..4096 rows");
  if (fuse == 2 && !L->strip_flux_ok)
    return fail(GG_ERR_ARG, "walking strips: two vertically adjacent fluid nodes link to more "
                            "than two boundary segments between them; use fuse 3 or 4");
  if (fuse >= 3 && strip_h != 6 && strip_h != 14)
    return fail(GG_ERR_ARG, "row-parallel tiles have 6 or 14 rows");
  GG_HIP(hipStreamSynchronize(L->stream));
  ++L->gen;
  if (fuse >= 2 && !L->d_pop_b) {
    const size_t pop_bytes = (size_t)NPOP * L->plane * L->esize;
    hipError_t e = dev_alloc(L, (void **)&L->d_pop_b, pop_bytes);
    if (e != hipSuccess) {
      L->d_pop_b = nullptr;
      return fail(GG_ERR_OOM, std::string("second plane set: ") + hipGetErrorString(e));
    }
    GG_HIP(hipMemset(L->d_pop_b, 0, pop_bytes));
  }
  if (fuse == 1 && L->d_pop_b) {
    GG_HIP(dev_free(L, L->d_pop_b));
    L->d_pop_b = nullptr;
  }
  L->fuse = fuse;
  if (fuse >= 2) L->strip_h = strip_h;
  const int q = fuse == 5 ? 8 : fuse >= 2 ? 4 : 2;
  L->graph_chunk = (L->graph_chunk + q - 1) / q * q;
  gg_drop_cde_graphs(L);
  gg_status st = gg_upload_desc(L);
  if (st != GG_OK) return st;
  return gg_rebuild_tiles(L);
}

gg_status gg_info(const gg_lattice *L, int64_t *n_fluid, int64_t *n_tiles, int64_t *t) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (n_fluid) *n_fluid = L->n_fluid;
  if (n_tiles) *n_tiles = L->n_tiles;
  if (t) *t = L->t;
  return GG_OK;
}

// Device buffers of one adjoint run, freed on every exit path.
struct AdjointBuffers {
  const gg_lattice *L;
  std::vector<void *> ptrs;
  explicit AdjointBuffers(const gg_lattice *lat) : L(lat) {}
  ~AdjointBuffers() {
    for (void *p : ptrs)
      if (p) (void)dev_free(L, p);
  }
  hipError_t alloc(void **p, size_t bytes) {
    *p = nullptr;
    hipError_t e = dev_alloc(L, p, bytes);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

gg_status gg_adjoint(gg_lattice *L, int64_t n, int64_t s, const double *weight,
                     const double *target, const int32_t *r_box, double *d_R, gg_grads *out) {
  if (L && special_boundaries(L))
    return fail(GG_ERR_STATE, "the adjoint does not cover pressure boundaries or the paper's walls");
  if (!L || !weight || !target || !out) return fail(GG_ERR_ARG, "NULL argument");
  if (n < 1) return fail(GG_ERR_ARG, "n_steps must be positive");
  if (s < 0) return fail(GG_ERR_ARG, "ckpt_every must be non-negative");
  int32_t box[4] = {0, 0, 0, 0};
  if (r_box) {
    for (int k = 0; k < 4; ++k) box[k] = r_box[k];
    if (box[0] < 0 || box[1] < 0 || box[2] < 1 || box[3] < 1 || box[0] + box[2] > L->nx ||
        box[1] + box[3] > L->ny)
      return fail(GG_ERR_ARG, "r_box must lie inside the lattice");
    if (!d_R) return fail(GG_ERR_ARG, "d_R is NULL while r_box is given");
  }
  gg_status st = check_segments(L);
  if (st != GG_OK) return st;
  if (s == 0) s = (int64_t)std::ceil(std::sqrt((double)n));
  s = std::min<int64_t>(s, n);
  const int64_t K = (n + s - 1) / s;
  const size_t pop_bytes = (size_t)NPOP * L->plane * L->esize;
  const size_t tsz = L->storage == GG_F64 ? 8 : 4;
  const size_t slot = (size_t)7 * L->plane * tsz;
  const size_t lam_bytes = (size_t)5 * L->plane * sizeof(double);
  const size_t nxy = (size_t)L->nx * L->ny;
  // Where the lattice steps in two-step passes, the adjoint steps go in
  // pairs too (the adjoint of the pass) over 62 x 6 tiles of all fluid
  // nodes, flagged where the tile or its halo touches a segment.
  std::vector<Tile> adj_tiles, adj_unused;
  const bool adj_pass = L->fuse >= 3;
  if (adj_pass) build_strips(L, 6, 0, false, adj_tiles, adj_unused, true);
  const int na = std::max({L->n_aux_tiles, (int)adj_tiles.size(), 1});

  AdjointBuffers B(L);
  void *ckpt, *scr_pop, *scr_desc, *scr_t, *scr_flux, *tape, *lam0, *lam1, *wdev, *tdev, *dRdev,
      *dcin, *pw, *pl;
  const size_t need = (size_t)K * pop_bytes + pop_bytes + (size_t)s * slot + 2 * lam_bytes;
  if (B.alloc(&ckpt, (size_t)K * pop_bytes) != hipSuccess || B.alloc(&scr_pop, pop_bytes) != hipSuccess ||
      B.alloc(&scr_desc, sizeof(LatDesc)) != hipSuccess || B.alloc(&scr_t, sizeof(int64_t)) != hipSuccess ||
      B.alloc(&scr_flux, 2 * GG_MAX_SEGMENTS * sizeof(double)) != hipSuccess ||
      B.alloc(&tape, (size_t)s * slot) != hipSuccess || B.alloc(&lam0, lam_bytes) != hipSuccess ||
      B.alloc(&lam1, lam_bytes) != hipSuccess || B.alloc(&wdev, nxy * sizeof(double)) != hipSuccess ||
      B.alloc(&tdev, nxy * sizeof(double)) != hipSuccess ||
      B.alloc(&dRdev, std::max<size_t>(1, (size_t)box[2] * box[3]) * sizeof(double)) != hipSuccess ||
      B.alloc(&dcin, GG_MAX_SEGMENTS * sizeof(double)) != hipSuccess ||
      B.alloc(&pw, na * sizeof(double)) != hipSuccess || B.alloc(&pl, na * sizeof(double)) != hipSuccess)
    return fail(GG_ERR_OOM, "adjoint needs about " + std::to_string(need >> 20) +
                                " MiB of device memory (checkpoints, tape, adjoint fields)");
  void *d_adj_tiles = nullptr;
  if (adj_pass && !adj_tiles.empty()) {
    if (B.alloc(&d_adj_tiles, adj_tiles.size() * sizeof(Tile)) != hipSuccess)
      return fail(GG_ERR_OOM, "adjoint tile list");
    GG_HIP(hipMemcpy(d_adj_tiles, adj_tiles.data(), adj_tiles.size() * sizeof(Tile),
                     hipMemcpyHostToDevice));
  }
  GG_HIP(hipMemset(lam0, 0, lam_bytes));
  GG_HIP(hipMemset(lam1, 0, lam_bytes));
  GG_HIP(hipMemset(dRdev, 0, std::max<size_t>(1, (size_t)box[2] * box[3]) * sizeof(double)));
  GG_HIP(hipMemset(dcin, 0, GG_MAX_SEGMENTS * sizeof(double)));
  GG_HIP(hipMemset(pw, 0, na * sizeof(double)));
  GG_HIP(hipMemset(pl, 0, na * sizeof(double)));
  GG_HIP(hipMemset(scr_flux, 0, 2 * GG_MAX_SEGMENTS * sizeof(double)));
  GG_HIP(hipMemcpy(wdev, weight, nxy * sizeof(double), hipMemcpyHostToDevice));
  GG_HIP(hipMemcpy(tdev, target, nxy * sizeof(double), hipMemcpyHostToDevice));

  // forward pass with checkpoints
  const int64_t t0 = L->t;
  for (int64_t k = 0; k < K; ++k) {
    GG_HIP(hipMemcpyAsync((char *)ckpt + (size_t)k * pop_bytes, L->d_pop, pop_bytes,
                          hipMemcpyDeviceToDevice, L->stream));
    st = gg_step(L, std::min<int64_t>(s, n - k * s));
    if (st != GG_OK) return st;
  }
  GG_HIP(launch_seed(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6, (const double *)wdev,
                     (const double *)tdev, lam0, (double *)pl, L->stream));

  // recomputation copy of the lattice: its own state, counter and fluxes
  // (and, where the lattice steps in row-parallel two-step passes, its own
  // second plane set: the recomputation then runs in passes too)
  void *scr_pop_b = nullptr;
  const bool rec_pass = pass_ok(L) && L->fuse >= 3 &&
                        B.alloc(&scr_pop_b, pop_bytes) == hipSuccess;
  (void)hipGetLastError();
  LatDesc hs = L->h;
  hs.pop = scr_pop;
  hs.pop_b = scr_pop_b;
  hs.t = (int64_t *)scr_t;
  hs.flux = (double *)scr_flux;
  GG_HIP(hipMemcpy(scr_desc, &hs, sizeof(hs), hipMemcpyHostToDevice));
  const LatDesc *sd = (const LatDesc *)scr_desc;
  const int block = L->tile_x * L->tile_y;
  const int txs = ilog2(L->tile_x);
  void *lam[2] = {lam0, lam1};
  int cur = 0;
  // Backward sweep, segment by segment from the last checkpoint: the
  // recomputation of a segment (from its checkpoint, writing the tape) and
  // the adjoint steps over it. With a second tape (when it fits), the
  // recomputation of segment k - 1 runs on a stream of its own while the
  // adjoint steps of segment k run on the lattice's stream: two
  // independent kernels that each leave part of the GPU idle on their own.
  void *tape2 = nullptr;
  const bool overlap = K > 1 && B.alloc(&tape2, (size_t)s * slot) == hipSuccess;
  (void)hipGetLastError();  // a failed allocation only means no overlap
  void *tapes[2] = {tape, overlap ? tape2 : tape};
  struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // ready 0/1, free 0/1
    ~SideStream() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
      for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    }
  } side;
  hipStream_t rs = L->stream;
  if (overlap) {
    GG_HIP(hipStreamCreateWithFlags(&side.s, hipStreamNonBlocking));
    for (hipEvent_t &e : side.ev) GG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    rs = side.s;
    GG_HIP(hipEventRecord(side.ev[0], L->stream));  // the seed and lambda set-up
    GG_HIP(hipStreamWaitEvent(rs, side.ev[0], 0));
  }
  auto recompute = [&](int64_t k, void *tp) -> hipError_t {
    const int64_t tk = t0 + k * s;
    const int64_t nk = std::min<int64_t>(s, n - k * s);
    hipError_t e = hipMemcpyAsync(scr_pop, (char *)ckpt + (size_t)k * pop_bytes, pop_bytes,
                                  hipMemcpyDeviceToDevice, rs);
    // (the recomputation's counter stays at tk: step j runs with dt = j)
    if (e == hipSuccess) e = launch_set_counter((int64_t *)scr_t, tk, rs);
    int64_t j = 0;
    auto single = [&]() {
      e = launch_step_tape(L->storage, L->pairs, block, ((tk + j) & 1) != 0, sd, L->d_tiles, L->n_tiles, txs,
                           (int)j, (char *)tp + (size_t)j * slot, rs);
      ++j;
    };
    if (rec_pass) {
      // an odd first step alone, then pairs of passes (four steps, ending
      // in the first plane set) that tape both of their steps; the
      // boundary tiles' kernel runs before the others on the same stream
      if (((tk + j) & 1) && j < nk && e == hipSuccess) single();
      for (; nk - j >= 4 && e == hipSuccess; j += 4)
        for (int q = 0; q < 2 && e == hipSuccess; ++q) {
          char *t0p = (char *)tp + (size_t)(j + 2 * q) * slot;
          char *t1p = t0p + slot;
          const int dt = (int)(j + 2 * q);
          if (L->fuse == 4) {
            e = launch_tile2(L->storage, L->pairs, true, L->strip_h, sd, L->d_strips, L->n_strips, q, dt, rs,
                             false, t0p, t1p);
          } else {
            if (L->n_seg_strips > 0)
              e = launch_tile2(L->storage, L->pairs, true, 2, sd, L->d_seg_strips, L->n_seg_strips, q, dt, rs,
                               false, t0p, t1p);
            if (e == hipSuccess)
              e = launch_tile2(L->storage, L->pairs, false, L->strip_h, sd, L->d_strips, L->n_strips, q, dt,
                               rs, false, t0p, t1p);
          }
        }
    }
    while (j < nk && e == hipSuccess) single();
    return e;
  };
  GG_HIP(recompute(K - 1, tapes[(K - 1) & 1]));
  if (overlap) GG_HIP(hipEventRecord(side.ev[(K - 1) & 1], rs));
  for (int64_t k = K - 1; k >= 0; --k) {
    const int64_t tk = t0 + k * s;
    const int64_t nk = std::min<int64_t>(s, n - k * s);
    const int b = (int)(k & 1);
    if (overlap && k > 0) {
      // segment k - 1 into the other tape, once the adjoint of segment
      // k + 1 (which read it) is done
      if (k + 1 <= K - 1) GG_HIP(hipStreamWaitEvent(rs, side.ev[2 + (1 - b)], 0));
      GG_HIP(recompute(k - 1, tapes[1 - b]));
      GG_HIP(hipEventRecord(side.ev[1 - b], rs));
    }
    if (overlap) GG_HIP(hipStreamWaitEvent(L->stream, side.ev[b], 0));
    for (int64_t j = nk - 1; j >= 0;) {
      const char *tj = (const char *)tapes[b] + (size_t)j * slot;
      if (d_adj_tiles && j >= 1) {
        GG_HIP(launch_adjoint2(L->storage, 6, L->d_desc, (const Tile *)d_adj_tiles,
                               (int)adj_tiles.size(), tk + j, lam[cur], lam[1 - cur], tj, tj - slot,
                               r_box ? (double *)dRdev : nullptr, box, (double *)dcin,
                               (double *)pw, L->stream));
        j -= 2;
      } else {
        GG_HIP(launch_adjoint(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6, tk + j,
                              lam[cur], lam[1 - cur], tj, r_box ? (double *)dRdev : nullptr, box,
                              (double *)dcin, (double *)pw, L->stream));
        j -= 1;
      }
      cur = 1 - cur;
    }
    if (overlap) {
      GG_HIP(hipEventRecord(side.ev[2 + b], L->stream));
    } else if (k > 0) {
      GG_HIP(recompute(k - 1, tapes[0]));
    }
  }
  GG_HIP(hipStreamSynchronize(L->stream));
  std::vector<double> hpw(na), hpl(na);
  GG_HIP(hipMemcpy(hpw.data(), pw, na * sizeof(double), hipMemcpyDeviceToHost));
  GG_HIP(hipMemcpy(hpl.data(), pl, na * sizeof(double), hipMemcpyDeviceToHost));
  double dom = 0.0, loss = 0.0;
  for (int k = 0; k < na; ++k) {
    dom += hpw[k];
    loss += hpl[k];
  }
  std::memset(out, 0, sizeof(*out));
  out->loss = loss;
  GG_HIP(hipMemcpy(out->d_c_in, dcin, GG_MAX_SEGMENTS * sizeof(double), hipMemcpyDeviceToHost));
  out->d_omega_g = dom;
  out->d_D = dom * (-1.0 / (L->tau_g * L->tau_g * L->cs2g));
  out->ckpt_every = s;
  out->n_checkpoints = K;
  if (r_box)
    GG_HIP(hipMemcpy(d_R, dRdev, (size_t)box[2] * box[3] * sizeof(double), hipMemcpyDeviceToHost));
  return GG_OK;
}

// ---------------------------------------------------------------------------
// Batched launch
// ---------------------------------------------------------------------------

struct gg_batch {
  std::vector<gg_lattice *> lats;
  gg_storage storage = GG_F32;
  bool pairs = true;  // the members' population layout
  hipStream_t stream = nullptr, cap_stream = nullptr;
  LatDesc *d_descs = nullptr;
  Tile *d_tiles[2] = {nullptr, nullptr};  // lattices at even / odd t at creation
  int n_tiles[2] = {0, 0};
  int tile_x = 64, tile_y = 4, persist = 0, chunk = 0;
  int64_t steps = 0;  // steps taken by the batch
  int64_t n_fluid = 0;
  std::vector<int64_t> t_created;  // member times when the batch was made
  // member configuration generations and second plane sets as copied into
  // the batch's descriptors at creation
  std::vector<uint64_t> gen_created;
  std::vector<uint8_t> pop_b_created;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // two-step pass over all members (fuse 3 or 4, tiles of `rows` rows);
  // fuse 5: four-step passes over the members' 58 x 6 tiles (the lists
  // with 4), two-step passes as fuse 3 for the last four steps of 8k + 4
  int fuse = 1, rows = 6;
  Tile *d_strips = nullptr, *d_seg_strips = nullptr;
  int n_strips = 0, n_seg_strips = 0;
  Tile *d_strips4 = nullptr, *d_seg_strips4 = nullptr;
  int n_strips4 = 0, n_seg_strips4 = 0;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

static void batch_free(gg_batch *B) {
  if (B->graph_exec) (void)hipGraphExecDestroy(B->graph_exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->d_descs) (void)hipFree(B->d_descs);
  for (int g = 0; g < 2; ++g)
    if (B->d_tiles[g]) (void)hipFree(B->d_tiles[g]);
  if (B->d_strips) (void)hipFree(B->d_strips);
  if (B->d_seg_strips) (void)hipFree(B->d_seg_strips);
  if (B->d_strips4) (void)hipFree(B->d_strips4);
  if (B->d_seg_strips4) (void)hipFree(B->d_seg_strips4);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  if (B->side) (void)hipStreamDestroy(B->side);
  if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
  if (B->ev_join) (void)hipEventDestroy(B->ev_join);
  delete B;
}

// The batch runs two-step passes when they are on, the members sit at even
// steps (the batch's step count plus the parity of the group they were all
// in at creation) and n is a multiple of 4 (pairs of passes end in the
// members' first plane sets).
static bool batch_passes(const gg_batch *B, int64_t s0, int64_t n) {
  return B->fuse >= 3 && n % 4 == 0 && ((s0 + (B->n_tiles[0] > 0 ? 0 : 1)) & 1) == 0;
}

// n steps of the batch on `st` (group parity from the batch's step count)
// The batch's copies of the members' descriptors still describe them: no
// member was reconfigured (buffers freed or reallocated, parameters
// changed) since the batch was made.
static gg_status batch_check_members(const gg_batch *B) {
  for (size_t k = 0; k < B->lats.size(); ++k)
    if (B->lats[k]->gen != B->gen_created[k])
      return fail(GG_ERR_STATE, "batch member " + std::to_string(k) +
                                    " was reconfigured after the batch was made; make a new batch");
  return GG_OK;
}

static hipError_t batch_launch(gg_batch *B, int64_t s0, int64_t n, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (batch_passes(B, s0, n)) {
    // one pass over all members: the boundary tiles' kernel on the side
    // stream (forked and joined) when both lists hold tiles
    auto pass = [&](bool four, int dir, int dt) -> hipError_t {
      const Tile *main = four ? B->d_strips4 : B->d_strips;
      const Tile *segl = four ? B->d_seg_strips4 : B->d_seg_strips;
      const int nm = four ? B->n_strips4 : B->n_strips;
      const int ns = four ? B->n_seg_strips4 : B->n_seg_strips;
      // (the boundary list holds 2-row tiles; fuse 4's one list, run with
      // the boundary rules, holds tiles of `rows` rows)
      auto run = [&](bool seg, bool seg_list, const Tile *list, int nl, hipStream_t s) {
        return four ? launch_tile4(B->storage, B->pairs, seg, B->d_descs, list, nl, dir, dt, s)
                    : launch_tile2(B->storage, B->pairs, seg, seg_list ? 2 : B->rows, B->d_descs, list,
                                   nl, dir, dt, s);
      };
      if (B->fuse == 4) return run(true, false, main, nm, st);
      const bool fork = ns > 0 && nm > 0;
      hipError_t r = hipSuccess;
      if (fork) {
        r = hipEventRecord(B->ev_fork, st);
        if (r == hipSuccess) r = hipStreamWaitEvent(B->side, B->ev_fork, 0);
        if (r == hipSuccess) r = run(true, true, segl, ns, B->side);
        if (r == hipSuccess) r = hipEventRecord(B->ev_join, B->side);
      } else if (ns > 0) {
        r = run(true, true, segl, ns, st);
      }
      if (r == hipSuccess) r = run(false, false, main, nm, st);
      if (fork && r == hipSuccess) r = hipStreamWaitEvent(st, B->ev_join, 0);
      return r;
    };
    // fuse 5: four-step passes in pairs, then the last four steps of a
    // run of 8k + 4 in two two-step passes
    const int64_t p4 = B->fuse == 5 ? n / 8 * 2 : 0;
    for (int64_t k = 0; k < p4 && e == hipSuccess; ++k) e = pass(true, (int)(k & 1), (int)(4 * k));
    for (int64_t k = 0; k < (n - 4 * p4) / 2 && e == hipSuccess; ++k)
      e = pass(false, (int)(k & 1), (int)(4 * p4 + 2 * k));
  } else {
    const int block = B->tile_x * B->tile_y;
    const int txs = ilog2(B->tile_x);
    for (int64_t dt = 0; dt < n && e == hipSuccess; ++dt)
      for (int g = 0; g < 2 && e == hipSuccess; ++g)
        if (B->n_tiles[g] > 0)
          e = launch_step(B->storage, B->pairs, block, ((s0 + dt + g) & 1) != 0, B->d_descs, B->d_tiles[g],
                          B->n_tiles[g], txs, (int)dt, st, B->persist);
  }
  if (e == hipSuccess) e = launch_advance(B->d_descs, (int)B->lats.size(), n, st);
  return e;
}

static gg_status batch_autotune(gg_lattice *const *lats, int32_t n, int32_t graph_chunk,
                                gg_batch **out);

gg_status gg_batch_create(gg_lattice *const *lats, int32_t n, int32_t tile_x, int32_t tile_y,
                          int32_t persist, int32_t graph_chunk, gg_batch **out) {
  if (!out || !lats || n < 1) return fail(GG_ERR_ARG, "need at least one lattice");
  *out = nullptr;
  if (persist == GG_AUTOTUNE) return batch_autotune(lats, n, graph_chunk, out);
  if (tile_x == 0 && tile_y == 0) {
    tile_x = 64;
    tile_y = 4;
  }
  const int bs = tile_x * tile_y;
  if (tile_x < 8 || (tile_x & (tile_x - 1)) || tile_y < 1 ||
      (bs != 64 && bs != 128 && bs != 256 && bs != 512))
    return fail(GG_ERR_ARG, "tile_x must be a power of two >= 8 and tile_x*tile_y one of 64, 128, 256, 512");
  if (persist < 0 || graph_chunk < 0 || graph_chunk > 100000) return fail(GG_ERR_ARG, "bad persist or graph_chunk");
  for (int k = 0; k < n; ++k) {
    if (!lats[k]) return fail(GG_ERR_ARG, "NULL lattice in the batch");
    if (lats[k]->storage != lats[0]->storage) return fail(GG_ERR_ARG, "batch members must share the storage type");
    if (lats[k]->pairs != lats[0]->pairs)
      return fail(GG_ERR_ARG, "batch members must share the population layout");
    if (lats[k]->stream != lats[0]->stream) return fail(GG_ERR_ARG, "batch members must share the HIP stream");
    for (int j = 0; j < k; ++j)
      if (lats[j] == lats[k]) return fail(GG_ERR_ARG, "a lattice appears twice in the batch");
    gg_status st = check_segments(lats[k]);
    if (st != GG_OK) return st;
    if (special_boundaries(lats[k]))
      return fail(GG_ERR_STATE, "batch members may not have pressure boundaries or the paper's walls");
  }
  gg_batch *B = new gg_batch();
  B->lats.assign(lats, lats + n);
  B->storage = lats[0]->storage;
  B->pairs = lats[0]->pairs;
  B->stream = lats[0]->stream;
  B->tile_x = tile_x;
  B->tile_y = tile_y;
  B->persist = persist;
  B->chunk = (graph_chunk + 1) / 2 * 2;
  std::vector<LatDesc> descs(n);
  std::vector<Tile> tiles[2];
  for (int k = 0; k < n; ++k) {
    descs[k] = lats[k]->h;
    build_tiles(lats[k], tile_x, tile_y, k, tiles[lats[k]->t & 1]);
    B->n_fluid += lats[k]->n_fluid;
    B->t_created.push_back(lats[k]->t);
    B->gen_created.push_back(lats[k]->gen);
    B->pop_b_created.push_back(descs[k].pop_b != nullptr);
  }
  hipError_t e = hipStreamSynchronize(B->stream);
  if (e == hipSuccess) e = hipMalloc(&B->d_descs, n * sizeof(LatDesc));
  if (e == hipSuccess) e = hipMemcpy(B->d_descs, descs.data(), n * sizeof(LatDesc), hipMemcpyHostToDevice);
  for (int g = 0; g < 2 && e == hipSuccess; ++g) {
    B->n_tiles[g] = (int)tiles[g].size();
    if (tiles[g].empty()) continue;
    e = hipMalloc(&B->d_tiles[g], tiles[g].size() * sizeof(Tile));
    if (e == hipSuccess)
      e = hipMemcpy(B->d_tiles[g], tiles[g].data(), tiles[g].size() * sizeof(Tile), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    batch_free(B);
    return fail(GG_ERR_HIP, std::string("batch set-up: ") + hipGetErrorString(e));
  }
  *out = B;
  return GG_OK;
}

// Library-side autotuner of a batch's launch form: each candidate (single
// steps over tiles of 64 x 4, 32 x 8 or 128 x 2 nodes; two-step passes over
// tiles of 6 or 14 rows with the boundary tiles in their own kernel, or of 6
// rows in the one kernel, when every member has its second plane set and
// all sit at steps of one parity) advances the members 4 + 16 steps, the 16
// timed with HIP events on their stream; the members' states, step counts
// and boundary fluxes are copied aside on the device first and put back
// after each candidate, so tuning leaves them as they were.
static gg_status batch_autotune(gg_lattice *const *lats, int32_t n, int32_t graph_chunk,
                                gg_batch **out) {
  for (int k = 0; k < n; ++k)
    if (!lats[k]) return fail(GG_ERR_ARG, "NULL lattice in the batch");
  hipStream_t st = lats[0]->stream;
  std::vector<size_t> off(n + 1, 0);
  for (int k = 0; k < n; ++k)
    off[k + 1] = off[k] + (size_t)NPOP * lats[k]->plane * lats[k]->esize +
                 2 * GG_MAX_SEGMENTS * sizeof(double) + sizeof(int64_t);
  void *save = nullptr;
  if (hipMalloc(&save, off[n]) != hipSuccess) return fail(GG_ERR_OOM, "autotune: state copies");
  struct Free {
    void *p;
    ~Free() { (void)hipFree(p); }
  } fr{save};
  std::vector<int64_t> t0(n);
  auto copy = [&](bool back) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int k = 0; k < n && e == hipSuccess; ++k) {
      gg_lattice *L = lats[k];
      char *p = (char *)save + off[k];
      const size_t pb = (size_t)NPOP * L->plane * L->esize;
      const size_t fb = 2 * GG_MAX_SEGMENTS * sizeof(double);
      void *d[3] = {L->d_pop, L->d_flux, L->d_t};
      void *h[3] = {p, p + pb, p + pb + fb};
      const size_t sz[3] = {pb, fb, sizeof(int64_t)};
      for (int q = 0; q < 3 && e == hipSuccess; ++q)
        e = hipMemcpyAsync(back ? d[q] : h[q], back ? h[q] : d[q], sz[q], hipMemcpyDeviceToDevice, st);
      if (back) L->t = t0[k];
    }
    return e;
  };
  for (int k = 0; k < n; ++k) t0[k] = lats[k]->t;
  GG_HIP(copy(false));
  bool passes = true;
  for (int k = 0; k < n; ++k)
    passes = passes && lats[k]->d_pop_b && ((lats[k]->t ^ lats[0]->t) & 1) == 0;
  struct Cand {
    int tx, ty, fuse, rows;
  };
  std::vector<Cand> cands = {{64, 4, 1, 6}, {32, 8, 1, 6}, {128, 2, 1, 6}};
  if (passes) {
    cands.push_back({64, 4, 3, 6});
    cands.push_back({64, 4, 3, 14});
    cands.push_back({64, 4, 4, 6});
    cands.push_back({64, 4, 4, 14});
    cands.push_back({64, 4, 5, 6});
  }
  hipEvent_t a = nullptr, b = nullptr;
  GG_HIP(hipEventCreate(&a));
  GG_HIP(hipEventCreate(&b));
  double best_ms = 1e300;
  Cand best = cands[0];
  gg_status st_all = GG_OK;
  for (const Cand &c : cands) {
    gg_batch *B = nullptr;
    gg_status s = gg_batch_create(lats, n, c.tx, c.ty, 0, graph_chunk, &B);
    if (s == GG_OK && c.fuse >= 3) s = gg_batch_set_two_step(B, c.fuse, c.rows);
    float ms = 0.0f;
    if (s == GG_OK) s = gg_batch_step(B, 4);
    if (s == GG_OK && hipEventRecord(a, st) != hipSuccess) s = fail(GG_ERR_HIP, "autotune event");
    if (s == GG_OK) s = gg_batch_step(B, 16);
    if (s == GG_OK && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                       hipEventElapsedTime(&ms, a, b) != hipSuccess))
      s = fail(GG_ERR_HIP, "autotune timing");
    if (B) gg_batch_destroy(B);
    if (copy(true) != hipSuccess) {
      st_all = fail(GG_ERR_HIP, "autotune: restoring the members' states");
      break;
    }
    if (s != GG_OK) continue;  // a candidate the members do not allow
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st_all != GG_OK) return st_all;
  GG_HIP(hipStreamSynchronize(st));
  gg_status s = gg_batch_create(lats, n, best.tx, best.ty, 0, graph_chunk, out);
  if (s == GG_OK && best.fuse >= 3) s = gg_batch_set_two_step(*out, best.fuse, best.rows);
  if (s != GG_OK && *out) {
    gg_batch_destroy(*out);
    *out = nullptr;
  }
  return s;
}

gg_status gg_batch_form(const gg_batch *B, int32_t *tile_x, int32_t *tile_y, int32_t *persist,
                        int32_t *fuse, int32_t *rows) {
  if (!B) return fail(GG_ERR_ARG, "batch is NULL");
  if (tile_x) *tile_x = B->tile_x;
  if (tile_y) *tile_y = B->tile_y;
  if (persist) *persist = B->persist;
  if (fuse) *fuse = B->fuse;
  if (rows) *rows = B->rows;
  return GG_OK;
}

gg_status gg_batch_step(gg_batch *B, int64_t n) {
  if (!B) return fail(GG_ERR_ARG, "batch is NULL");
  if (n < 0) return fail(GG_ERR_ARG, "n must be non-negative");
  // members stepped on their own since the batch was created would no
  // longer sit in their parity group
  for (size_t k = 0; k < B->lats.size(); ++k) {
    const gg_lattice *L = B->lats[k];
    if (L->t - B->t_created[k] != B->steps)
      return fail(GG_ERR_STATE, "batch member " + std::to_string(k) +
                                    " was stepped, loaded or re-initialised outside the batch");
    if (special_boundaries(L))
      return fail(GG_ERR_STATE, "batch member " + std::to_string(k) +
                                    " has a pressure boundary or the paper's walls");
  }
  gg_status cst = batch_check_members(B);
  if (cst != GG_OK) return cst;
  int64_t left = n;
  const int K = B->chunk;
  if (B->fuse >= 3) {
    // all members in one parity group; s_even: a batch step count at which
    // they sit at even steps
    const int64_t s_even = B->n_tiles[0] > 0 ? 0 : 1;
    if (((B->steps + s_even) & 1) && left > 0) {  // to even member steps
      GG_HIP(batch_launch(B, B->steps, 1, B->stream));
      B->steps += 1;
      left -= 1;
    }
    if (K > 0 && left >= K) {
      if (!B->graph_exec) {  // K is a multiple of 4: passes only
        GG_HIP(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = batch_launch(B, s_even, K, B->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(B->cap_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return fail(GG_ERR_HIP, std::string("batch graph capture: ") +
                                      hipGetErrorString(e != hipSuccess ? e : e2));
        }
        B->graph = g;
        GG_HIP(hipGraphInstantiate(&B->graph_exec, B->graph, nullptr, nullptr, 0));
      }
      while (left >= K) {
        GG_HIP(hipGraphLaunch(B->graph_exec, B->stream));
        left -= K;
        B->steps += K;
      }
    }
    const int64_t quads = left / 4 * 4;
    if (quads > 0) {
      GG_HIP(batch_launch(B, B->steps, quads, B->stream));
      B->steps += quads;
      left -= quads;
    }
    if (left > 0) {
      GG_HIP(batch_launch(B, B->steps, left, B->stream));
      B->steps += left;
    }
    for (gg_lattice *L : B->lats) L->t += n;
    return GG_OK;
  }
  if (K > 0 && (B->steps & 1) && left >= K + 1) {  // replays start on an even batch step
    GG_HIP(batch_launch(B, B->steps, 1, B->stream));
    B->steps += 1;
    left -= 1;
  }
  if (K > 0 && !(B->steps & 1) && left >= K) {
    if (!B->graph_exec) {
      GG_HIP(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = batch_launch(B, 0, K, B->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(B->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(GG_ERR_HIP, std::string("batch graph capture: ") +
                                    hipGetErrorString(e != hipSuccess ? e : e2));
      }
      B->graph = g;
      GG_HIP(hipGraphInstantiate(&B->graph_exec, B->graph, nullptr, nullptr, 0));
    }
    while (left >= K) {
      GG_HIP(hipGraphLaunch(B->graph_exec, B->stream));
      left -= K;
      B->steps += K;
    }
  }
  if (left > 0) {
    GG_HIP(batch_launch(B, B->steps, left, B->stream));
    B->steps += left;
  }
  for (gg_lattice *L : B->lats) L->t += n;
  return GG_OK;
}

gg_status gg_batch_set_two_step(gg_batch *B, int32_t fuse, int32_t rows) {
  if (!B) return fail(GG_ERR_ARG, "batch is NULL");
  if (fuse != 1 && fuse != 3 && fuse != 4 && fuse != 5)
    return fail(GG_ERR_ARG, "fuse must be 1, 3, 4 or 5");
  for (size_t k = 0; k < B->lats.size() && fuse == 5; ++k) {
    const gg_lattice *L = B->lats[k];
    if ((L->p.periodic_x && L->nx < 4) || (L->p.periodic_y && L->ny < 4))
      return fail(GG_ERR_ARG, "member " + std::to_string(k) +
                                  ": the four-step pass needs periodic axes of 4 nodes or more");
  }
  if (fuse >= 3 && rows != 6 && rows != 14) return fail(GG_ERR_ARG, "tiles have 6 or 14 rows");
  if (fuse >= 3 && B->n_tiles[0] > 0 && B->n_tiles[1] > 0)
    return fail(GG_ERR_STATE, "the two-step pass needs all members at steps of one parity");
  gg_status cst = batch_check_members(B);
  if (cst != GG_OK) return cst;
  for (size_t k = 0; k < B->lats.size() && fuse >= 3; ++k)
    if (!B->lats[k]->d_pop_b || !B->pop_b_created[k])
      return fail(GG_ERR_STATE, "member " + std::to_string(k) +
                                    " has no second plane set (gg_set_two_step with fuse >= 2)");
  GG_HIP(hipStreamSynchronize(B->stream));
  if (B->graph_exec) (void)hipGraphExecDestroy(B->graph_exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->graph_exec = nullptr;
  B->graph = nullptr;
  if (B->d_strips) (void)hipFree(B->d_strips);
  if (B->d_seg_strips) (void)hipFree(B->d_seg_strips);
  B->d_strips = B->d_seg_strips = nullptr;
  B->n_strips = B->n_seg_strips = 0;
  if (B->d_strips4) (void)hipFree(B->d_strips4);
  if (B->d_seg_strips4) (void)hipFree(B->d_seg_strips4);
  B->d_strips4 = B->d_seg_strips4 = nullptr;
  B->n_strips4 = B->n_seg_strips4 = 0;
  B->fuse = fuse;
  B->rows = rows;
  if (fuse == 1) return GG_OK;
  std::vector<Tile> sv, ss, sv4, ss4;
  for (size_t k = 0; k < B->lats.size(); ++k) {
    build_strips(B->lats[k], rows, (int)k, fuse != 4, sv, ss);
    if (fuse == 5) build_strips(B->lats[k], 6, (int)k, true, sv4, ss4, 2, 58);
  }
  B->n_strips4 = (int)sv4.size();
  B->n_seg_strips4 = (int)ss4.size();
  if (!sv4.empty()) {
    GG_HIP(hipMalloc(&B->d_strips4, sv4.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(B->d_strips4, sv4.data(), sv4.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  if (!ss4.empty()) {
    GG_HIP(hipMalloc(&B->d_seg_strips4, ss4.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(B->d_seg_strips4, ss4.data(), ss4.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  B->n_strips = (int)sv.size();
  B->n_seg_strips = (int)ss.size();
  if (!sv.empty()) {
    GG_HIP(hipMalloc(&B->d_strips, sv.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(B->d_strips, sv.data(), sv.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  if (!ss.empty()) {
    GG_HIP(hipMalloc(&B->d_seg_strips, ss.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(B->d_seg_strips, ss.data(), ss.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  if (!B->side) {
    GG_HIP(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
    GG_HIP(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
    GG_HIP(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
  }
  // replays run whole passes: a multiple of 4 steps, of 8 with fuse 5
  const int q = fuse == 5 ? 8 : 4;
  B->chunk = (B->chunk + q - 1) / q * q;
  return GG_OK;
}

gg_status gg_batch_info(const gg_batch *B, int64_t *n_tiles, int64_t *n_fluid) {
  if (!B) return fail(GG_ERR_ARG, "batch is NULL");
  if (n_tiles) *n_tiles = (int64_t)B->n_tiles[0] + B->n_tiles[1];
  if (n_fluid) *n_fluid = B->n_fluid;
  return GG_OK;
}

void gg_batch_destroy(gg_batch *B) {
  if (!B) return;
  (void)hipStreamSynchronize(B->stream);
  batch_free(B);
}

gg_status gg_step_timed(gg_lattice *L, int64_t n, double *ms_even, double *ms_odd) {
  if (L && special_boundaries(L))
    return fail(GG_ERR_STATE, "timed steps do not cover pressure boundaries or the paper's walls");
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (n < 1) return fail(GG_ERR_ARG, "n must be positive");
  gg_status st = check_segments(L);
  if (st != GG_OK) return st;
  const int block = L->tile_x * L->tile_y;
  const int txs = ilog2(L->tile_x);
  std::vector<hipEvent_t> ev(2 * (size_t)n, nullptr);
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < ev.size() && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
  const int64_t t0 = L->t;
  for (int64_t dt = 0; dt < n && e == hipSuccess; ++dt) {
    e = hipEventRecord(ev[2 * dt], L->stream);
    if (e == hipSuccess)
      e = launch_step(L->storage, L->pairs, block, ((t0 + dt) & 1) != 0, L->d_desc, L->d_tiles,
                      L->n_tiles, txs, (int)dt, L->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * dt + 1], L->stream);
  }
  if (e == hipSuccess) e = launch_advance(L->d_desc, 1, n, L->stream);
  if (e == hipSuccess) L->t += n;
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  double tot[2] = {0.0, 0.0};
  int64_t cnt[2] = {0, 0};
  for (int64_t dt = 0; dt < n && e == hipSuccess; ++dt) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, ev[2 * dt], ev[2 * dt + 1]);
    const int par = (int)((t0 + dt) & 1);
    tot[par] += ms;
    cnt[par] += 1;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return fail(GG_ERR_HIP, std::string("timed steps: ") + hipGetErrorString(e));
  if (ms_even) *ms_even = cnt[0] ? tot[0] / (double)cnt[0] : 0.0;
  if (ms_odd) *ms_odd = cnt[1] ? tot[1] / (double)cnt[1] : 0.0;
  return GG_OK;
}

gg_status gg_step2_timed(gg_lattice *L, int64_t n_pairs, double *ms_pass) {
  if (L && special_boundaries(L))
    return fail(GG_ERR_STATE, "timed passes do not cover pressure boundaries or the paper's walls");
  if (!L || !ms_pass) return fail(GG_ERR_ARG, "NULL argument");
  if (n_pairs < 1) return fail(GG_ERR_ARG, "n_pairs must be positive");
  if (L->fuse < 2) return fail(GG_ERR_STATE, "the two-step pass is off");
  if (L->t & 1) return fail(GG_ERR_STATE, "the two-step pass starts on an even step");
  gg_status st = check_segments(L);
  if (st != GG_OK) return st;
  const int64_t n = 2 * n_pairs;  // passes, even: the state ends in the first plane set
  std::vector<hipEvent_t> ev(2 * (size_t)n, nullptr);
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < ev.size() && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
  for (int64_t k = 0; k < n && e == hipSuccess; ++k) {
    e = hipEventRecord(ev[2 * k], L->stream);
    if (e == hipSuccess) e = launch_pass(L, (int)(k & 1), (int)(2 * k), L->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * k + 1], L->stream);
  }
  if (e == hipSuccess) e = launch_advance(L->d_desc, 1, 2 * n, L->stream);
  if (e == hipSuccess) L->t += 2 * n;
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  double tot = 0.0;
  for (int64_t k = 0; k < n && e == hipSuccess; ++k) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
    tot += ms;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return fail(GG_ERR_HIP, std::string("timed passes: ") + hipGetErrorString(e));
  *ms_pass = tot / (double)n;
  return GG_OK;
}

gg_status gg_stream_copy(void *dst, const void *src, size_t bytes, int32_t reps,
                         void *hip_stream, double *ms) {
  if (!dst || !src || !ms || reps < 1 || bytes % 16 != 0)
    return fail(GG_ERR_ARG, "copy needs device buffers, reps >= 1 and a multiple of 16 bytes");
  hipStream_t st = (hipStream_t)hip_stream;
  hipEvent_t a = nullptr, b = nullptr;
  GG_HIP(hipEventCreate(&a));
  GG_HIP(hipEventCreate(&b));
  double total = 0.0;
  hipError_t e = hipSuccess;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch_copy(dst, src, bytes, st);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float x = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&x, a, b);
    total += x;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(GG_ERR_HIP, std::string("copy: ") + hipGetErrorString(e));
  *ms = total / reps;
  return GG_OK;
}

// ---------------------------------------------------------------------------
// Compound alone on frozen velocity fields
// ---------------------------------------------------------------------------

static size_t field_esize(const gg_lattice *L) { return L->storage == GG_F64 ? 8 : 4; }

// Grow the field buffer to at least n slots (new slots zero), keeping the
// contents of the old ones.
static gg_status grow_fields(gg_lattice *L, int n) {
  if (n <= L->n_ufield) return GG_OK;
  const size_t slot_bytes = 2 * (size_t)L->plane * field_esize(L);
  void *p = nullptr;
  hipError_t e = dev_alloc(L, &p, (size_t)n * slot_bytes);
  if (e != hipSuccess) return fail(GG_ERR_OOM, std::string("velocity fields: ") + hipGetErrorString(e));
  e = hipMemset(p, 0, (size_t)n * slot_bytes);
  if (e == hipSuccess && L->d_ufield)
    e = hipMemcpy(p, L->d_ufield, (size_t)L->n_ufield * slot_bytes, hipMemcpyDeviceToDevice);
  if (e != hipSuccess) {
    (void)dev_free(L, p);
    return fail(GG_ERR_HIP, std::string("velocity fields: ") + hipGetErrorString(e));
  }
  ++L->gen;
  if (L->d_ufield) GG_HIP(dev_free(L, L->d_ufield));
  L->d_ufield = p;
  L->n_ufield = n;
  return gg_upload_desc(L);
}

gg_status gg_set_velocity_field(gg_lattice *L, int32_t slot, const double *ux, const double *uy,
                                double scale, gg_where where) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (!std::isfinite(scale)) return fail(GG_ERR_ARG, "scale must be finite");
  if (slot < 0 || slot >= GG_MAX_FIELDS) return fail(GG_ERR_ARG, "slot must lie in 0..GG_MAX_FIELDS-1");
  if ((ux == nullptr) != (uy == nullptr)) return fail(GG_ERR_ARG, "give both components or neither");
  GG_HIP(hipStreamSynchronize(L->stream));
  gg_status st = grow_fields(L, slot + 1);
  if (st != GG_OK) return st;
  if (!ux) {
    GG_HIP(launch_capture(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6, slot, scale,
                          L->stream));
    GG_HIP(hipStreamSynchronize(L->stream));
    L->ufield_set |= 1u << slot;
    return GG_OK;
  }
  const size_t n = (size_t)L->nx * L->ny;
  double *dev[2] = {const_cast<double *>(ux), const_cast<double *>(uy)};
  if (where == GG_HOST) {
    for (int q = 0; q < 2; ++q) {
      const double *src = q ? uy : ux;
      for (int y = 0; y < L->ny; ++y)
        for (int x = 0; x < L->nx; ++x)
          if (L->mask[(size_t)y * L->nx + x] == GG_MASK_FLUID && !std::isfinite(src[(size_t)y * L->nx + x]))
            return fail(GG_ERR_ARG, "velocity field has non-finite entries on the fluid");
    }
    // the compound's linear equilibrium stays non-negative only for
    // |u_x|, |u_y| <= c_sg^2 = (1 - w0) / 2
    double umax = 0.0;
    for (size_t k = 0; k < n; ++k)
      if (L->mask[k] == GG_MASK_FLUID)
        umax = std::max(umax, std::max(std::fabs(scale * ux[k]), std::fabs(scale * uy[k])));
    if (umax > L->cs2g * (1.0 + 1e-12))
      return fail(GG_ERR_ARG, "scaled velocity " + std::to_string(umax) +
                                  " exceeds the compound lattice's positivity limit (1 - w0) / 2 = " +
                                  std::to_string(L->cs2g));
    dev[0] = dev[1] = nullptr;
    for (int q = 0; q < 2 && st == GG_OK; ++q) {
      if (dev_alloc(L, (void **)&dev[q], n * sizeof(double)) != hipSuccess)
        st = fail(GG_ERR_OOM, "hipMalloc of a velocity field failed");
      else if (hipMemcpy(dev[q], q ? uy : ux, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        st = fail(GG_ERR_HIP, "copy of a velocity field failed");
    }
  }
  if (st == GG_OK) {
    hipError_t e = launch_put_field(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6, slot,
                                    dev[0], dev[1], scale, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) st = fail(GG_ERR_HIP, std::string("velocity field: ") + hipGetErrorString(e));
  }
  if (where == GG_HOST)
    for (int q = 0; q < 2; ++q)
      if (dev[q]) (void)dev_free(L, dev[q]);
  if (st == GG_OK) L->ufield_set |= 1u << slot;
  return st;
}

gg_status gg_set_phase_fields(gg_lattice *L, const int32_t *slots, int32_t n) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (n < 0 || n > GG_MAX_PHASES || (n > 0 && !slots))
    return fail(GG_ERR_ARG, "n must lie in 0..GG_MAX_PHASES with a slot per phase");
  for (int k = 0; k < n; ++k)
    if (slots[k] < 0 || slots[k] >= GG_MAX_FIELDS)
      return fail(GG_ERR_ARG, "slot must lie in 0..GG_MAX_FIELDS-1");
  GG_HIP(hipStreamSynchronize(L->stream));
  for (int k = 0; k < GG_MAX_PHASES; ++k) L->phase_field[k] = (int8_t)(k < n ? slots[k] : 0);
  return gg_upload_desc(L);
}

gg_status gg_set_cde_launch(gg_lattice *L, int32_t rows) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (rows != 0 && rows != 6 && rows != 14 && rows != -6 && rows != -10)
    return fail(GG_ERR_ARG, "rows must be 0, 6, 14 (two-step passes) or -6, -10 (four-step passes)");
  GG_HIP(hipStreamSynchronize(L->stream));
  L->cde_rows = rows;
  gg_drop_cde_graphs(L);
  return GG_OK;
}

// Tile lists of the compound-only passes for the current row count: the
// two-step pass's (6 rows when the four-step pass is on) and the four-step
// pass's (58 columns, segment flag for a link within two nodes of the
// tile, in vertical stripes per XCD as the coupled four-step pass's).
static gg_status cde_tiles(gg_lattice *L) {
  if (L->cde_rows == 0 || L->cde_tiles_rows == L->cde_rows) return GG_OK;
  std::vector<Tile> list, unused, list4;
  L->cde_halo_seg = has_pressure(L);
  build_strips(L, L->cde_rows < 0 ? 6 : L->cde_rows, 0, false, list, unused, L->cde_halo_seg);
  if (L->cde_rows < 0) {
    build_strips(L, -L->cde_rows, 0, false, list4, unused, 2, 58);
    std::stable_sort(list4.begin(), list4.end(), [&](const Tile &a, const Tile &b) {
      const int sa = (int)((int64_t)a.x0 * 8 / L->nx), sb = (int)((int64_t)b.x0 * 8 / L->nx);
      return sa != sb ? sa < sb : (a.y0 != b.y0 ? a.y0 < b.y0 : a.x0 < b.x0);
    });
  }
  if (L->d_cde_tiles) GG_HIP(dev_free(L, L->d_cde_tiles));
  if (L->d_cde_tiles4) GG_HIP(dev_free(L, L->d_cde_tiles4));
  L->d_cde_tiles = L->d_cde_tiles4 = nullptr;
  L->n_cde_tiles = (int)list.size();
  L->n_cde_tiles4 = (int)list4.size();
  L->cde_tiles_rows = 0;
  if (!list.empty()) {
    GG_HIP(dev_alloc(L, (void **)&L->d_cde_tiles, list.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(L->d_cde_tiles, list.data(), list.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  if (!list4.empty()) {
    GG_HIP(dev_alloc(L, (void **)&L->d_cde_tiles4, list4.size() * sizeof(Tile)));
    GG_HIP(hipMemcpy(L->d_cde_tiles4, list4.data(), list4.size() * sizeof(Tile), hipMemcpyHostToDevice));
  }
  L->cde_tiles_rows = L->cde_rows;
  return GG_OK;
}

// n compound-only steps from a lattice whose counter reads t0 (host mirror),
// then the counter advances by n. With passes on (cde_rows != 0 and the
// second plane set present), the steps from an even t go in pairs of
// passes (8 steps in four-step passes, then 4 in two-step passes) that end
// in the first plane set; an odd-t first step and the leftover run as
// single steps.
static hipError_t launch_cde_steps(gg_lattice *L, int64_t t0, int64_t n, hipStream_t st) {
  hipError_t e = hipSuccess;
  int64_t dt = 0;
  auto single = [&](int64_t k) {
    return launch_cde(L->storage, L->pairs, ((t0 + k) & 1) != 0, L->d_desc, L->d_aux_tiles,
                      L->n_aux_tiles, 6, (int)k, st);
  };
  if (L->cde_rows != 0 && L->d_pop_b && L->cde_tiles_rows == L->cde_rows && L->wall_scheme == 0) {
    const bool press = L->n_press > 0;
    if ((t0 & 1) && n > 0) {
      e = single(dt);
      if (e == hipSuccess && press)
        e = launch_rescale(L->storage, L->d_desc, L->d_press, L->n_press, (int)dt, false, st);
      ++dt;
    }
    if (L->cde_rows < 0 && !press) {
      // four-step passes in pairs (ending in the first plane set)
      const int64_t p4 = (n - dt) / 8 * 2;
      for (int64_t k = 0; k < p4 && e == hipSuccess; ++k)
        e = launch_cde_tile4(L->storage, L->pairs, -L->cde_rows, L->d_desc, L->d_cde_tiles4,
                             L->n_cde_tiles4, (int)(k & 1), (int)(dt + 4 * k), st);
      dt += 4 * p4;
    }
    const int64_t passes = (n - dt) / 4 * 2;
    // (pressure: each pass after the first rescales the state it loads, the
    // kernel the state the last one leaves, in pop_b after dir 0)
    const bool at_load = press && L->cde_halo_seg;
    for (int64_t k = 0; k < passes && e == hipSuccess; ++k) {
      e = launch_cde_tile2(L->storage, L->pairs, L->cde_rows < 0 ? 6 : L->cde_rows, L->d_desc,
                           L->d_cde_tiles, L->n_cde_tiles,
                           (int)(k & 1) | (at_load && k > 0 ? 2 : 0), (int)(dt + 2 * k), st,
                           press);
      if (e == hipSuccess && press && (!at_load || k == passes - 1))
        e = launch_rescale(L->storage, L->d_desc, L->d_press, L->n_press, (int)(dt + 2 * k + 1),
                           false, st, (k & 1) == 0);
    }
    dt += 2 * passes;
  }
  for (; dt < n && e == hipSuccess; ++dt) {
    if (L->n_wall > 0)
      e = launch_wall_save(L->storage, L->d_desc, L->d_wall, L->n_wall, L->d_wall_links,
                           L->n_wall_links, (int)dt, false, L->d_wall_save, st);
    if (e == hipSuccess) e = single(dt);
    if (e == hipSuccess && L->n_wall > 0)
      e = launch_wall_apply(L->storage, L->d_desc, L->d_wall_links, L->n_wall_links, (int)dt,
                            L->d_wall_save, false, st);
    if (e == hipSuccess && L->n_press > 0)
      e = launch_rescale(L->storage, L->d_desc, L->d_press, L->n_press, (int)dt, false, st);
  }
  if (e == hipSuccess) e = launch_advance(L->d_desc, 1, n, st);
  return e;
}

gg_status gg_cde_step(gg_lattice *L, int64_t n) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (n < 0 || (n & 1))
    return fail(GG_ERR_ARG, "n must be even and non-negative (the fluid planes keep their layout)");
  gg_status st = check_segments(L);
  if (st != GG_OK) return st;
  const int np = std::max<int>(1, (int)L->phases.size());
  for (int k = 0; k < np; ++k) {
    const int s = L->phase_field[k];
    if (s >= L->n_ufield || !((L->ufield_set >> s) & 1u))
      return fail(GG_ERR_STATE, "velocity field slot " + std::to_string(s) + " of phase " +
                                    std::to_string(k) + " was never set");
  }
  if ((st = cde_tiles(L)) != GG_OK || (st = pressure_nodes(L)) != GG_OK ||
      (st = wall_nodes(L)) != GG_OK)
    return st;
  int64_t left = n;
  const int K = L->graph_chunk;  // even
  const int par = (int)(L->t & 1);
  if (K > 0 && left >= K) {
    if (!L->cde_exec[par]) {
      GG_HIP(hipStreamBeginCapture(L->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = launch_cde_steps(L, par, K, L->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(L->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(GG_ERR_HIP, std::string("graph capture: ") +
                                    hipGetErrorString(e != hipSuccess ? e : e2));
      }
      L->cde_graph[par] = g;
      GG_HIP(hipGraphInstantiate(&L->cde_exec[par], g, nullptr, nullptr, 0));
    }
    while (left >= K) {
      GG_HIP(hipGraphLaunch(L->cde_exec[par], L->stream));
      left -= K;
      L->t += K;
    }
  }
  if (left > 0) {
    GG_HIP(launch_cde_steps(L, L->t, left, L->stream));
    L->t += left;
  }
  return GG_OK;
}

gg_status gg_set_wall_scheme(gg_lattice *L, int32_t scheme) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  if (scheme != GG_WALL_BOUNCE_BACK && scheme != GG_WALL_PAPER)
    return fail(GG_ERR_ARG, "unknown wall scheme");
  GG_HIP(hipStreamSynchronize(L->stream));
  L->wall_scheme = scheme;
  L->wall_dirty = true;
  // (the four-step pass's lists follow the wall scheme)
  return L->tiles4 != pass4_ok(L) ? gg_rebuild_tiles(L) : GG_OK;
}

gg_status gg_permute_tiles(gg_lattice *L, uint64_t seed) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  GG_HIP(hipStreamSynchronize(L->stream));
  std::mt19937_64 rng(seed);
  auto shuffle = [&](Tile *d, int n) -> hipError_t {
    if (n <= 1) return hipSuccess;
    std::vector<Tile> h((size_t)n);
    hipError_t e = hipMemcpy(h.data(), d, h.size() * sizeof(Tile), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    std::shuffle(h.begin(), h.end(), rng);
    return hipMemcpy(d, h.data(), h.size() * sizeof(Tile), hipMemcpyHostToDevice);
  };
  GG_HIP(shuffle(L->d_tiles, L->n_tiles));
  GG_HIP(shuffle(L->d_strips, L->n_strips));
  GG_HIP(shuffle(L->d_seg_strips, L->n_seg_strips));
  GG_HIP(shuffle(L->d_strips4, L->n_strips4));
  GG_HIP(shuffle(L->d_seg_strips4, L->n_seg_strips4));
  GG_HIP(shuffle(L->d_cde_tiles, L->n_cde_tiles));
  GG_HIP(shuffle(L->d_cde_tiles4, L->n_cde_tiles4));
  gg_drop_cde_graphs(L);
  if (L->graph_exec) (void)hipGraphExecDestroy(L->graph_exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->graph_exec = nullptr;
  L->graph = nullptr;
  return GG_OK;
}

gg_status gg_sync(gg_lattice *L) {
  if (!L) return fail(GG_ERR_ARG, "lattice is NULL");
  GG_HIP(hipStreamSynchronize(L->stream));
  return GG_OK;
}

}  // extern "C"
