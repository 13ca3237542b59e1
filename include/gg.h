/*
 * gg.h - C ABI of the MI355X (gfx950) coupled lattice Boltzmann library.
 *
 * The library advances, on one GPU, the coupled scheme of Tanaka & Iber,
 * "Simulation of a Microfluidic Gradient Generator using Lattice Boltzmann
 * Methods" (arXiv:1307.4703):
 *   - fluid: D2Q9 lattice BGK (paper Eqs. 3-7), relaxation time tau_f,
 *     kinematic viscosity nu = (tau_f - 1/2)/3;
 *   - compound: multi-distribution advection-diffusion lattice (paper
 *     Eqs. 8-9) on D2Q5 with rest weight w0 (w0 = 0 is the paper's D2Q4),
 *     linear equilibrium g_i^eq = w_i C (1 + e_i.u/cs2), cs2 = (1 - w0)/2,
 *     D = cs2 (tau_g - 1/2), driven by the velocity of the same node at the
 *     same step (the one-way coupling of the Results section), with the
 *     source term R - kC of paper Eq. 2;
 *   - one fused collide-and-stream per time step on a masked lattice, with
 *     halfway bounce-back walls and boundary segments (inlets / outlets)
 *     that a periodic valve schedule opens and closes (the alternate
 *     flushing of the Experimental Layout section).
 *
 * Conventions for every function below:
 *   - Arrays are row-major with x fastest: element (x, y) is at y*nx + x.
 *   - Pointers are borrowed for the duration of the call; the library copies
 *     what it keeps. GG_DEVICE pointers are HIP device pointers that the
 *     library reads or writes on the lattice's stream.
 *   - Every call returns a gg_status; on failure nothing is thrown, the
 *     library state is left as before the call where that is possible, and
 *     gg_last_error() returns a message (thread-local).
 *   - Work is issued on the HIP stream given to gg_create. gg_step returns
 *     before the GPU is done; gg_read, gg_read_populations, gg_diagnostics
 *     and gg_save wait for the stream.
 */
#ifndef GG_H
#define GG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Mask values: 0 fluid, 1 wall, GG_FIRST_SEGMENT .. GG_FIRST_SEGMENT +
 * GG_MAX_SEGMENTS - 1 ghost cells of a boundary segment. */
#define GG_MASK_FLUID 0
#define GG_MASK_WALL 1
#define GG_FIRST_SEGMENT 2
#define GG_MAX_SEGMENTS 16
#define GG_MAX_PHASES 64
#define GG_MAX_FIELDS 16

typedef enum gg_status {
  GG_OK = 0,
  GG_ERR_ARG = 1,        /* invalid argument */
  GG_ERR_MASK = 2,       /* invalid geometry */
  GG_ERR_OOM = 3,        /* device or host allocation failed */
  GG_ERR_HIP = 4,        /* a HIP runtime call failed */
  GG_ERR_NONFINITE = 5,  /* diagnostics found a NaN or Inf population */
  GG_ERR_STATE = 6       /* call not valid in the current state */
} gg_status;

/* Population storage. Collision arithmetic is FP64 for GG_F64 and FP32
 * otherwise. Every storage type holds the deviations from rest,
 * h_i = f_i - w_i rho0 and h^g_i = g_i - w^g_i c_shift, and the step
 * computes on them; GG_F16_SHIFTED stores them in IEEE binary16, rounded to
 * nearest even. */
typedef enum gg_storage { GG_F64 = 0, GG_F32 = 1, GG_F16_SHIFTED = 2 } gg_storage;

typedef enum gg_where { GG_HOST = 0, GG_DEVICE = 1 } gg_where;

/* Boundary segment kinds.
 * GG_SEG_INLET : while open, a velocity inlet. Each link from a ghost cell
 *   into fluid node z carries the moving-wall bounce-back of the halfway
 *   wall, F(z,i) = f*(z,opp i) - 6 w_i rho0 (e_opp.u_w), with wall velocity
 *   u_w = -n u(s): a parabola of centre speed u_max across the segment,
 *   zero half a cell beyond its outermost ghost cells, evaluated at the
 *   tangential coordinate s of z; the compound gets anti-bounce-back for
 *   the Dirichlet value C_in: G(z,i) = -g*(z,opp i) + 2 w^g_i C_in.
 * GG_SEG_OUTLET : while open, an outflow at the reference density rho0 with
 *   zero normal gradient of the velocity (anti-bounce-back using the
 *   node's own velocity), and zero-gradient for the compound.
 * GG_SEG_PRESSURE : while open, the paper's pressure boundary (Boundary
 *   Conditions section, Eq. 10; configured with gg_set_pressure_segment):
 *   each population arriving from a ghost cell keeps the node's value of
 *   the step before ("do nothing", zeroth-order extrapolation in time),
 *   then, after the step, every population of the node is multiplied by
 *   rho_s / rho so that its density is the segment's rho_s and its velocity
 *   is unchanged. With hold_c the compound is treated alike and rescaled to
 *   C_in (where C <= 0 the node takes the equilibrium at rest of C_in);
 *   otherwise it leaves with zero gradient as at an outlet. A node with
 *   links to two pressure segments follows the first one met in direction
 *   order 1..8 (of the source cells x - e_i).
 * A closed segment is a wall (halfway bounce-back for f and g). */
typedef enum gg_seg_kind { GG_SEG_INLET = 1, GG_SEG_OUTLET = 2, GG_SEG_PRESSURE = 3 } gg_seg_kind;

typedef struct gg_params {
  double tau_f;       /* fluid relaxation time, > 1/2 (paper Eq. 4) */
  double D;           /* compound diffusion coefficient, > 0 (after Eq. 9) */
  double w0;          /* compound rest weight, 0 <= w0 < 1 */
  double rho0;        /* reference density: default initial density,
                         density of inlet/outlet links, shift of f */
  double k_decay;     /* first-order decay rate k >= 0 in R - kC (Eq. 2) */
  double c_shift;     /* shift C_s of the compound populations (finite);
                         0 keeps a compound at 0 exact, a mid-range value
                         uses the range of binary16 best */
  int32_t periodic_x; /* nonzero: x wraps; else the x edges are walls */
  int32_t periodic_y;
} gg_params;

/* One phase of a periodic valve schedule. Bit (id - GG_FIRST_SEGMENT) of
 * open_mask opens segment id for `duration` steps; bit k of c_in_set makes
 * c_in[k] the inlet concentration of segment GG_FIRST_SEGMENT + k in this
 * phase (otherwise the value given to gg_set_segment applies). */
typedef struct gg_phase {
  int64_t duration;
  uint32_t open_mask;
  uint32_t c_in_set;
  double c_in[GG_MAX_SEGMENTS];
} gg_phase;

/* FP64 diagnostics at the current time t (populations before collision). */
typedef struct gg_diag {
  int64_t t;             /* completed time steps since gg_init */
  int64_t n_fluid;       /* fluid nodes */
  int64_t n_nonfinite;   /* fluid nodes with a NaN/Inf population */
  double mass;           /* sum over fluid nodes of sum_i f_i */
  double solute;         /* sum over fluid nodes of sum_i g_i */
  double mass_in;        /* accumulated net mass entering through inlets */
  double mass_out;       /* ... through outlets (negative = leaving) */
  double solute_in;      /* accumulated net compound through inlets */
  double solute_out;     /* ... through outlets */
  double max_u;          /* max |u| over fluid nodes */
  double max_u_region;   /* max |u| over fluid nodes flagged by gg_set_region */
  double max_pe_region;  /* max_u_region / D: the largest cell Peclet number */
  double seg_mass[GG_MAX_SEGMENTS];    /* accumulated net mass per segment */
  double seg_solute[GG_MAX_SEGMENTS];  /* accumulated net compound per segment */
} gg_diag;

typedef struct gg_lattice gg_lattice;
typedef struct gg_batch gg_batch;

/* Create a lattice from a mask (host, nx*ny bytes). Fluid nodes with no
 * fluid neighbour among their 8 neighbours, unknown mask values and more
 * than two distinct segments next to one fluid node are GG_ERR_MASK.
 * `hip_stream` (a hipStream_t, may be NULL for the null stream) carries all
 * later work. Populations start at equilibrium with rho0, u = 0, C = 0. */
gg_status gg_create(const uint8_t *mask, int32_t nx, int32_t ny,
                    const gg_params *params, gg_storage storage,
                    void *hip_stream, gg_lattice **out);

/* Device memory from the caller (e.g. a framework's caching allocator):
 * alloc(bytes, ctx) returns device memory of the lattice's GPU, or NULL
 * when it cannot (the call then fails with GG_ERR_OOM); release(ptr, ctx)
 * takes back what alloc gave. The library calls release only once the
 * device is idle, so queued work never touches memory handed back. */
typedef struct gg_alloc {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*release)(void *ptr, void *ctx);
  void *ctx;
} gg_alloc;

/* gg_create with every device buffer of the lattice (populations, second
 * plane set, lists, velocity fields, read-back staging, the adjoint's
 * checkpoints and tape) taken from `alloc` (NULL: hipMalloc, as gg_create).
 * The allocator must stay valid until gg_destroy returns. Batches allocate
 * their own small lists with hipMalloc. Errors as gg_create, and GG_ERR_ARG
 * for an allocator without both functions. */
gg_status gg_create_ex(const uint8_t *mask, int32_t nx, int32_t ny,
                       const gg_params *params, gg_storage storage,
                       void *hip_stream, const gg_alloc *alloc, gg_lattice **out);

/* Configure segment `id` (a mask value >= GG_FIRST_SEGMENT). (nrm_x, nrm_y)
 * is the outward unit normal, along an axis, pointing from the fluid into
 * the ghost line; every ghost cell of the segment must have a fluid cell
 * one step against the normal (GG_ERR_MASK otherwise). u_max is the centre
 * speed of an inlet profile, c_in its default concentration. */
gg_status gg_set_segment(gg_lattice *lat, int32_t id, gg_seg_kind kind,
                         int32_t nrm_x, int32_t nrm_y, double u_max,
                         double c_in);

/* Configure segment `id` as a pressure boundary (GG_SEG_PRESSURE) holding
 * density rho (> 0; pressure rho / 3) and, if hold_c is nonzero, the
 * compound at c_in (per-phase overrides as for inlets). Geometry rules as
 * for gg_set_segment. While a lattice has such a segment, the rescaling
 * follows each single step in a kernel of its own; the row-parallel
 * two-step pass (fuse 3 and 4) rescales between its two steps in registers
 * and is followed by that kernel, except that in the one-kernel form (fuse
 * 4) each pass after the first rescales the state it loads instead and
 * the kernel follows only the last pass of a run (the same state as single
 * steps, bit for bit); walking strips (fuse 2) give way to single steps;
 * the compound-only passes (gg_set_cde_launch) rescale the compound as the
 * one-kernel form does. gg_adjoint, gg_batch_create, gg_step_timed and
 * gg_step2_timed refuse such a lattice (GG_ERR_STATE): the rescaling is
 * not linear in the compound. */
gg_status gg_set_pressure_segment(gg_lattice *lat, int32_t id, int32_t nrm_x,
                                  int32_t nrm_y, double rho, double c_in,
                                  int32_t hold_c);

/* Periodic valve schedule: phases repeat with period sum(duration); the
 * phase in force during step t -> t+1 is the one containing
 * (t - t_origin) mod period. n_phases = 0 removes the schedule (every
 * configured segment open). */
gg_status gg_set_schedule(gg_lattice *lat, const gg_phase *phases,
                          int32_t n_phases, int64_t t_origin);

/* Per-node source R (nx*ny doubles, host or device) of paper Eq. 2; NULL
 * removes it. Only the bounding box of its nonzero entries is stored. */
gg_status gg_set_source(gg_lattice *lat, const double *R, gg_where where);

/* Region flag per node (host, nx*ny bytes, nonzero = inside) for the
 * region velocity and Peclet diagnostics; NULL clears it. */
gg_status gg_set_region(gg_lattice *lat, const uint8_t *region);

/* Equilibrium initial state at every fluid node from nx*ny arrays (NULL:
 * rho0, 0, 0, 0 respectively): f = f^eq(rho, u), the quadratic equilibrium
 * of paper Eq. 5 with the weights of Eq. 6, and g = g^eq(C, u), the linear
 * equilibrium of Eq. 9 (a chip at rest with C = 0 is the Results section's
 * start). Resets t to 0 and the accumulated boundary fluxes to zero. */
gg_status gg_init(gg_lattice *lat, const double *rho, const double *ux,
                  const double *uy, const double *C, gg_where where);

/* Advance n >= 0 time steps. Each step is the collide-then-stream split the
 * paper states after Eq. 7, for both lattices at once: at every fluid node
 * the BGK collision of the fluid (Eq. 4, equilibrium Eqs. 5-6, moments
 * Eq. 7) and of the compound with the node's own velocity (Eq. 8,
 * equilibrium Eq. 9, source R - kC of Eq. 2), then streaming along the
 * velocities of Eq. 3 with the link rules of walls, closed valves and open
 * segments (Boundary Conditions section; see gg_seg_kind) at the valve
 * phase of the step (gg_set_schedule). Asynchronous. With the two-step pass
 * on (the default, see gg_set_two_step) the steps from an even t go in
 * passes of two steps each, in groups of four steps; a leftover or odd-t
 * step runs as a single step. Both ways give the same state, bit for bit.
 * With a monitor set (gg_set_monitor) the FP64 reductions run in between. */
gg_status gg_step(gg_lattice *lat, int64_t n);

/* Macroscopic fields at the current time (nx*ny doubles each; NaN off the
 * fluid; NULL skips a field): rho = sum f_i, u = sum f_i e_i / rho,
 * C = sum g_i (paper Eq. 7 and the definition after Eq. 9). */
gg_status gg_read(gg_lattice *lat, double *rho, double *ux, double *uy,
                  double *C, gg_where where);

/* Populations at the current time in natural order: f[i*nx*ny + y*nx + x]
 * for i = 0..8 and g[i*nx*ny + ...] for i = 0..4 (FP64; zero off the
 * fluid; NULL skips). Directions follow paper Eq. 3: 1..4 = +x, +y, -x, -y;
 * 5..8 = (+1,+1), (-1,+1), (-1,-1), (+1,-1). */
gg_status gg_read_populations(gg_lattice *lat, double *f, double *g,
                              gg_where where);

/* FP64 diagnostics of the current state: the mass and compound totals and
 * accumulated boundary fluxes of the conservation checks, max |u| over the
 * fluid and over the region of gg_set_region (the cell chamber, whose flow
 * must stay negligible: Abstract and Results section) and the largest cell
 * Peclet number there (Eq. 12 with one cell as length). Waits for the
 * stream; the per-tile partial sums live in a buffer allocated on the first
 * call (see gg_diagnostics_noalloc). GG_ERR_NONFINITE (with *out filled) if
 * any fluid node holds a non-finite population. */
gg_status gg_diagnostics(gg_lattice *lat, gg_diag *out);

/* Checkpoint and resume: a snapshot of the full state (populations in their
 * raw storage form and layout, time, fluxes) to a host buffer, and back.
 * No passage of the paper defines it; the long runs of its Results section
 * (four hours of chip time) are what it serves. With buf NULL, *nbytes
 * receives the size needed. Both wait for the stream. gg_load accepts only a
 * snapshot of a lattice with the same mask dimensions and storage
 * (GG_ERR_ARG otherwise), converting one of the other population layout
 * (gg_set_layout) into the lattice's; resuming gives bit for bit the run
 * that was not interrupted. */
gg_status gg_save(gg_lattice *lat, void *buf, size_t *nbytes);
gg_status gg_load(gg_lattice *lat, const void *buf, size_t nbytes);

/* Kernel launch shape of the single steps: tiles of tile_x * tile_y nodes
 * (one work-group each, tile_x * tile_y in {64, 128, 256, 512}, tile_x a
 * multiple of 8); only tiles holding a fluid node are launched.
 * graph_chunk > 0 replays gg_step in HIP graphs of that many steps (rounded
 * up to even, to a multiple of 4 with the two-step pass, of 8 with fuse =
 * 5); 0 launches every step. */
gg_status gg_set_launch(gg_lattice *lat, int32_t tile_x, int32_t tile_y,
                        int32_t graph_chunk);

/* Two-step pass (fuse = 2, 3 or 4; a new lattice starts with fuse = 3,
 * strip_h = 6), four-step pass (fuse = 5) or single steps only (fuse =
 * 1). The pass reads the state
 * of an even step once and writes the state two steps later into a second
 * set of population planes (same size as the first; allocated while
 * fuse >= 2, freed by fuse = 1), so every population crosses HBM once per
 * two steps instead of once per step.
 *   fuse = 2: one wavefront walks a strip of 62 columns x strip_h rows
 *     (1..4096), keeping the first step's result of each row in registers;
 *   fuse = 3: one work-group of strip_h + 2 wavefronts (strip_h 6 or 14)
 *     does a tile of 62 columns x strip_h rows, all rows at once, with the
 *     first step's row-crossing populations exchanged through LDS;
 *   fuse = 4: the tiles of fuse = 3, with the boundary-segment rules
 *     compiled into the one kernel that does every tile (with 2 and 3 the
 *     strips and tiles that touch a segment run in a kernel of their own,
 *     beside the others on a second stream, which keeps the boundary code
 *     out of the others' register budget);
 *   fuse = 5: runs of 8k steps from an even step in passes of four steps
 *     (temporal blocking over the AA pairs of steps, collide-and-stream
 *     after Eq. 7 four times per trip through memory): one work-group of
 *     12 wavefronts per tile of 58 columns x 6 rows with a three-node halo,
 *     each step's row-crossing populations through LDS; the tiles whose
 *     nodes within two of their own link to a segment run as 58 x 2 tiles
 *     in a kernel of their own on the second stream, as with fuse = 3.
 *     Other runs step as with fuse = 3 (strip_h 6 or 14). Lattices without
 *     pressure segments or the paper's walls, periodic axes of 4 nodes or
 *     more; otherwise fuse = 5 steps as fuse = 3. The
 *     result is that of single steps, bit for bit, as for every form.
 * Each collides a one-node halo around its strip or tile once more for the
 * first step. Errors: GG_ERR_ARG for other values, and for fuse = 2 where
 * two vertically adjacent fluid nodes link to more than two boundary
 * segments between them (a walking strip sums their fluxes in one record
 * of two segments); GG_ERR_OOM if the planes do not fit. */
gg_status gg_set_two_step(gg_lattice *lat, int32_t fuse, int32_t strip_h);

/* Layout of the population planes in device memory (the state's values do
 * not depend on it; every step computes the same bits in either):
 *   GG_LAYOUT_PAIRED (a new lattice's layout): f_i and g_i of a node side
 *     by side for i = 0..4, the fluid and compound populations that stream
 *     along the same velocity e_i (Eq. 3), so the coupled pass moves each
 *     such pair with one memory access; f5..f8 in planes of their own;
 *   GG_LAYOUT_PLANES: one plane per population, node-contiguous, which the
 *     compound-only steps (gg_cde_step) read at the full width of their
 *     accesses (in the paired layout they fetch the f halves too).
 * Switching converts the stored state (through the second plane set, or a
 * buffer of its size while fuse = 1) and waits for the lattice's stream.
 * Snapshots record their layout; gg_load converts a snapshot of the other
 * layout. Errors: GG_ERR_ARG for other values, GG_ERR_OOM. */
#define GG_LAYOUT_PLANES 0
#define GG_LAYOUT_PAIRED 1
gg_status gg_set_layout(gg_lattice *lat, int32_t layout);
gg_status gg_get_layout(const gg_lattice *lat, int32_t *layout);

/* Compound alone on frozen velocity fields. The paper lets the flow of a
 * valve configuration settle (it does so far faster than the compound) and
 * then advances the advection-diffusion lattice alone under that fixed
 * velocity (Results section): per node a step then moves the 5 compound
 * populations, 2 velocity components and the link code (FP32 storage: 49
 * bytes) instead of the 14 populations of the coupled step.
 *
 * gg_set_velocity_field stores scale times a velocity field in slot
 * 0..GG_MAX_FIELDS-1 (device memory: two planes of the compute type per
 * slot, FP64 for GG_F64, FP32 otherwise, allocated on first use and kept
 * until gg_destroy). ux, uy: nx*ny doubles (y*nx + x; host or device per
 * `where`; only fluid entries are read, and on the host they must be
 * finite); scale * u is formed in FP64 and rounded to the compute type.
 * With ux = uy = NULL the slot receives scale times the velocity of the
 * current fluid state, computed as the coupled step computes it (paper
 * Eq. 7 in the compute type), times scale in the compute type. scale rescales a
 * flow computed at one time step to the compound lattice's larger one (the
 * paper raises the peak velocity to its chosen U^LB this way). The caller
 * keeps the scaled speed inside the compound lattice's positivity limit,
 * |u_x|, |u_y| <= c_sg^2 = (1 - w0) / 2 (1/3 for w0 = 1/3, 1/2 for the
 * paper's D2Q4): beyond it the linear equilibrium turns negative and the
 * compound-only steps become unstable; host fields beyond it are refused
 * (GG_ERR_ARG), device fields and captures are not checked. Synchronises
 * the lattice's stream. Errors: GG_ERR_ARG (slot out of range, one of ux/uy
 * NULL, non-finite scale or host entries, host entries beyond the limit),
 * GG_ERR_OOM. */
gg_status gg_set_velocity_field(gg_lattice *lat, int32_t slot, const double *ux,
                                const double *uy, double scale, gg_where where);

/* slots[k] (0..GG_MAX_FIELDS-1): the field used while schedule phase k is
 * in force, k < n <= GG_MAX_PHASES; phases from n on, and every phase after
 * gg_set_phase_fields(lat, NULL, 0) (the default), use slot 0. Without a
 * schedule, slots[0] is used throughout. */
gg_status gg_set_phase_fields(gg_lattice *lat, const int32_t *slots, int32_t n);

/* Advance the compound alone n steps (n even, >= 0; else GG_ERR_ARG): at
 * every fluid node the compound collides (Eqs. 8-9 with the source of
 * Eq. 2) with the velocity of the field of the phase in force and streams,
 * with the link rules of the coupled step for walls, closed valves, inlets
 * (C_in of the phase) and outlets; solute fluxes through open segments
 * accumulate as in gg_step. The fluid populations are left untouched and t
 * advances by n (an even n keeps the fluid planes in the layout that t's
 * parity expects, so gg_step may follow). With the field of each step equal
 * to the velocity the coupled step's fluid has at that step, the compound
 * equals the coupled step's. Asynchronous; replays graphs of graph_chunk
 * steps (gg_set_launch). GG_ERR_STATE if a phase's slot was never set.
 * Steps from an even t go in two-step passes (see gg_set_cde_launch) while
 * the second plane set exists (gg_set_two_step with fuse >= 2, the
 * default); the result is the same bit for bit either way. */
gg_status gg_cde_step(gg_lattice *lat, int64_t n);

/* Launch form of gg_cde_step: rows = 6 or 14 (the default) runs pairs of
 * steps as one pass over memory, one work-group of rows + 2 wavefronts per
 * tile of 62 columns x rows, which reads the compound state and the field
 * once and writes the state two steps later into the second plane set
 * (the compound planes only); rows = -6 or -10 runs runs of 8k steps in
 * passes of four steps (one work-group of -rows + 6 wavefronts per tile of
 * 58 columns x -rows rows with a three-node halo; lattices with pressure
 * segments, and the last four steps of a run of 8k + 4, in two-step passes
 * of 6-row tiles); rows = 0 keeps to single steps. GG_ERR_ARG for other
 * values. Every form gives the single steps' result bit for bit. */
gg_status gg_set_cde_launch(gg_lattice *lat, int32_t rows);

/* Number of fluid nodes and launched tiles. */
gg_status gg_info(const gg_lattice *lat, int64_t *n_fluid, int64_t *n_tiles,
                  int64_t *t);

/* Batched launch: many lattices advanced together, one flat launch over
 * the concatenated tile lists of all of them per step (two when the
 * lattices sit at steps of different parity), graph-captured in chunks of
 * graph_chunk steps (0: plain launches). All lattices must share the
 * storage type and the HIP stream; the batch copies their configuration
 * (parameters, segments, schedules) at creation, so later changes to a
 * member need a new batch: once a member was reconfigured (any call that
 * changes its parameters, segments, schedule, source, region, velocity
 * fields or plane sets), gg_batch_step and gg_batch_set_two_step return
 * GG_ERR_STATE. The members' states advance in place: after
 * gg_batch_step(b, n) every member is n steps further, exactly as after
 * gg_step(member, n). tile_x, tile_y as in gg_set_launch (0, 0: 64 x 4);
 * persist > 0 caps the grid at that many work-groups, which then loop over
 * the tiles (a persistent launch); 0 launches one work-group per tile.
 * persist = GG_AUTOTUNE: the library picks the form (tile_x and tile_y are
 * then ignored): each candidate (single steps over tiles of 64 x 4, 32 x 8
 * or 128 x 2 nodes; when every member has its second plane set and all sit
 * at steps of one parity, two-step passes with 6- or 14-row tiles and the
 * boundary tiles apart, or 6- or 14-row tiles in one kernel, or four-step
 * passes) advances the members
 * 20 steps, 16 of them timed with HIP events on their stream, and the
 * fastest is kept (gg_batch_form reports it). The members' states, step
 * counts and boundary fluxes are copied aside on the device (hipMalloc of
 * their total state size, freed before returning) and put back after every
 * candidate, so the members are left as they were. Waits for the stream. */
#define GG_AUTOTUNE (-1)
gg_status gg_batch_create(gg_lattice *const *lats, int32_t n, int32_t tile_x,
                          int32_t tile_y, int32_t persist, int32_t graph_chunk,
                          gg_batch **out);
gg_status gg_batch_step(gg_batch *batch, int64_t n);

/* The launch form of a batch (tile shape, persistent grid, two-step form
 * and tile rows as gg_batch_set_two_step takes them); any pointer may be
 * NULL. */
gg_status gg_batch_form(const gg_batch *batch, int32_t *tile_x, int32_t *tile_y,
                        int32_t *persist, int32_t *fuse, int32_t *rows);

/* Two-step pass for the batch (see gg_set_two_step): fuse 3 or 4 with
 * tiles of rows = 6 or 14 rows, over the members' tiles in one flat list
 * (fuse 3: the boundary tiles of all members in a second list on a second
 * stream); fuse 5: four-step passes over the members' 58 x 6 tiles (the
 * boundary tiles apart), runs of 8k + 4 steps ending in two two-step
 * passes of fuse 3's form with `rows` rows (GG_ERR_ARG for a member with a
 * periodic axis under 4 nodes); fuse = 1 goes back to
 * single steps. Every member must have its
 * second plane set (fuse >= 2 on the member, the default) and all members
 * must sit at steps of one parity (else GG_ERR_STATE). The states advance
 * exactly as with single steps. */
gg_status gg_batch_set_two_step(gg_batch *batch, int32_t fuse, int32_t rows);
gg_status gg_batch_info(const gg_batch *batch, int64_t *n_tiles, int64_t *n_fluid);
void gg_batch_destroy(gg_batch *batch);

/* Gradients returned by gg_adjoint. */
typedef struct gg_grads {
  double loss;                      /* 1/2 sum_x weight(x) (C(x) - target(x))^2 */
  double d_c_in[GG_MAX_SEGMENTS];   /* dL/dC_in of segment GG_FIRST_SEGMENT + k,
                                       for a change of its inlet concentration
                                       in every phase in which it is open */
  double d_D;                       /* dL/dD */
  double d_omega_g;                 /* dL/d(1/tau_g) */
  int64_t ckpt_every;               /* steps between checkpoints used */
  int64_t n_checkpoints;
} gg_grads;

/* Discrete adjoint of the coupled step with respect to the compound's
 * parameters. From the current state at time t0, advances n_steps >= 1
 * (the lattice ends at t0 + n_steps, as after gg_step), evaluates
 * L = 1/2 sum_x weight(x) (C(x) - target(x))^2 on the final compound field,
 * then runs the hand-written adjoint of each step backwards. The fluid does
 * not depend on the compound (one-way coupling), so only the compound
 * populations carry an adjoint; the fluid velocity of each step is
 * recomputed from checkpoints taken every ckpt_every steps (0: ceil(sqrt(n)))
 * and taped for one segment at a time. weight and target are host arrays of
 * nx*ny doubles. r_box = {x0, y0, w, h} (or NULL) selects the nodes whose
 * source gradient dL/dR is written to d_R (host, w*h doubles, row-major).
 * Device memory: about n/ckpt_every copies of the state plus ckpt_every
 * tape slots of 7 fields; GG_ERR_OOM if it does not fit. */
gg_status gg_adjoint(gg_lattice *lat, int64_t n_steps, int64_t ckpt_every,
                     const double *weight, const double *target,
                     const int32_t *r_box, double *d_R, gg_grads *out);

/* Instrumentation: advance n >= 1 steps launching every step kernel
 * between two HIP events on the lattice's stream (no graphs) and return the
 * mean event-measured duration, in ms, of the even-step and of the
 * odd-step kernels (either pointer may be NULL). Waits for the stream. */
gg_status gg_step_timed(gg_lattice *lat, int64_t n, double *ms_even, double *ms_odd);

/* Instrumentation: with the two-step pass on and t even, run 2 * n_pairs
 * passes (4 * n_pairs steps) between HIP events on the lattice's stream and
 * return the mean event-measured duration of one pass, in ms. Waits for
 * the stream. GG_ERR_STATE if the pass is off or t is odd. */
gg_status gg_step2_timed(gg_lattice *lat, int64_t n_pairs, double *ms_pass);

/* Instrumentation: copy `bytes` (a multiple of 16) from src to dst, both
 * device buffers, `reps` times with a plain streaming kernel on hip_stream,
 * and return in *ms the mean event-measured duration of one copy. Used to
 * measure achievable HBM bandwidth and to calibrate traffic counters. */
gg_status gg_stream_copy(void *dst, const void *src, size_t bytes, int32_t reps,
                         void *hip_stream, double *ms);

/* Wall conditions at the links from walls and closed or unconfigured valve
 * cells (paper, Boundary Conditions section):
 *   GG_WALL_BOUNCE_BACK (default): halfway bounce-back, the population
 *     leaving z toward the wall comes back along the opposite link.
 *   GG_WALL_PAPER : the paper's walls. The wall cell s = z - e_i next to
 *     fluid node z is a ghost node emitting along e_i the equilibrium
 *     f_i^eq(rho_s, u_s) of the density extrapolated linearly from the
 *     fluid, rho_s = 2 rho(z) - rho(z + e_i) (rho(z) where z + e_i is not
 *     fluid), and the momentum that vanishes at the halfway wall, u_s =
 *     -j(z) / rho_s; the compound takes the non-equilibrium extrapolation
 *     of Guo et al. (no flux through the wall): g_i^eq(C(z), u_s) +
 *     (1 - omega_g) (g_i(z) - g_i^eq(C(z), u(z))). All quantities are those
 *     of step t (before the collision). In the compound-only step u(z) is
 *     the frozen field's and u_s = -u(z).
 * With GG_WALL_PAPER, steps run one at a time (no two-step passes), with a
 * save kernel before and a fix-up kernel after each; the adjoint, the timed
 * calls and batches refuse such lattices. Mass is not conserved exactly
 * (the ghost density is extrapolated). Errors: GG_ERR_ARG for a NULL
 * lattice or an unknown scheme. */
typedef enum gg_wall_scheme { GG_WALL_BOUNCE_BACK = 0, GG_WALL_PAPER = 1 } gg_wall_scheme;
gg_status gg_set_wall_scheme(gg_lattice *lat, int32_t scheme);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * diagnostics of gg_diagnostics, with the reduction's partial records in a
 * fixed array of 6 * 2048 + 8 doubles (98,368 bytes) that the library
 * holds in device memory on every GPU it runs on until the process ends,
 * instead of the per-lattice buffer gg_diagnostics allocates on first use.
 * The reduction runs at most 2048 work-groups, each folding every 2048-th
 * 64 x 4 tile, so the array fits every lattice: no lattice is too large.
 * Calls no hipMalloc or hipFree (the array's device address is looked up
 * once per GPU). Calls that overlap on one GPU (other threads, other
 * lattices) race on the one array: serialise them. The totals can differ
 * from gg_diagnostics' in the last bits (another summation order); maxima,
 * counts and boundary fluxes are the same. Waits for the lattice's stream.
 * Errors: GG_ERR_ARG (NULL argument), GG_ERR_HIP, GG_ERR_NONFINITE (with
 * *out filled). */
gg_status gg_diagnostics_noalloc(gg_lattice *lat, gg_diag *out);

/* Monitor (the diagnostics of the Results section on the hot path: the
 * flow in the chamber must stay negligible, Abstract and Results; cell
 * Peclet number of Eq. 12; mass and compound totals of the conservation
 * checks): with every > 0, gg_step launches the FP64 reduction of
 * gg_diagnostics on the lattice's stream after each step that ends a
 * multiple of `every` steps counted from the call, without waiting for the
 * GPU, and keeps the last result (with a copy of the boundary-flux
 * accumulators taken at the same point) in device memory; every = 0 turns
 * it off. Steps between two reductions still run in graph replays and
 * two-step passes. Device memory: 40 doubles plus 6 doubles per 64 x 4
 * tile holding fluid, allocated here (GG_ERR_OOM). GG_ERR_ARG for every
 * < 0. */
gg_status gg_set_monitor(gg_lattice *lat, int64_t every);

/* The last monitor reduction (waits for the stream): out->t is the step it
 * was taken at; *count (may be NULL) the reductions since gg_set_monitor.
 * GG_ERR_STATE if none has run; GG_ERR_NONFINITE (with *out filled) if
 * that reduction found a non-finite population. */
gg_status gg_monitor_read(gg_lattice *lat, gg_diag *out, int64_t *count);

/* Result of gg_step_profile. The dominant kernel is the one that takes the
 * most HBM traffic: the kernel over the interior tile list of each two-step
 * pass (with fuse 2 and 3 the boundary tiles run in a second kernel beside
 * it on a side stream; with fuse 4 it is the pass's only kernel), of each
 * four-step pass where fuse 5 runs them (two-step passes of leftover steps
 * are then counted apart, in n_pass2), or the step kernel of each single
 * step. */
typedef struct gg_profile {
  double ms_total;          /* HIP events around the whole call */
  int64_t n_pass;           /* plain launches of the pass's dominant kernel */
  double ms_pass;           /* their summed event-measured duration */
  int64_t n_graph;          /* graph replays (gg_set_launch graph_chunk) */
  double ms_graph;          /* their summed event-measured duration */
  int64_t graph_passes;     /* two-step passes inside those replays */
  int64_t graph_singles;    /* single steps inside those replays */
  int64_t n_single[2];      /* single steps at even / odd t */
  double ms_single[2];      /* their summed duration */
  int64_t n_monitor;        /* monitor reductions launched (gg_set_monitor) */
  int64_t pass_fluid;       /* fluid nodes owned by the tiles of the pass's
                               dominant kernel (steps_per_pass updates each
                               per launch) */
  int64_t pass_side_fluid;  /* fluid nodes owned by the side kernel's tiles */
  int64_t pass_tiles;       /* tiles of the dominant kernel (one work-group of
                               rows + 2 wavefronts each, 8 * ceil(tiles / 8)
                               work-groups launched) */
  int64_t pass_side_tiles;  /* tiles of the side kernel (2 rows each) */
  int64_t n_pass2;          /* with the four-step pass: plain launches of the
                               two-step passes of leftover steps (their
                               interior kernel), and */
  double ms_pass2;          /* their summed duration */
  int32_t fuse, rows;       /* launch form used (fuse 1: single steps only) */
  int32_t steps_per_pass;   /* 2, or 4 where the four-step pass runs (fuse
                               5; its tiles are then the pass_ fields') */
} gg_profile;

/* Instrumentation: gg_step(lat, n) with a pair of HIP events recorded on
 * the lattice's stream around every plain launch of the dominant kernel,
 * around every graph replay (whose passes or steps are counted) and around
 * the whole call; waits for the stream and returns the event-measured
 * durations. The launches are those of gg_step (graph replays, plain
 * passes, single steps, monitor reductions), and the state advances
 * exactly as with gg_step. Errors as gg_step, GG_ERR_HIP if an event
 * fails. */
gg_status gg_step_profile(gg_lattice *lat, int64_t n, gg_profile *out);

/* Instrumentation: shuffle the order of the tiles and strips the steps
 * are launched over (seeded), e.g. to check that the result does not depend
 * on the order in which work-groups run. Waits for the stream. */
gg_status gg_permute_tiles(gg_lattice *lat, uint64_t seed);

/* Wait for all work issued on the lattice's stream. */
gg_status gg_sync(gg_lattice *lat);

void gg_destroy(gg_lattice *lat);

/* Message of the last failed call on this thread. */
const char *gg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GG_H */
