/*
 * FP64 CPU oracle for the coupled lattice Boltzmann step of
 * Tanaka & Iber, "Simulation of a Microfluidic Gradient Generator using
 * Lattice Boltzmann Methods" (arXiv:1307.4703).
 *
 * TEST INFRASTRUCTURE. This file is the slow, obviously correct reference
 * that the HIP path is checked against. Only the test-suite, the smoke entry
 * point and the CPU-baseline leg of the benchmark may load it. It shares no
 * code, header, table or layout with the library under paper_1307_4703_amd/.
 *
 * Layout: array-of-structures, f[(y*nx + x)*9 + i] and g[(y*nx + x)*5 + i],
 * two arrays (old -> new) per step; nothing is done in place.
 *
 * What is computed per time step, for every fluid node x (mask == 0):
 *   1. moments of f (Eq. 7; the printed upper limit 9 is read as 8),
 *   2. BGK relaxation of f toward the quadratic equilibrium (Eqs. 4-6),
 *   3. compound C = sum of g and the linear equilibrium driven by the SAME
 *      node's fluid velocity from step 1 (Eq. 9 and the sentence after it:
 *      u is handed over from the fluid solver),
 *   4. BGK relaxation of g (Eq. 8) plus the source/decay term R - kC of the
 *      advection-diffusion equation (Eq. 2),
 *   5. free flight along e_i (the collide-then-stream split described after
 *      Eq. 7), with link rules where the cell a population comes from is
 *      not fluid:
 *        wall or closed valve  -> halfway bounce-back for f and g,
 *        open velocity inlet   -> moving-wall bounce-back for f,
 *                                 anti-bounce-back (Dirichlet C_in) for g,
 *        open outlet           -> f: anti-bounce-back at the reference
 *                                 density with the node's own velocity;
 *                                 g: zero-gradient (ghost emits what z emits),
 *        open pressure segment -> the paper's pressure boundary: "do
 *                                 nothing" (each missing population keeps
 *                                 the node's value of step t, a zeroth-order
 *                                 extrapolation in time), then every
 *                                 population of the node is rescaled so that
 *                                 its density is the segment's (Eq. 10: u is
 *                                 unchanged); the compound likewise, rescaled
 *                                 to C_in, where the segment prescribes it,
 *                                 and otherwise zero-gradient as at an
 *                                 outlet.
 *      Outside the domain counts as wall unless that axis is periodic.
 * With wall_scheme = 1 the links from walls and closed valves take the
 * paper's wall conditions instead of bounce-back (see wall_links below).
 *
 * Compile with -ffp-contract=off so every product and sum is rounded as
 * written.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 directions of Eq. (3): 0 rest; 1..4 along the axes at angles
 * (i-1)*pi/2; 5..8 along the diagonals at pi/4, 3pi/4, 5pi/4, 7pi/4. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Index of the direction opposite to e_i. */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* Weights of Eq. (6). */
static const double WF[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Segment kinds (per mask value >= 2). */
#define ORC_SEG_NONE 0
#define ORC_SEG_INLET 1
#define ORC_SEG_OUTLET 2
#define ORC_SEG_PRESSURE 3

typedef struct orc_lattice {
  int32_t nx, ny;
  int32_t periodic_x, periodic_y;
  const uint8_t *mask;  /* ny*nx: 0 fluid, 1 wall, >= 2 segment (ghost) id */
  double tau_f;         /* fluid relaxation time (Eq. 4) */
  double tau_g;         /* compound relaxation time (Eq. 8) */
  double w0;            /* rest weight of the compound lattice (0 = D2Q4) */
  double rho_w;         /* reference density of inlet and outlet links */
  double k_decay;       /* first-order decay rate k in R_total = R - kC */
  const double *R;      /* ny*nx source, or NULL for zero */
  /* per mask value 0..255 */
  const int32_t *seg_kind;   /* ORC_SEG_* */
  const int32_t *seg_nrm;    /* [256][2] outward unit normal (into the ghost) */
  const double *seg_umax;    /* centre-line inflow speed */
  const double *seg_s0;      /* lower halfway-wall tangential coordinate */
  const double *seg_s1;      /* upper halfway-wall tangential coordinate */
  const double *seg_rho;     /* density held by a pressure segment */
  const int32_t *seg_fixc;   /* pressure segment also holds C = C_in */
  int32_t wall_scheme;       /* 0: halfway bounce-back; 1: the paper's walls */
} orc_lattice;

/* ---------------------------------------------------------------- */
/* Equilibria                                                          */
/* ---------------------------------------------------------------- */

/* Quadratic equilibrium, Eq. (5) with the weights of Eq. (6). */
void orc_feq(double rho, double ux, double uy, double *out9) {
  double usq = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    out9[i] = rho * WF[i] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
  }
}

/* Weights of the compound lattice: D2Q5 with rest weight w0 and the four
 * axis weights (1 - w0)/4. w0 = 0 is the paper's D2Q4 lattice. */
static void orc_gweights(double w0, double *wg5) {
  wg5[0] = w0;
  for (int i = 1; i < 5; ++i) wg5[i] = (1.0 - w0) / 4.0;
}

/* Linear equilibrium of the compound lattice. Eq. (9) is
 * g_i^eq = (C/4)(1 + 2 e_i.u) on D2Q4; its general form on D2Q5 is
 * g_i^eq = w_i C (1 + e_i.u / cs2) with cs2 = (1 - w0)/2, which reduces to
 * Eq. (9) at w0 = 0 (w_i = 1/4, 1/cs2 = 2). */
void orc_geq(double C, double ux, double uy, double w0, double *out5) {
  double wg[5];
  orc_gweights(w0, wg);
  double cs2 = (1.0 - w0) / 2.0;
  for (int i = 0; i < 5; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    out5[i] = wg[i] * C * (1.0 + eu / cs2);
  }
}

/* ---------------------------------------------------------------- */
/* Geometry helpers                                                    */
/* ---------------------------------------------------------------- */

/* Cell type seen from a link. Returns the mask value of cell (x, y) after
 * periodic wrap, or 1 (wall) when (x, y) lies outside a non-periodic edge. */
static int cell_code(const orc_lattice *L, int x, int y, int *xw, int *yw) {
  if (x < 0 || x >= L->nx) {
    if (!L->periodic_x) return 1;
    x = (x + L->nx) % L->nx;
  }
  if (y < 0 || y >= L->ny) {
    if (!L->periodic_y) return 1;
    y = (y + L->ny) % L->ny;
  }
  *xw = x;
  *yw = y;
  return L->mask[(size_t)y * L->nx + x];
}

/* Mask value of the open pressure segment that fluid node (x, y) takes its
 * boundary condition from at this step: the source cell x - e_i of the
 * lowest-numbered direction i that is a ghost cell of an open pressure
 * segment; 0 if there is none. */
static int pressure_segment(const orc_lattice *L, int x, int y, const uint8_t *open) {
  for (int i = 1; i < 9; ++i) {
    int xs = 0, ys = 0;
    int code = cell_code(L, x - EX[i], y - EY[i], &xs, &ys);
    if (code >= 2 && L->seg_kind[code] == ORC_SEG_PRESSURE && open[code]) return code;
  }
  return 0;
}

/* Rescaling of a pressure-boundary node after streaming (Eq. 10): every f_i
 * times rho_m / rho, so that the density is the segment's and the velocity
 * is unchanged. Returns the mass added. */
static double rescale_f(const orc_lattice *L, int m, double *fz) {
  double rho = 0.0;
  for (int i = 0; i < 9; ++i) rho += fz[i];
  double gam = L->seg_rho[m] / rho;
  for (int i = 0; i < 9; ++i) fz[i] *= gam;
  return L->seg_rho[m] - rho;
}

/* The compound at a pressure-boundary node whose segment prescribes it:
 * every g_i times C_in / C, or, when C is not positive (nothing to
 * rescale), the equilibrium at rest w_i C_in. Returns the compound added. */
static double rescale_g(const orc_lattice *L, int m, double *gz, const double *c_in) {
  if (!L->seg_fixc[m]) return 0.0;
  double wg[5];
  orc_gweights(L->w0, wg);
  double C = 0.0;
  for (int i = 0; i < 5; ++i) C += gz[i];
  if (C > 0.0) {
    double gam = c_in[m] / C;
    for (int i = 0; i < 5; ++i) gz[i] *= gam;
  } else {
    for (int i = 0; i < 5; ++i) gz[i] = wg[i] * c_in[m];
  }
  return c_in[m] - C;
}

/* Parabolic inflow profile across a velocity-inlet segment, evaluated at the
 * tangential coordinate s of the fluid node next to the ghost line; zero at
 * the two halfway wall positions s0 and s1. */
static double inlet_speed(const orc_lattice *L, int seg, int x, int y) {
  const int32_t *n = L->seg_nrm + 2 * seg;
  double s = (n[0] != 0) ? (double)y : (double)x;
  double s0 = L->seg_s0[seg], s1 = L->seg_s1[seg];
  double w = s1 - s0;
  return 4.0 * L->seg_umax[seg] * (s - s0) * (s1 - s) / (w * w);
}

/* ---------------------------------------------------------------- */
/* One coupled time step, t -> t+1                                     */
/* ---------------------------------------------------------------- */

/* Post-collision populations of one fluid node (steps 1-4 above). */
static void collide_node(const orc_lattice *L, size_t node, const double *fx,
                         const double *gx, double *fpost, double *gpost,
                         double *u) {
  double wg[5];
  orc_gweights(L->w0, wg);
  /* 1. moments of f, Eq. (7) */
  double rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < 9; ++i) {
    rho += fx[i];
    jx += fx[i] * EX[i];
    jy += fx[i] * EY[i];
  }
  double ux = jx / rho, uy = jy / rho;
  u[0] = ux;
  u[1] = uy;
  /* 2. BGK for f, Eq. (4) */
  double feq[9];
  orc_feq(rho, ux, uy, feq);
  double omega_f = 1.0 / L->tau_f;
  for (int i = 0; i < 9; ++i) fpost[i] = fx[i] - omega_f * (fx[i] - feq[i]);
  /* 3. compound and its equilibrium with the node's own u, Eq. (9) */
  double C = 0.0;
  for (int i = 0; i < 5; ++i) C += gx[i];
  double geq[5];
  orc_geq(C, ux, uy, L->w0, geq);
  /* 4. BGK for g, Eq. (8), plus the reaction term of Eq. (2) */
  double omega_g = 1.0 / L->tau_g;
  double src = (L->R ? L->R[node] : 0.0) - L->k_decay * C;
  for (int i = 0; i < 5; ++i)
    gpost[i] = gx[i] - omega_g * (gx[i] - geq[i]) + wg[i] * src;
}

/* The paper's wall conditions (Boundary Conditions section), for a fluid
 * node z whose link i comes from a wall or closed-valve cell s = z - e_i:
 * the cell s is taken as a node whose populations at step t are
 *   fluid: the equilibrium f_i^eq(rho_s, u_s), its momentum interpolated
 *     linearly through zero at the wall, which lies halfway between s and
 *     z (j_s = -j(z)), its density extrapolated linearly from the fluid
 *     along e_i (rho_s = 2 rho(z) - rho(z + e_i), or rho(z) where z + e_i
 *     is not fluid), u_s = j_s / rho_s;
 *   compound: the no-flux condition by non-equilibrium extrapolation (Guo
 *     et al.): the post-collision population of s is the equilibrium of
 *     z's concentration at the ghost velocity plus z's non-equilibrium part
 *     relaxed by the collision, g_i^eq(C(z), u_s) + (1 - omega_g)
 *     (g_i(z) - g_i^eq(C(z), u(z))) (zero normal gradient of C);
 * and what it emits along e_i arrives at z at t + 1. Every quantity is of
 * step t (the populations before the collision), so the rule needs no
 * value of step t + 1. Fills fz[i] (and gz[i], i <= 4) for every such link
 * of the node at (x, y); f, g: the state at step t. */
static void wall_links(const orc_lattice *L, int x, int y, const double *f, const double *g,
                       const uint8_t *open, double *fz, double *gz) {
  const int nx = L->nx;
  const size_t node = (size_t)y * nx + x;
  const double omega_g = 1.0 / L->tau_g;
  double rho = 0.0, jx = 0.0, jy = 0.0, C = 0.0;
  for (int k = 0; k < 9; ++k) {
    rho += f[9 * node + k];
    jx += f[9 * node + k] * EX[k];
    jy += f[9 * node + k] * EY[k];
  }
  for (int k = 0; k < 5; ++k) C += g[5 * node + k];
  const double ux = jx / rho, uy = jy / rho;
  for (int i = 1; i < 9; ++i) {
    int xs = 0, ys = 0;
    int code = cell_code(L, x - EX[i], y - EY[i], &xs, &ys);
    if (code == 0) continue;
    if (!(code == 1 || L->seg_kind[code] == ORC_SEG_NONE || !open[code])) continue;
    double rho_s = rho;
    int xa = 0, ya = 0;
    if (cell_code(L, x + EX[i], y + EY[i], &xa, &ya) == 0) {
      size_t a = (size_t)ya * nx + xa;
      double rho_a = 0.0;
      for (int k = 0; k < 9; ++k) rho_a += f[9 * a + k];
      rho_s = 2.0 * rho - rho_a;
    }
    double feq[9];
    orc_feq(rho_s, -jx / rho_s, -jy / rho_s, feq);
    fz[i] = feq[i];
    if (i <= 4) {
      double gs[5], gz0[5];
      orc_geq(C, -jx / rho_s, -jy / rho_s, L->w0, gs);
      orc_geq(C, ux, uy, L->w0, gz0);
      gz[i] = gs[i] + (1.0 - omega_g) * (g[5 * node + i] - gz0[i]);
    }
  }
}

/* The compound's wall rule of wall_links in the compound-only step, where
 * the velocity of z is the frozen field's u and the ghost's is -u. */
static void wall_links_cde(const orc_lattice *L, int x, int y, const double *g, double ux,
                           double uy, const uint8_t *open, double *gz) {
  const size_t node = (size_t)y * L->nx + x;
  const double omega_g = 1.0 / L->tau_g;
  double C = 0.0;
  for (int k = 0; k < 5; ++k) C += g[5 * node + k];
  double gs[5], gz0[5];
  orc_geq(C, -ux, -uy, L->w0, gs);
  orc_geq(C, ux, uy, L->w0, gz0);
  for (int i = 1; i < 5; ++i) {
    int xs = 0, ys = 0;
    int code = cell_code(L, x - EX[i], y - EY[i], &xs, &ys);
    if (code == 0) continue;
    if (!(code == 1 || L->seg_kind[code] == ORC_SEG_NONE || !open[code])) continue;
    gz[i] = gs[i] + (1.0 - omega_g) * (g[5 * node + i] - gz0[i]);
  }
}

/* open[m]  : nonzero if segment with mask value m is open at step t.
 * c_in[m]  : compound concentration imposed by open inlet m at step t.
 * flux_mass[m], flux_solute[m] : accumulate the net amount of fluid mass and
 *   compound entering the domain through segment m during this step: for
 *   every link from a ghost cell of m into a fluid node z, the population
 *   arriving at z minus the one z sent toward that ghost cell.
 * The per-row partial sums are added in row order, so the result does not
 * depend on the number of threads.
 *
 * Written in pull form: first every fluid node collides (into fp, gp), then
 * every fluid node z gathers each incoming population F(z, i) from the cell
 * s = z - e_i it comes from. */
void orc_step(const orc_lattice *L, const double *f, const double *g,
              double *fn, double *gn, const uint8_t *open, const double *c_in,
              double *flux_mass, double *flux_solute) {
  const int nx = L->nx, ny = L->ny;
  const size_t n = (size_t)nx * ny;
  double wg[5];
  orc_gweights(L->w0, wg);

  double *fp = (double *)calloc(9 * n, sizeof(double));
  double *gp = (double *)calloc(5 * n, sizeof(double));
  double *fu = (double *)calloc(2 * n, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t node = (size_t)y * nx + x;
      if (L->mask[node] == 0)
        collide_node(L, node, f + 9 * node, g + 5 * node, fp + 9 * node,
                     gp + 5 * node, fu + 2 * node);
    }

  memset(fn, 0, sizeof(double) * 9 * n);
  memset(gn, 0, sizeof(double) * 5 * n);
  /* per-row flux partials [ny][256 mask values][mass, solute] */
  double *rowflux = (double *)calloc((size_t)ny * 512, sizeof(double));

#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    double *rf = rowflux + (size_t)y * 512;
    for (int x = 0; x < nx; ++x) {
      size_t node = (size_t)y * nx + x;
      if (L->mask[node] != 0) continue;
      fn[9 * node] = fp[9 * node];
      gn[5 * node] = gp[5 * node];
      for (int i = 1; i < 9; ++i) {
        int opp = OPP[i];
        int has_g = (i <= 4);
        int xs = 0, ys = 0;
        int code = cell_code(L, x - EX[i], y - EY[i], &xs, &ys);
        double out_f = fp[9 * node + opp];        /* sent by z toward s */
        double out_g = has_g ? gp[5 * node + opp] : 0.0;
        if (code == 0) { /* free flight from a fluid neighbour */
          size_t s = (size_t)ys * nx + xs;
          fn[9 * node + i] = fp[9 * s + i];
          if (has_g) gn[5 * node + i] = gp[5 * s + i];
          continue;
        }
        int kind = (code >= 2) ? L->seg_kind[code] : ORC_SEG_NONE;
        if (kind != ORC_SEG_NONE && !open[code]) kind = ORC_SEG_NONE;
        double in_f, in_g = 0.0;
        if (kind == ORC_SEG_NONE) {
          /* wall or closed valve: halfway bounce-back */
          in_f = out_f;
          in_g = out_g;
        } else if (kind == ORC_SEG_INLET) {
          /* moving-wall bounce-back with the wall velocity u_w = -n u(s):
           * F(z, i) = f*(z, opp) - 6 w rho_w (e_opp . u_w) */
          const int32_t *nr = L->seg_nrm + 2 * code;
          double us = inlet_speed(L, code, x, y);
          double uwx = -nr[0] * us, uwy = -nr[1] * us;
          double eu = EX[opp] * uwx + EY[opp] * uwy;
          in_f = out_f - 6.0 * WF[i] * L->rho_w * eu;
          /* anti-bounce-back: Dirichlet value C_in at the halfway wall */
          if (has_g) in_g = -out_g + 2.0 * wg[i] * c_in[code];
        } else if (kind == ORC_SEG_PRESSURE) {
          /* do nothing: the missing population keeps its value of step t
           * (the rescaling below then sets the density); the compound the
           * same where the segment holds C_in, otherwise it leaves with
           * zero gradient (the ghost emits what z emits), the natural
           * outflow condition the paper cites for its outlet */
          in_f = f[9 * node + i];
          if (has_g) in_g = L->seg_fixc[code] ? g[5 * node + i] : gp[5 * node + i];
        } else {
          /* open outlet. Fluid: anti-bounce-back at the reference density
           * rho_w with the node's own velocity (zero normal gradient of u):
           * F(z, i) = -f*(z, opp) + 2 w rho_w [1 + 4.5 (e_i.u)^2 - 1.5 u.u].
           * Compound: zero-gradient, the ghost cell emits what z emits. */
          double ux = fu[2 * node + 0], uy = fu[2 * node + 1];
          double eu = EX[i] * ux + EY[i] * uy;
          in_f = -out_f + 2.0 * WF[i] * L->rho_w *
                             (1.0 + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy));
          if (has_g) in_g = gp[5 * node + i];
        }
        fn[9 * node + i] = in_f;
        rf[2 * code + 0] += in_f - out_f;
        if (has_g) {
          gn[5 * node + i] = in_g;
          rf[2 * code + 1] += in_g - out_g;
        }
      }
      /* the paper's walls replace the bounce-back of wall links */
      if (L->wall_scheme == 1) wall_links(L, x, y, f, g, open, fn + 9 * node, gn + 5 * node);
      /* pressure boundary: rescale the streamed state of the node */
      int m = pressure_segment(L, x, y, open);
      if (m) {
        rf[2 * m + 0] += rescale_f(L, m, fn + 9 * node);
        rf[2 * m + 1] += rescale_g(L, m, gn + 5 * node, c_in);
      }
    }
  }

  for (int y = 0; y < ny; ++y)
    for (int m = 0; m < 256; ++m) {
      if (flux_mass) flux_mass[m] += rowflux[(size_t)y * 512 + 2 * m + 0];
      if (flux_solute) flux_solute[m] += rowflux[(size_t)y * 512 + 2 * m + 1];
    }
  free(rowflux);
  free(fp);
  free(gp);
  free(fu);
}

/* ---------------------------------------------------------------- */
/* Compound lattice alone on a frozen velocity field, t -> t+1         */
/* ---------------------------------------------------------------- */

/* The paper's production path (Results section): the flow reaches its
 * steady state long before the compound does, so the velocity field of
 * each valve configuration is computed once and the advection-diffusion
 * lattice is then advanced on its own, driven by that fixed field. One step
 * of that lattice: at every fluid node, C = sum g_i, the linear equilibrium
 * of Eq. (9) with the given u(x), BGK relaxation (Eq. 8) and the reaction
 * term R - kC of Eq. (2); then free flight with the compound's link rules
 * (walls and closed valves bounce back, open inlets hold C_in by
 * anti-bounce-back, open outlets let the compound leave with zero
 * gradient). ux, uy: ny*nx velocity components (ignored off the fluid).
 * flux_solute[m] accumulates the compound entering through segment m. */
void orc_cde_step(const orc_lattice *L, const double *g, double *gn,
                  const double *ux, const double *uy, const uint8_t *open,
                  const double *c_in, double *flux_solute) {
  const int nx = L->nx, ny = L->ny;
  const size_t n = (size_t)nx * ny;
  double wg[5];
  orc_gweights(L->w0, wg);
  const double omega = 1.0 / L->tau_g;

  double *gp = (double *)calloc(5 * n, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t node = (size_t)y * nx + x;
      if (L->mask[node] != 0) continue;
      const double *gx = g + 5 * node;
      double C = 0.0;
      for (int i = 0; i < 5; ++i) C += gx[i];
      double geq[5];
      orc_geq(C, ux[node], uy[node], L->w0, geq);
      double src = (L->R ? L->R[node] : 0.0) - L->k_decay * C;
      for (int i = 0; i < 5; ++i)
        gp[5 * node + i] = gx[i] - omega * (gx[i] - geq[i]) + wg[i] * src;
    }

  memset(gn, 0, sizeof(double) * 5 * n);
  double *rowflux = (double *)calloc((size_t)ny * 256, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    double *rf = rowflux + (size_t)y * 256;
    for (int x = 0; x < nx; ++x) {
      size_t node = (size_t)y * nx + x;
      if (L->mask[node] != 0) continue;
      gn[5 * node] = gp[5 * node];
      for (int i = 1; i < 5; ++i) {
        int xs = 0, ys = 0;
        int code = cell_code(L, x - EX[i], y - EY[i], &xs, &ys);
        double out = gp[5 * node + OPP[i]];
        if (code == 0) {
          gn[5 * node + i] = gp[5 * ((size_t)ys * nx + xs) + i];
          continue;
        }
        int kind = (code >= 2) ? L->seg_kind[code] : ORC_SEG_NONE;
        if (kind != ORC_SEG_NONE && !open[code]) kind = ORC_SEG_NONE;
        double in;
        if (kind == ORC_SEG_NONE)
          in = out;
        else if (kind == ORC_SEG_INLET)
          in = -out + 2.0 * wg[i] * c_in[code];
        else if (kind == ORC_SEG_PRESSURE)
          in = L->seg_fixc[code] ? g[5 * node + i] : gp[5 * node + i];
        else
          in = gp[5 * node + i];
        gn[5 * node + i] = in;
        rf[code] += in - out;
      }
      if (L->wall_scheme == 1) wall_links_cde(L, x, y, g, ux[node], uy[node], open, gn + 5 * node);
      int m = pressure_segment(L, x, y, open);
      if (m) rf[m] += rescale_g(L, m, gn + 5 * node, c_in);
    }
  }
  for (int y = 0; y < ny; ++y)
    for (int m = 0; m < 256; ++m)
      if (flux_solute) flux_solute[m] += rowflux[(size_t)y * 256 + m];
  free(rowflux);
  free(gp);
}

/* ---------------------------------------------------------------- */
/* Initialisation and read-back                                        */
/* ---------------------------------------------------------------- */

/* f = f^eq(rho, u), g = g^eq(C, u) at every fluid node; zero elsewhere. */
void orc_init_eq(const orc_lattice *L, const double *rho, const double *ux,
                 const double *uy, const double *C, double *f, double *g) {
  size_t n = (size_t)L->nx * L->ny;
  memset(f, 0, sizeof(double) * 9 * n);
  memset(g, 0, sizeof(double) * 5 * n);
  for (size_t k = 0; k < n; ++k) {
    if (L->mask[k] != 0) continue;
    orc_feq(rho[k], ux[k], uy[k], f + 9 * k);
    orc_geq(C[k], ux[k], uy[k], L->w0, g + 5 * k);
  }
}

/* Macroscopic fields of Eq. (7) and C = sum_i g_i; NaN at non-fluid nodes. */
void orc_moments(const orc_lattice *L, const double *f, const double *g,
                 double *rho, double *ux, double *uy, double *C) {
  size_t n = (size_t)L->nx * L->ny;
  for (size_t k = 0; k < n; ++k) {
    if (L->mask[k] != 0) {
      rho[k] = ux[k] = uy[k] = C[k] = NAN;
      continue;
    }
    double r = 0.0, jx = 0.0, jy = 0.0, c = 0.0;
    for (int i = 0; i < 9; ++i) {
      r += f[9 * k + i];
      jx += f[9 * k + i] * EX[i];
      jy += f[9 * k + i] * EY[i];
    }
    for (int i = 0; i < 5; ++i) c += g[5 * k + i];
    rho[k] = r;
    ux[k] = jx / r;
    uy[k] = jy / r;
    C[k] = c;
  }
}

/* Total fluid mass and compound over fluid nodes, Neumaier-compensated. */
void orc_totals(const orc_lattice *L, const double *f, const double *g,
                double *mass, double *solute) {
  size_t n = (size_t)L->nx * L->ny;
  double sm = 0.0, cm = 0.0, ss = 0.0, cs = 0.0;
  for (size_t k = 0; k < n; ++k) {
    if (L->mask[k] != 0) continue;
    for (int i = 0; i < 9; ++i) {
      double v = f[9 * k + i], t = sm + v;
      cm += (fabs(sm) >= fabs(v)) ? (sm - t) + v : (v - t) + sm;
      sm = t;
    }
    for (int i = 0; i < 5; ++i) {
      double v = g[5 * k + i], t = ss + v;
      cs += (fabs(ss) >= fabs(v)) ? (ss - t) + v : (v - t) + ss;
      ss = t;
    }
  }
  *mass = sm + cm;
  *solute = ss + cs;
}

/* Number of OpenMP threads a step uses (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for the following steps (timing of the oracle on one core). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------- */
/* Discrete adjoint of one compound step (test infrastructure)         */
/* ---------------------------------------------------------------- */

/* The compound update t -> t+1 is affine in g for a given fluid state:
 *   collision  g*_i = (1 - w) g_i + (w W_i(u) - k wg_i) C + wg_i R,
 *              W_i(u) = wg_i (1 + e_i.u / cs2), C = sum_j g_j   (Eqs. 2, 8, 9)
 *   streaming  G(z, i) = g*_i(z - e_i)            (fluid source)
 *              G(z, i) = g*_opp(z)                (wall, closed valve)
 *              G(z, i) = -g*_opp(z) + 2 wg_i C_in (open inlet)
 *              G(z, i) = g*_i(z)                  (open outlet)
 * Given lam = dL/dG at t+1, this computes dL/dg at t (lam_out) and adds the
 * step's contribution to dL/dR (per node), dL/dC_in (per mask value) and
 * dL/domega_g. f and g are the populations at time t (u is taken from f).
 * Each node gathers lam* = dL/dg* over every use of its post-collision
 * populations, then applies the transposed collision matrix. */
void orc_adjoint_step(const orc_lattice *L, const double *f, const double *g,
                      const double *lam, double *lam_out, const uint8_t *open,
                      double *dR, double *dcin, double *domega) {
  const int nx = L->nx, ny = L->ny;
  const size_t n = (size_t)nx * ny;
  const double omega = 1.0 / L->tau_g;
  const double cs2 = (1.0 - L->w0) / 2.0;
  double wg[5];
  orc_gweights(L->w0, wg);
  memset(lam_out, 0, sizeof(double) * 5 * n);
  double *rowacc = (double *)calloc((size_t)ny * 257, sizeof(double));

#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    double *ra = rowacc + (size_t)y * 257;
    for (int x = 0; x < nx; ++x) {
      size_t node = (size_t)y * nx + x;
      if (L->mask[node] != 0) continue;
      const double *fx = f + 9 * node, *gx = g + 5 * node, *lx = lam + 5 * node;
      double rho = 0.0, jx = 0.0, jy = 0.0, C = 0.0;
      for (int i = 0; i < 9; ++i) {
        rho += fx[i];
        jx += fx[i] * EX[i];
        jy += fx[i] * EY[i];
      }
      for (int i = 0; i < 5; ++i) C += gx[i];
      double ux = jx / rho, uy = jy / rho;

      double ls[5];
      ls[0] = lx[0];
      for (int j = 1; j < 5; ++j) {
        ls[j] = 0.0;
        int opp = OPP[j];
        int xt = 0, yt = 0;
        int code = cell_code(L, x + EX[j], y + EY[j], &xt, &yt);
        if (code == 0) {
          ls[j] += lam[5 * ((size_t)yt * nx + xt) + j];
        } else {
          int kind = (code >= 2) ? L->seg_kind[code] : ORC_SEG_NONE;
          if (kind != ORC_SEG_NONE && !open[code]) kind = ORC_SEG_NONE;
          if (kind == ORC_SEG_NONE) {
            ls[j] += lx[opp];
          } else if (kind == ORC_SEG_INLET) {
            ls[j] -= lx[opp];
            ra[code] += 2.0 * wg[opp] * lx[opp];
          } /* open outlet ahead: g*_j leaves the domain */
        }
        int xs = 0, ys = 0;
        int scode = cell_code(L, x - EX[j], y - EY[j], &xs, &ys);
        if (scode >= 2 && L->seg_kind[scode] == ORC_SEG_OUTLET && open[scode])
          ls[j] += lx[j]; /* the outlet ghost behind re-emits g*_j */
      }

      double W[5], s = 0.0, dr = 0.0, dw = 0.0;
      for (int j = 0; j < 5; ++j) {
        W[j] = wg[j] * (1.0 + (EX[j] * ux + EY[j] * uy) / cs2);
        s += (omega * W[j] - L->k_decay * wg[j]) * ls[j];
        dr += wg[j] * ls[j];
        dw -= ls[j] * (gx[j] - W[j] * C);
      }
      for (int i = 0; i < 5; ++i) lam_out[5 * node + i] = (1.0 - omega) * ls[i] + s;
      if (dR) dR[node] += dr;
      ra[256] += dw;
    }
  }
  for (int y = 0; y < ny; ++y) {
    for (int m = 0; m < 256; ++m) dcin[m] += rowacc[(size_t)y * 257 + m];
    *domega += rowacc[(size_t)y * 257 + 256];
  }
  free(rowacc);
}
