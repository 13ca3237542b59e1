/*
 * step_emu.c - storage-rounded replay of one coupled time step, for tests.
 *
 * Test instrument, not part of the library and not the oracle: it replays
 * the arithmetic the GPU kernels do on the deviations from rest
 * (h_i = f_i - w_i rho0, k_i = g_i - w_i C_s), in the kernels' operation
 * order and compute type, with every stored population rounded to the
 * storage type, so that the GPU state after some steps can be compared with
 * it bit for bit. A difference then points at a bug rather than at precision
 * loss. The scheme itself (paper Eqs. 4-9: BGK collision of the D2Q9 fluid
 * toward the quadratic equilibrium, BGK collision of the D2Q5 compound
 * toward the linear equilibrium driven by the same node's velocity, the
 * source R - kC of Eq. 2, streaming) and the link rules (halfway
 * bounce-back, the moving-wall inlet with anti-bounce-back for C_in, the
 * outflow at rho0 with zero-gradient compound) are those of the oracle; the
 * operation order below is the kernels' (one rounding per written product,
 * sum or fused multiply-add, no contraction: built with -ffp-contract=off).
 *
 * Compute type EMU_T (float or double, chosen at build time). Storage:
 * 0 the compute type itself, 1 IEEE binary16 (rounded to nearest even).
 * Layout: natural order, plane i of n = nx*ny values, node (x, y) at y*nx+x.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifndef EMU_T
#define EMU_T float
#endif
typedef EMU_T T;

#define NSEG 16
#define NPH 64

/* D2Q9 directions (paper Eq. 3): 0 rest, 1..4 +x, +y, -x, -y, 5..8 the
 * diagonals (+1,+1), (-1,+1), (-1,-1), (+1,-1); 0..4 are the D2Q5 set. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int REV[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* weights of Eq. 6 in double, as the kernels hold them */
static const double W9[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

typedef struct emu_lattice {
  int32_t nx, ny, periodic_x, periodic_y;
  const uint8_t *mask;              /* ny*nx: 0 fluid, 1 wall, 2.. segment */
  double tau_f, D, w0, rho0, k_decay, c_shift;
  int32_t storage;                  /* 0 compute type, 1 binary16 */
  int32_t seg_kind[NSEG];           /* 0 unset, 1 inlet, 2 outlet */
  int32_t seg_nx[NSEG], seg_ny[NSEG];
  double seg_umax[NSEG], seg_s0[NSEG], seg_s1[NSEG], seg_cin[NSEG];
  int32_t n_phases, pad;
  int64_t period, t_origin;
  int64_t phase_start[NPH];
  uint32_t phase_open[NPH];
  double phase_cin[NPH][NSEG];      /* merged with the segment defaults */
  int32_t r_x0, r_y0, r_w, r_h;     /* source box (r_w = 0: none) */
  const double *R;                  /* r_w*r_h, row-major */
} emu_lattice;

/* ---- binary16 <-> binary32, round to nearest even ---------------------- */
static uint16_t to_half_bits(float v) {
  uint32_t u;
  memcpy(&u, &v, 4);
  const uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
  const uint32_t a = u & 0x7FFFFFFFu;
  if (a >= 0x7F800000u) /* inf or NaN */
    return (uint16_t)(sign | 0x7C00u | (a > 0x7F800000u ? 0x200u : 0u));
  if (a >= 0x477FF000u) return (uint16_t)(sign | 0x7C00u); /* rounds to inf */
  if (a < 0x38800000u) {
    /* below the smallest normal half (2^-14): a multiple of 2^-24 */
    if (a < 0x33000000u) return sign; /* below half of 2^-24 (ties to 0) */
    const int e = (int)(a >> 23);           /* biased binary32 exponent */
    const uint32_t m = (a & 0x7FFFFFu) | 0x800000u;
    const int shift = 126 - e;               /* value = m * 2^(e-150); unit 2^-24 */
    const uint32_t q = m >> shift, rem = m & ((1u << shift) - 1u), half = 1u << (shift - 1);
    const uint32_t r = q + ((rem > half || (rem == half && (q & 1u))) ? 1u : 0u);
    return (uint16_t)(sign | r);
  }
  /* normal: rebias the exponent, keep 10 of 23 mantissa bits */
  const uint32_t rem = a & 0x1FFFu, q = (a - 0x38000000u) >> 13;
  const uint32_t r = q + ((rem > 0x1000u || (rem == 0x1000u && (q & 1u))) ? 1u : 0u);
  return (uint16_t)(sign | r);
}

static float from_half_bits(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  const uint32_t e = (h >> 10) & 0x1Fu, m = h & 0x3FFu;
  float v;
  if (e == 0) {
    v = ldexpf((float)m, -24);
  } else if (e == 31) {
    uint32_t u = sign | 0x7F800000u | (m << 13);
    memcpy(&v, &u, 4);
    return v;
  } else {
    uint32_t u = ((e + 112u) << 23) | (m << 13);
    memcpy(&v, &u, 4);
  }
  uint32_t u;
  memcpy(&u, &v, 4);
  u |= sign;
  memcpy(&v, &u, 4);
  return v;
}

uint16_t emu_to_half(float v) { return to_half_bits(v); }
float emu_from_half(uint16_t h) { return from_half_bits(h); }

static T stored(const emu_lattice *L, T v) {
  if (L->storage == 1) return (T)from_half_bits(to_half_bits((float)v));
  return v;
}

/* e_i . u written out per direction, as the kernels form it (+0 for the
 * rest direction) */
static T edu(int i, T ux, T uy) {
  switch (i) {
    case 0: return (T)0;
    case 1: return ux;
    case 2: return uy;
    case 3: return -ux;
    case 4: return -uy;
    case 5: return ux + uy;
    case 6: return uy - ux;
    case 7: return -(ux + uy);
    default: return ux - uy;
  }
}

static T fused(T a, T b, T c) {
  return sizeof(T) == 4 ? (T)fmaf((float)a, (float)b, (float)c) : (T)fma((double)a, (double)b, (double)c);
}

/* om w_axis of the fluid: omega / 9 with at most p - 4 significant bits,
 * and a multiple of 2^-p where 9 ka < 1/2 */
static double fluid_ka(double omega, int p) {
  const double ka = omega / 9.0;
  int ex;
  frexp(ka, &ex);
  int e = ex - (p - 4);
  double q = ldexp(nearbyint(ldexp(ka, -e)), e);
  if (9.0 * q < 0.5 && e < -p) {
    e = -p;
    q = ldexp(nearbyint(ldexp(ka, -e)), e);
  }
  return q;
}

double emu_fluid_ka(double omega, int p) { return fluid_ka(omega, p); }

/* phase in force during step t (fixed at the start of the step) */
static int phase_of(const emu_lattice *L, int64_t t) {
  if (L->n_phases == 0) return -1;
  int64_t tau = (t - L->t_origin) % L->period;
  if (tau < 0) tau += L->period;
  int k = 0;
  while (k + 1 < L->n_phases && L->phase_start[k + 1] <= tau) ++k;
  return k;
}

/* mask value of the cell (x, y) seen from the lattice: wrapped along
 * periodic axes, wall beyond the other edges */
static int cell(const emu_lattice *L, int x, int y) {
  if (x < 0 || x >= L->nx) {
    if (!L->periodic_x) return 1;
    x = (x + L->nx) % L->nx;
  }
  if (y < 0 || y >= L->ny) {
    if (!L->periodic_y) return 1;
    y = (y + L->ny) % L->ny;
  }
  return L->mask[(size_t)y * L->nx + x];
}

/* One step from the deviations h (9 planes) and k (5 planes) at time t to
 * h_out, k_out at t + 1, rounded to the storage type. Entries off the
 * fluid are left as they are in the outputs. */
void emu_step(const emu_lattice *L, int64_t t, const T *h, const T *k, T *h_out, T *k_out) {
  const int nx = L->nx, ny = L->ny;
  const size_t n = (size_t)nx * ny;
  /* the kernels' constants: derived in double, then taken to the compute type */
  const double cs2g = (1.0 - L->w0) / 2.0;
  const double tau_g = 0.5 + L->D / cs2g;
  const T om_g = (T)(1.0 / tau_g);
  const T ics = (T)(1.0 / cs2g), rho0 = (T)L->rho0, cs = (T)L->c_shift;
  const T wa = (T)((1.0 - L->w0) / 4.0);
  const T wg[5] = {(T)1 - (T)4 * wa, wa, wa, wa, wa};
  /* relaxation written as (1 - om) x + (om w_i) x^eq-part, with the
   * library's constants: for the fluid om w_axis = ka rounded to p - 4
   * significant bits (and to a multiple of 2^-p where 9 ka < 1/2), so that
   * 9 ka, 1 - 9 ka and every product with the weights are exact; for the
   * compound the rounded 1 - om, the rate 1 - (1 - om) that goes with it,
   * and its products with the weights */
  const int p = sizeof(T) == 4 ? 24 : 53;
  const T f_ka = (T)fluid_ka(1.0 / L->tau_f, p);
  const T f_omc = (T)1 - (T)9 * f_ka;
  const T f_k0 = (T)4 * f_ka, f_kd = f_ka * (T)0.25, f_k3a = (T)3 * f_ka, f_k3d = f_k3a * (T)0.25;
  const T g_omc = (T)1 - om_g, g_ome = (T)1 - g_omc;
  const T g_ka = g_ome * wa, g_k0 = g_ome - (T)4 * g_ka, g_ki = g_ka * ics;
  const T fk[9] = {f_k0, f_ka, f_ka, f_ka, f_ka, f_kd, f_kd, f_kd, f_kd};
  const T fr3[9] = {0, f_k3a, f_k3a, f_k3a, f_k3a, f_k3d, f_k3d, f_k3d, f_k3d};
  const int ph = phase_of(L, t);
  const uint32_t open = ph < 0 ? 0xFFFFFFFFu : L->phase_open[ph];
  /* post-collision values of every node, and the value that arrives at each
   * node along each direction from a non-fluid cell */
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const size_t id = (size_t)y * nx + x;
      if (L->mask[id] != 0) continue;
      T f[9], g[5], pf[9], pg[5], inf[9], ing[5];
      for (int i = 0; i < 9; ++i) f[i] = h[i * n + id];
      for (int i = 0; i < 5; ++i) g[i] = k[i * n + id];
      /* moments, Eq. 7, on the deviations */
      /* the populations moving in +x (a) and in -x (b), shared with j_x */
      const T a = (f[1] + f[5]) + f[8];
      const T b = (f[3] + f[6]) + f[7];
      const T dr = ((f[0] + f[2]) + f[4]) + (a + b);
      const T rho = rho0 + dr;
      const T jx = a - b;
      const T jy = ((f[2] - f[4]) + (f[5] - f[7])) + (f[6] - f[8]);
      const T ir = (T)1 / rho;
      const T ux = jx * ir, uy = jy * ir;
      const T uu = fused(ux, ux, uy * uy);
      /* fluid: f_i^eq - w_i rho0 = w_i (drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)),
       * the even part w_i (q + 4.5 rho (e.u)^2) with q = drho - 1.5 rho u.u
       * and the odd part 3 w_i rho e.u, each times om; pf_i = (1 - om) f_i + both */
      const T q = fused(rho, (T)(-1.5) * uu, dr);
      const T r45 = (T)4.5 * rho;
      pf[0] = fused(f_omc, f[0], f_k0 * q);
      for (int i = 1; i < 5; ++i) {
        /* i and its opposite REV[i] share e.u up to the sign; e.u as the
         * kernels form it for the direction of the pair they take first */
        const int a = (i <= 2) ? i : 4 + i - 2; /* 1, 2, 5, 6 */
        const int o = REV[a];
        const T eu = edu(a, ux, uy);
        const T ev = fk[a] * fused(r45 * eu, eu, q);
        const T od = (fr3[a] * rho) * eu;
        pf[a] = fused(f_omc, f[a], ev + od);
        pf[o] = fused(f_omc, f[o], ev - od);
      }
      /* compound: g_i^eq - w_i C_s = w_i (dC + C e.u / cs2), plus w_i (R - kC);
       * pg_i = (1 - om) g_i + om w_i dC + w_i src +- om w_i C e.u / cs2 */
      T dc = g[0];
      for (int i = 1; i < 5; ++i) dc = dc + g[i];
      const T C = cs + dc;
      T src = -(T)L->k_decay * C;
      if (L->R && L->r_w > 0) {
        const int rx = x - L->r_x0, ry = y - L->r_y0;
        if (rx >= 0 && rx < L->r_w && ry >= 0 && ry < L->r_h) src += (T)L->R[(size_t)ry * L->r_w + rx];
      }
      const T even0 = fused(g_k0, dc, wg[0] * src);
      const T even = fused(g_ka, dc, wa * src);
      const T oddc = g_ki * C;
      const T ox = oddc * ux, oy = oddc * uy;
      pg[0] = fused(g_omc, g[0], even0);
      pg[1] = fused(g_omc, g[1], even + ox);
      pg[3] = fused(g_omc, g[3], even - ox);
      pg[2] = fused(g_omc, g[2], even + oy);
      pg[4] = fused(g_omc, g[4], even - oy);
      /* links from non-fluid cells: bounce-back, or an open segment's rule */
      for (int j = 0; j < 9; ++j) inf[j] = pf[REV[j]];
      for (int j = 0; j < 5; ++j) ing[j] = pg[REV[j]];
      for (int j = 1; j < 9; ++j) {
        const int code = cell(L, x - CX[j], y - CY[j]);
        if (code < 2) continue;
        const int s = code - 2;
        if (!((open >> s) & 1u)) continue; /* closed valve: a wall */
        if (L->seg_kind[s] == 1) {
          const T q = L->seg_nx[s] != 0 ? (T)y : (T)x;
          const T s0 = (T)L->seg_s0[s], s1 = (T)L->seg_s1[s];
          const T iw2 = (T)(1.0 / ((L->seg_s1[s] - L->seg_s0[s]) * (L->seg_s1[s] - L->seg_s0[s])));
          const T us = (((T)(4.0 * L->seg_umax[s]) * (q - s0)) * (s1 - q)) * iw2;
          const T en = (T)(CX[j] * L->seg_nx[s] + CY[j] * L->seg_ny[s]);
          inf[j] = fused((((T)(-6) * (T)W9[j]) * rho0) * en, us, pf[REV[j]]);
          if (j < 5) {
            const T cin = (T)(ph < 0 ? L->seg_cin[s] : L->phase_cin[ph][s]);
            ing[j] = fused((T)2 * wg[j], cin - cs, -pg[REV[j]]);
          }
        } else {
          const T eu = edu(j, ux, uy);
          inf[j] = fused(((T)2 * (T)W9[j]) * rho0, fused((T)4.5 * eu, eu, (T)(-1.5) * uu), -pf[REV[j]]);
          if (j < 5) ing[j] = pg[j];
        }
      }
      /* stream: f_i(x + e_i, t + 1) = pf_i(x) into fluid neighbours; the
       * values arriving from non-fluid cells are this node's own */
      for (int i = 0; i < 9; ++i) {
        if (cell(L, x - CX[i], y - CY[i]) != 0) h_out[i * n + id] = stored(L, inf[i]);
        int xx = x + CX[i], yy = y + CY[i];
        if (xx < 0 || xx >= nx) {
          if (!L->periodic_x) continue;
          xx = (xx + nx) % nx;
        }
        if (yy < 0 || yy >= ny) {
          if (!L->periodic_y) continue;
          yy = (yy + ny) % ny;
        }
        const size_t jd = (size_t)yy * nx + xx;
        if (L->mask[jd] == 0) h_out[i * n + jd] = stored(L, pf[i]);
      }
      for (int i = 0; i < 5; ++i) {
        if (cell(L, x - CX[i], y - CY[i]) != 0) k_out[i * n + id] = stored(L, ing[i]);
        int xx = x + CX[i], yy = y + CY[i];
        if (xx < 0 || xx >= nx) {
          if (!L->periodic_x) continue;
          xx = (xx + nx) % nx;
        }
        if (yy < 0 || yy >= ny) {
          if (!L->periodic_y) continue;
          yy = (yy + ny) % ny;
        }
        const size_t jd = (size_t)yy * nx + xx;
        if (L->mask[jd] == 0) k_out[i * n + jd] = stored(L, pg[i]);
      }
    }
}
