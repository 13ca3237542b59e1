// Per-node pieces of the coupled step shared by the single-step kernels and
// the two-step kernel: valve phase, wavefront reductions, neighbour offsets,
// plane addressing, the AA-pattern load, and the collision of one node with
// its boundary links. Every kernel that advances the lattice computes a node
// through collide_node, so all of them do the same arithmetic.
#pragma once

#include "gg_device.h"

namespace gg {

struct PhaseNow {
  uint32_t open;
  const GG_CONST double *cin;
  const GG_CONST float *cin_f;  // the same in FP32
  int index;                    // phase number (0 without a schedule)
};

// Valve phase in force during step t (fixed at the start of the step).
__device__ __forceinline__ PhaseNow phase_at(CDesc &L, int64_t t) {
  if (L.n_phases == 0) return {0xFFFFFFFFu, L.seg_cin, L.seg_cin_f, 0};
  int64_t tau = (t - L.t_origin) % L.period;
  if (tau < 0) tau += L.period;
  int k = 0;
  while (k + 1 < L.n_phases && L.phase_start[k + 1] <= tau) ++k;
  return {L.phase_open[k], L.phase_cin[k], L.phase_cin_f[k], k};
}

// Inlet parameters of segment s in the compute type T (pre-rounded for FP32).
template <class T> struct SegT;
template <> struct SegT<double> {
  static __device__ __forceinline__ double umax4(CDesc &L, int s) { return 4.0 * L.seg_umax[s]; }
  static __device__ __forceinline__ double s0(CDesc &L, int s) { return L.seg_s0[s]; }
  static __device__ __forceinline__ double s1(CDesc &L, int s) { return L.seg_s1[s]; }
  static __device__ __forceinline__ double iw2(CDesc &L, int s) { return L.seg_inv_w2[s]; }
  static __device__ __forceinline__ double cin(const PhaseNow &p, int s) { return p.cin[s]; }
  static __device__ __forceinline__ double rho(CDesc &L, int s) { return L.seg_rho[s]; }
};
template <> struct SegT<float> {
  static __device__ __forceinline__ float umax4(CDesc &L, int s) { return L.seg_umax4_f[s]; }
  static __device__ __forceinline__ float s0(CDesc &L, int s) { return L.seg_s0_f[s]; }
  static __device__ __forceinline__ float s1(CDesc &L, int s) { return L.seg_s1_f[s]; }
  static __device__ __forceinline__ float iw2(CDesc &L, int s) { return L.seg_inv_w2_f[s]; }
  static __device__ __forceinline__ float cin(const PhaseNow &p, int s) { return p.cin_f[s]; }
  static __device__ __forceinline__ float rho(CDesc &L, int s) { return L.seg_rho_f[s]; }
};

// Lattice constants in the compute type T: the descriptor's FP64 values, or
// their FP32 roundings stored beside them (no conversion in the kernels).
template <class T> struct DK;
template <> struct DK<double> {
  static __device__ __forceinline__ double rho0(CDesc &L) { return L.rho0; }
  static __device__ __forceinline__ double om_f(CDesc &L) { return L.omega_f; }
  static __device__ __forceinline__ double om_g(CDesc &L) { return L.omega_g; }
  static __device__ __forceinline__ double wga(CDesc &L) { return L.wg_axis; }
  static __device__ __forceinline__ double ics(CDesc &L) { return L.inv_cs2g; }
  static __device__ __forceinline__ double kdec(CDesc &L) { return L.k_decay; }
  static __device__ __forceinline__ double cs(CDesc &L) { return L.c_shift; }
  static __device__ __forceinline__ const GG_CONST CollK<double> &ck(CDesc &L) { return L.ck; }
};
template <> struct DK<float> {
  static __device__ __forceinline__ float rho0(CDesc &L) { return L.rho0_f; }
  static __device__ __forceinline__ float om_f(CDesc &L) { return L.omega_f_f; }
  static __device__ __forceinline__ float om_g(CDesc &L) { return L.omega_g_f; }
  static __device__ __forceinline__ float wga(CDesc &L) { return L.wg_axis_f; }
  static __device__ __forceinline__ float ics(CDesc &L) { return L.inv_cs2g_f; }
  static __device__ __forceinline__ float kdec(CDesc &L) { return L.k_decay_f; }
  static __device__ __forceinline__ float cs(CDesc &L) { return L.c_shift_f; }
  static __device__ __forceinline__ const GG_CONST CollK<float> &ck(CDesc &L) { return L.ck_f; }
};

// e_i . u for direction i (paper Eq. 3 velocities), written out per
// direction: the same value as e_x u_x + e_y u_y, without the products by
// zero and one that IEEE arithmetic would otherwise have to carry out (the
// rest direction gives +0).
template <class T> __device__ __forceinline__ T e_dot_u(int i, T ux, T uy) {
  switch (i) {
    case 0: return T(0);
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

// Sum over the 64 lanes of a wavefront; every lane must be active.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Add per-lane boundary fluxes (up to two segments per lane, seg < 0 for
// none) into the FP64 accumulators: one atomic per segment and wavefront.
__device__ __forceinline__ void flush_flux(double *flux, int sa, double ma, double ca, int sb,
                           double mb, double cb) {
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const int seg = slot ? sb : sa;
    const double dm = slot ? mb : ma;
    const double dc = slot ? cb : ca;
    unsigned long long pend = __ballot(seg >= 0);
    while (pend) {
      const int lead = __ffsll(pend) - 1;
      const int s = __shfl(seg, lead);
      const bool mine = seg == s;
      const double a = wave_sum(mine ? dm : 0.0);
      const double b = wave_sum(mine ? dc : 0.0);
      if ((int)__lane_id() == lead) {
        atomicAdd(flux + 2 * s, a);
        atomicAdd(flux + 2 * s + 1, b);
      }
      pend &= ~__ballot(mine);
    }
  }
}

// Element offset of x + e_k for k = 0..8: wrapped along periodic axes,
// otherwise possibly in the padding around the lattice (always addressable).
struct Neigh {
  uint32_t idx[9];
  __device__ __forceinline__ Neigh(CDesc &L, int x, int y) {
    const int xm = (x == 0 && L.periodic_x) ? L.nx - 1 : x - 1;
    const int xp = (x == L.nx - 1 && L.periodic_x) ? 0 : x + 1;
    const int ym = (y == 0 && L.periodic_y) ? L.ny - 1 : y - 1;
    const int yp = (y == L.ny - 1 && L.periodic_y) ? 0 : y + 1;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int xx = EX[k] > 0 ? xp : (EX[k] < 0 ? xm : x);
      const int yy = EY[k] > 0 ? yp : (EY[k] < 0 ? ym : y);
      idx[k] = (uint32_t)(L.node0 + yy * L.pitch + xx);
    }
  }
};

// Deviations df_i(x,t), dg_i(x,t) in natural order for step parity ODD.
template <class S, bool ODD>
__device__ __forceinline__ void load_state(const Planes<typename Pop<S>::W> &pl, uint32_t node,
                                           uint8_t lc, const Neigh &nb,
                                           typename Pop<S>::T *f, typename Pop<S>::T *g) {
  using P = Pop<S>;
  if (!ODD) {
    if (pl.pairs) {  // (f_i, g_i) side by side: one access each
#pragma unroll
      for (int i = 0; i < 5; ++i) P::ld_pair(pl.at(i, node), f[i], g[i]);
#pragma unroll
      for (int i = 5; i < 9; ++i) f[i] = P::ld(pl.at(i, node));
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = P::ld(pl.at(i, node));
#pragma unroll
      for (int i = 0; i < 5; ++i) g[i] = P::ld(pl.at(9 + i, node));
    }
  } else if (pl.pairs) {
    // streamed in from x - e_i, stored by that node in slot opp(i) (f and g
    // of one direction side by side)
    P::ld_pair(pl.at(0, node), f[0], g[0]);
#pragma unroll
    for (int i = 1; i < 5; ++i) P::ld_pair(pl.at(OPP[i], nb.idx[OPP[i]]), f[i], g[i]);
#pragma unroll
    for (int i = 5; i < 9; ++i) f[i] = P::ld(pl.at(OPP[i], nb.idx[OPP[i]]));
  } else {
    // streamed in from x - e_i, stored by that node in slot opp(i)
    f[0] = P::ld(pl.at(0, node));
#pragma unroll
    for (int i = 1; i < 9; ++i) f[i] = P::ld(pl.at(OPP[i], nb.idx[OPP[i]]));
    g[0] = P::ld(pl.at(9, node));
#pragma unroll
    for (int i = 1; i < 5; ++i) g[i] = P::ld(pl.at(9 + OPP[i], nb.idx[OPP[i]]));
  }
  if (ODD) {
    if (lc != 0) {
      // x - e_i not fluid: this node stored the boundary value in its own slot i
#pragma unroll
      for (int i = 1; i < 9; ++i)
        if ((lc >> (OPP[i] - 1)) & 1) f[i] = P::ld(pl.at(i, node));
#pragma unroll
      for (int i = 1; i < 5; ++i)
        if ((lc >> (OPP[i] - 1)) & 1) g[i] = P::ld(pl.at(9 + i, node));
    }
  }
}

// Boundary fluxes of one lane: up to two segments (a node touches at most
// two), net population change per link, summed over the lane's links in A
// (FP64, or the compute type where the lane's few terms are summed before
// the FP64 wavefront sum) and flushed into the FP64 accumulators.
template <class A> struct FluxT {
  int sa = -1, sb = -1;
  A ma = A(0), ca = A(0), mb = A(0), cb = A(0);
  template <class V> __device__ __forceinline__ void add(int s, V dm, V dc) {
    if (sa < 0 || sa == s) {
      sa = s; ma += (A)dm; ca += (A)dc;
    } else {
      sb = s; mb += (A)dm; cb += (A)dc;
    }
  }
  // every lane of the wavefront must call this
  __device__ __forceinline__ void flush(double *flux) {
    flush_flux(flux, sa, (double)ma, (double)ca, sb, (double)mb, (double)cb);
    sa = sb = -1;
    ma = ca = mb = cb = A(0);
  }
};
using Flux = FluxT<double>;

// Pieces of the two-step passes: 62 owned columns per wavefront (lanes 1..62
// of the columns x0 - 1 .. x0 + 62), the row count of a tile or strip kept
// in its flags above bit 8, lane shifts that carry a population one column
// right (from_left) or left (from_right), and the test whether x - e_j is
// not fluid for a node with link code lc (j = 1..8). The four-step pass
// owns 58 columns (lanes 3..60 of the columns x0 - 3 .. x0 + 60).
constexpr int STRIP_W = 62;
constexpr int STRIP4_W = 58;
__device__ __forceinline__ int strip_rows(int flags) { return flags >> 8; }
template <class T> __device__ __forceinline__ T from_left(T v) { return __shfl_up(v, 1); }
template <class T> __device__ __forceinline__ T from_right(T v) { return __shfl_down(v, 1); }
__device__ __forceinline__ bool src_solid(uint8_t lc, int j) { return (lc >> (OPP[j] - 1)) & 1; }

// Fused multiply-add with one rounding, for both compute types.
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Density and velocity of the fluid at a node from its deviations df
// (paper Eq. 7, sum over i = 0..8): rho = rho0 + sum df_i; the rest part
// w_i rho0 carries no momentum.
template <class T>
__device__ __forceinline__ void node_velocity(CDesc &L, const T *f, T &rho, T &drho, T &ux,
                                              T &uy) {
#pragma clang fp contract(off)
  // the populations moving in +x and in -x, shared by rho and j_x
  const T a = (f[1] + f[5]) + f[8];
  const T b = (f[3] + f[6]) + f[7];
  drho = ((f[0] + f[2]) + f[4]) + (a + b);
  rho = DK<T>::rho0(L) + drho;
  const T jx = a - b;
  const T jy = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
  const T inv_rho = T(1) / rho;
  ux = jx * inv_rho;
  uy = jy * inv_rho;
}

// Compound collision at (x, y) with fluid velocity u: linear equilibrium
// (Eq. 9), BGK (Eq. 8), source R - kC of Eq. 2 distributed with the
// lattice weights. With C = C_s + dC, g^eq_i - w_i C_s = w_i (dC + C e.u / cs2):
// a part even in e_i, w_i dC, and an odd one, w_i C e.u / cs2, so opposite
// directions share every product but the last:
//   pg_i = (1 - om) g_i + om w_i (dC + C e.u / cs2) + w_i src.
template <class T>
__device__ __forceinline__ void compound_collide(CDesc &L, int x, int y, const T *g, T ux, T uy,
                                                 T *pg) {
#pragma clang fp contract(off)
  const GG_CONST CollK<T> &K = DK<T>::ck(L);
  const T dC = g[0] + g[1] + g[2] + g[3] + g[4];
  const T C = DK<T>::cs(L) + dC;
  T src = -DK<T>::kdec(L) * C;
  if (L.has_source) {
    const int rx = x - L.r_x0, ry = y - L.r_y0;
    if (rx >= 0 && rx < L.r_w && ry >= 0 && ry < L.r_h)
      src += (T)((const GG_GLOBAL double *)L.R)[ry * L.r_w + rx];
  }
  const T even0 = fmad(K.g_k0, dC, K.g_w0 * src);
  const T even = fmad(K.g_ka, dC, DK<T>::wga(L) * src);
  const T oddC = K.g_ki * C;
  const T ox = oddC * ux, oy = oddC * uy;
  pg[0] = fmad(K.g_omc, g[0], even0);
  pg[1] = fmad(K.g_omc, g[1], even + ox);
  pg[3] = fmad(K.g_omc, g[3], even - ox);
  pg[2] = fmad(K.g_omc, g[2], even + oy);
  pg[4] = fmad(K.g_omc, g[4], even - oy);
}

// One pair of opposite fluid directions i, o = opp(i) with e = e_i.u: the
// even part k (q + 4.5 rho e^2) and the odd part r e of om w (f^eq - w rho0)
// (k = om w, r = 3 om w rho, q = drho - 1.5 rho u.u).
template <class T>
__device__ __forceinline__ void relax_pair(T omc, T fi, T fo, T e, T k, T r, T r45, T q, T &pi,
                                           T &po) {
#pragma clang fp contract(off)
  const T ev = k * fmad(r45 * e, e, q);
  const T od = r * e;
  pi = fmad(omc, fi, ev + od);
  po = fmad(omc, fo, ev - od);
}

// BGK relaxation of the fluid deviations toward the quadratic equilibrium
// (Eqs. 4-6): f^eq_i - w_i rho0 = w_i (drho + rho (3 e.u + 4.5 (e.u)^2 -
// 1.5 u.u)), split into the part even in e_i, w_i (drho - 1.5 rho u.u +
// 4.5 rho (e.u)^2), and the odd one, 3 w_i rho e.u; opposite directions
// share both:  pf_i = (1 - om) f_i + om w_i (even_i +- odd_i).
template <class T>
__device__ __forceinline__ void fluid_collide(CDesc &L, const T *f, T rho, T drho, T ux, T uy,
                                              T usq, T *pf) {
#pragma clang fp contract(off)
  const GG_CONST CollK<T> &K = DK<T>::ck(L);
  const T q = fmad(rho, T(-1.5) * usq, drho);
  const T r45 = T(4.5) * rho;
  const T ra = K.f_k3a * rho, rd = K.f_k3d * rho;
  pf[0] = fmad(K.f_omc, f[0], K.f_k0 * q);
  relax_pair<T>(K.f_omc, f[1], f[3], ux, K.f_ka, ra, r45, q, pf[1], pf[3]);
  relax_pair<T>(K.f_omc, f[2], f[4], uy, K.f_ka, ra, r45, q, pf[2], pf[4]);
  relax_pair<T>(K.f_omc, f[5], f[7], ux + uy, K.f_kd, rd, r45, q, pf[5], pf[7]);
  relax_pair<T>(K.f_omc, f[6], f[8], uy - ux, K.f_kd, rd, r45, q, pf[6], pf[8]);
}

// Collision of fluid node (x, y) with link code lc, from the deviations f, g
// of step t (phase ph): post-collision deviations pf, pg, and in_f[j],
// in_g[j], the value that arrives at (x, y) along direction j at t + 1 when
// x - e_j is not fluid (bounce-back from a wall or closed valve, or the rule
// of an open segment). Fluxes through open segments go into fx when count.
// nbr, when given, holds the mask values of the cells x + e_k (k = 1..8,
// wrapped on periodic axes, walls beyond the others) loaded beforehand, as
// bytes k - 1 of nbr[0] (k = 1..4) and nbr[1] (k = 5..8).
//
// PRESS compiles the pressure-boundary rule in. The two-step passes leave it
// out unless the lattice has pressure segments (their own instantiation),
// which keeps the node's pre-collision populations out of the others'
// register budget and their control flow as it was; without it an open
// pressure link would take the outlet rule.
template <class T, bool PRESS = true, class FX = Flux>
__device__ __forceinline__ void collide_node(CDesc &L, int x, int y, uint8_t lc, bool seg_tile,
                                             const PhaseNow &ph, const T *f, const T *g, T *pf,
                                             T *pg, T *in_f, T *in_g, FX &fx, bool count,
                                             const uint32_t *nbr = nullptr) {
  // Every kernel that advances the lattice inlines this function; the fused
  // multiply-adds are written out and no other contraction is allowed, so
  // each of them rounds exactly the same way whatever code surrounds it.
#pragma clang fp contract(off)
  const int nx = L.nx, ny = L.ny, pitch = L.pitch;
  const T rho0 = DK<T>::rho0(L);
  T rho, drho, ux, uy;
  node_velocity<T>(L, f, rho, drho, ux, uy);
  const T usq = fmad(ux, ux, uy * uy);

  fluid_collide<T>(L, f, rho, drho, ux, uy, usq, pf);
  compound_collide<T>(L, x, y, g, ux, uy, pg);
  const T cs = DK<T>::cs(L);
  const T wga = DK<T>::wga(L);
  const T wg[5] = {T(1) - T(4) * wga, wga, wga, wga, wga};

  // Value arriving at x along direction j when x - e_j is not fluid: the
  // bounced population f*(x, opp j) for a wall or closed valve; open
  // segments overwrite below. (For fluid x - e_j the same slot carries
  // f*(x, opp j) to that neighbour.)
#pragma unroll
  for (int j = 0; j < 9; ++j) in_f[j] = pf[OPP[j]];
#pragma unroll
  for (int j = 0; j < 5; ++j) in_g[j] = pg[OPP[j]];

  if (seg_tile && lc != 0) {
    // (every rule below is written for the deviations; w_j = w_opp(j), so
    // the rest parts cancel except where noted)
#pragma unroll
    for (int j = 1; j < 9; ++j) {
      if (!((lc >> (OPP[j] - 1)) & 1)) continue;  // x - e_j is fluid
      int sx = x - EX[j], sy = y - EY[j];
      bool inside = true;
      if (sx < 0 || sx >= nx) {
        if (L.periodic_x) sx = (sx + nx) % nx; else inside = false;
      }
      if (sy < 0 || sy >= ny) {
        if (L.periodic_y) sy = (sy + ny) % ny; else inside = false;
      }
      const int code = nbr ? (int)((nbr[(OPP[j] - 1) >> 2] >> (8 * ((OPP[j] - 1) & 3))) & 0xFFu)
                     : inside ? (int)((const GG_GLOBAL uint8_t *)L.mask)[L.node0 + sy * pitch + sx]
                              : GG_MASK_WALL;
      if (code < GG_FIRST_SEGMENT) continue;
      const int s = code - GG_FIRST_SEGMENT;
      if (!((ph.open >> s) & 1u)) continue;  // closed valve: a wall
      T vf, vg = T(0);
      if (L.seg_kind[s] == GG_SEG_INLET) {
        // moving-wall bounce-back, wall velocity -n u(s) with a parabolic
        // profile across the segment; anti-bounce-back for C_in
        const T coord = L.seg_nx[s] != 0 ? (T)y : (T)x;
        const T us = SegT<T>::umax4(L, s) * (coord - SegT<T>::s0(L, s)) *
                     (SegT<T>::s1(L, s) - coord) * SegT<T>::iw2(L, s);
        const T en = (T)(EX[j] * L.seg_nx[s] + EY[j] * L.seg_ny[s]);
        vf = fmad(T(-6) * (T)WF[j] * rho0 * en, us, pf[OPP[j]]);
        if (j < 5) vg = fmad(T(2) * wg[j], SegT<T>::cin(ph, s) - cs, -pg[OPP[j]]);
      } else if (PRESS && L.seg_kind[s] == GG_SEG_PRESSURE) {
        // do nothing: the node's own value of step t (the density is set by
        // the rescaling after the step); the compound alike where it is
        // held, else zero-gradient as at an outlet
        vf = f[j];
        if (j < 5) vg = L.seg_holdc[s] ? g[j] : pg[j];
      } else {
        // outflow at the reference density with the node's own u;
        // the compound leaves with zero gradient
        const T eu = e_dot_u<T>(j, ux, uy);
        vf = fmad(T(2) * (T)WF[j] * rho0, fmad(T(4.5) * eu, eu, T(-1.5) * usq), -pf[OPP[j]]);
        if (j < 5) vg = pg[j];
      }
      const T dm = vf - pf[OPP[j]];
      const T dc = (j < 5) ? vg - pg[OPP[j]] : T(0);
      in_f[j] = vf;
      if (j < 5) in_g[j] = vg;
      if (count) fx.add(s, dm, dc);
    }
  }
}

// Link rules of the compound alone (the compound lines of collide_node):
// in_g[j], the value arriving at (x, y) along j when x - e_j is not fluid,
// from the pre- and post-collision g, pg; solute fluxes through open
// segments into fx.
template <class T, bool PRESS = true>
__device__ __forceinline__ void compound_links(CDesc &L, int x, int y, uint8_t lc, bool seg_tile,
                                               const PhaseNow &ph, const T *g, const T *pg,
                                               T *in_g, Flux &fx, bool count) {
#pragma clang fp contract(off)
  const int nx = L.nx, ny = L.ny, pitch = L.pitch;
  const T cs = DK<T>::cs(L);
  const T wga = DK<T>::wga(L);
  const T wg[5] = {T(1) - T(4) * wga, wga, wga, wga, wga};
#pragma unroll
  for (int j = 0; j < 5; ++j) in_g[j] = pg[OPP[j]];
  if (!seg_tile || lc == 0) return;
#pragma unroll
  for (int j = 1; j < 5; ++j) {
    if (!((lc >> (OPP[j] - 1)) & 1)) continue;  // x - e_j is fluid
    int sx = x - EX[j], sy = y - EY[j];
    bool inside = true;
    if (sx < 0 || sx >= nx) {
      if (L.periodic_x) sx = (sx + nx) % nx; else inside = false;
    }
    if (sy < 0 || sy >= ny) {
      if (L.periodic_y) sy = (sy + ny) % ny; else inside = false;
    }
    const int code = inside ? (int)((const GG_GLOBAL uint8_t *)L.mask)[L.node0 + sy * pitch + sx]
                            : GG_MASK_WALL;
    if (code < GG_FIRST_SEGMENT) continue;
    const int s = code - GG_FIRST_SEGMENT;
    if (!((ph.open >> s) & 1u)) continue;  // closed valve: a wall
    const T vg = L.seg_kind[s] == GG_SEG_INLET
                     ? fmad(T(2) * wg[j], SegT<T>::cin(ph, s) - cs, -pg[OPP[j]])
                 : (PRESS && L.seg_kind[s] == GG_SEG_PRESSURE && L.seg_holdc[s]) ? g[j]
                                                                               : pg[j];
    in_g[j] = vg;
    if (count) fx.add(s, 0.0, (double)(vg - pg[OPP[j]]));
  }
}

// Pressure boundary (Eq. 10): the first segment, in direction order of the
// source cells x - e_j, that is a pressure segment open at phase ph, or -1.
// nbr as for collide_node (required).
__device__ __forceinline__ int pressure_source(CDesc &L, uint8_t lc, const PhaseNow &ph,
                                               const uint32_t *nbr) {
  int s = -1;
#pragma unroll
  for (int j = 1; j < 9; ++j) {
    if (s >= 0 || !((lc >> (OPP[j] - 1)) & 1)) continue;  // found, or x - e_j fluid
    const int code = (int)((nbr[(OPP[j] - 1) >> 2] >> (8 * ((OPP[j] - 1) & 3))) & 0xFFu);
    if (code < GG_FIRST_SEGMENT) continue;
    const int q = code - GG_FIRST_SEGMENT;
    if (L.seg_kind[q] == GG_SEG_PRESSURE && ((ph.open >> q) & 1u)) s = q;
  }
  return s;
}

// The rescaling of a node that takes boundary values from the open pressure
// segment s at a step of phase ph, applied to its streamed state (the
// deviations df, dg): every f_i multiplied so that rho = rho_s (velocity
// unchanged; skipped unless fluid), and where the segment holds the
// compound, every g_i so that C = C_in, or the equilibrium at rest of C_in
// where C <= 0. dm, dc: the mass and compound added. In the deviation form
// gamma (w rho0 + df) - w rho0 = gamma df + (gamma - 1) w rho0.
template <class T>
__device__ __forceinline__ void rescale_node(CDesc &L, int s, const PhaseNow &ph, bool fluid,
                                             T *f, T *g, double &dm, double &dc) {
#pragma clang fp contract(off)
  dm = dc = 0.0;
  if (fluid) {
    T drho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const T rho = (T)L.rho0 + drho;
    const T rs = SegT<T>::rho(L, s);
    const T gam = rs / rho;
    const T rest = (gam - T(1)) * (T)L.rho0;
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = fmad(gam, f[i], rest * (T)WF[i]);
    dm = (double)rs - (double)rho;
  }
  if (L.seg_holdc[s]) {
    const T cs = (T)L.c_shift;
    const T wga = (T)L.wg_axis;
    const T wg[5] = {T(1) - T(4) * wga, wga, wga, wga, wga};
    const T C = cs + (g[0] + g[1] + g[2] + g[3] + g[4]);
    const T cin = SegT<T>::cin(ph, s);
    if (C > T(0)) {
      const T gam = cin / C;
      const T rest = (gam - T(1)) * cs;
#pragma unroll
      for (int i = 0; i < 5; ++i) g[i] = fmad(gam, g[i], rest * wg[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 5; ++i) g[i] = wg[i] * (cin - cs);
    }
    dc = (double)cin - (double)C;
  }
}

}  // namespace gg
