// Device-side data of the coupled lattice: descriptor layout shared by the
// host runtime and the gfx950 kernels, lattice constants and storage traits.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <limits>

#include "gg.h"

namespace gg {

// D2Q9 velocity set of paper Eq. 3 (0 rest; 1..4 axes; 5..8 diagonals) and
// the weights of Eq. 6. Directions 0..4 double as the D2Q5 compound lattice.
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr double WF[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Link code byte per node: bit k-1 set <=> cell x + e_k is not fluid
// (k = 1..8). NOT_FLUID marks a node that is not updated.
constexpr uint8_t NOT_FLUID = 0xFF;

// Constants of the two BGK collisions in the compute type T, in the form
// the collision evaluates them: x* = omc x + (om w_i) x^eq-part, with the
// relaxation rate folded into the weights (paper Eqs. 4-6 for the fluid,
// Eqs. 8-9 for the compound).
//
// Fluid: ka = om w_axis is taken with at most p - 4 significant bits (p the
// mantissa width of T; also a multiple of 2^-p when 9 ka < 1/2), so that
// the rate actually used, 9 ka, and every other constant (om w_0 = 4 ka,
// om w_diag = ka / 4, 3 om w_axis, 3 om w_diag) is exact in T, and
// 1 - 9 ka is exact as well. The weights' own rounding then moves neither
// the mass nor the momentum that the relaxation carries: with weights
// rounded one by one, the momentum of every node grew or shrank by a fixed
// factor of about 1e-7 per step in FP32, which acts as a body force on the
// whole flow. The rate moves by at most 2^(4-p) relative (1e-6 in FP32)
// for om >= 9/32, and by at most 2^-(p+1) 9/om below.
//
// Compound: omc is 1 - om rounded, ome = 1 - omc the rate used (1 - om is
// exact for om >= 1/2, otherwise omc lies in [1/2, 1), where 1 - omc is
// exact), and the rest product is ome - 4 (ome w_axis), exact for axis
// weights (1 - w0)/4 with 0 <= w0 <= 1/2: the five products sum to ome and
// the collision carries no bias in proportion to C.
template <class T> struct CollK {
  T f_omc, f_k0, f_ka, f_kd, f_k3a, f_k3d;  // 1 - om_f; om w_0, w_axis, w_diag; 3 om w_axis, w_diag
  T g_omc, g_k0, g_ka, g_ki, g_w0, g_pad;   // 1 - om_g; om w_0, w_axis; om w_axis / cs2; 1 - 4 w_axis
};

// Host side: om w_axis of the fluid rounded as described above.
inline double collk_fluid_ka(double omega_f, int p) {
  const double ka = omega_f / 9.0;
  int ex;
  std::frexp(ka, &ex);                 // ka = m 2^ex, m in [1/2, 1)
  int e = ex - (p - 4);                // keep p - 4 bits
  double q = std::ldexp(std::nearbyint(std::ldexp(ka, -e)), e);
  if (9.0 * q < 0.5 && e < -p) {       // 1 - 9 ka exact: a multiple of 2^-p
    e = -p;
    q = std::ldexp(std::nearbyint(std::ldexp(ka, -e)), e);
  }
  return q;
}

template <class T>
inline CollK<T> make_collk(double omega_f, double omega_g, double wg_axis, double inv_cs2g) {
#pragma clang fp contract(off)
  CollK<T> k;
  const int p = std::numeric_limits<T>::digits;
  const T ka = (T)collk_fluid_ka(omega_f, p);
  k.f_omc = T(1) - T(9) * ka;
  k.f_k0 = T(4) * ka;
  k.f_ka = ka;
  k.f_kd = ka * T(0.25);
  k.f_k3a = T(3) * ka;
  k.f_k3d = k.f_k3a * T(0.25);
  const T omg = (T)omega_g;
  k.g_omc = T(1) - omg;
  const T gome = T(1) - k.g_omc;
  const T wga = (T)wg_axis;
  k.g_ka = gome * wga;
  k.g_k0 = gome - T(4) * k.g_ka;
  k.g_ki = k.g_ka * (T)inv_cs2g;
  k.g_w0 = T(1) - T(4) * wga;
  k.g_pad = T(0);
  return k;
}

// Tile flag: some node of the tile has a link into a boundary segment.
constexpr int TILE_TOUCHES_SEGMENT = 1;

// One launched tile: lattice (instance) index, origin, flags.
struct Tile {
  int32_t inst, x0, y0, flags;
};

constexpr int NPOP = 14;  // 9 f planes then 5 g planes

// Everything a kernel needs about one lattice. Lives in device memory and
// is read with uniform (scalar) loads; the host re-uploads it when the
// parameters change. The time counter lives apart (*t) so that uploads
// never race with the device-side advance.
//
// Plane layout: node (x, y) sits at element node0 + y*pitch + x. Rows are
// padded (pitch > nx, a multiple of 64 elements) and one padding row lies
// before and after the lattice, so the cells x = -1, x = nx, y = -1 and
// y = ny are addressable: stores toward a non-fluid neighbour outside the
// lattice land there and are never read. The population planes are laid
// out plane-major or paired (see Planes).
struct LatDesc {
  int32_t nx, ny, pitch, periodic_x;
  int32_t periodic_y, n_phases, has_source, has_region;
  int32_t node0, pairs;     // pairs: the paired population layout
  int64_t plane;            // elements between population planes
  void *pop;                // 14 planes of the storage type
  void *pop_b;              // second plane set of the two-step pass (or null)
  const uint8_t *link;      // link codes, plane layout
  const uint8_t *mask;      // mask values, plane layout
  const uint8_t *region;    // region flags, plane layout (or null)
  const double *R;          // source patch, row-major r_w x r_h
  int32_t r_x0, r_y0, r_w, r_h;
  int64_t *t;               // completed steps (device counter)
  double *flux;             // [GG_MAX_SEGMENTS][2] accumulated mass, solute
  double omega_f, omega_g;  // 1/tau_f, 1/tau_g
  double w0, wg_axis;       // compound weights: rest, each axis direction
  double inv_cs2g;          // 1/cs2 of the compound lattice
  double rho0;              // reference density (inlet/outlet links)
  double k_decay;
  double c_shift;           // C_s: the planes hold g_i - w_i C_s
  // the same constants rounded to FP32 once on the host, for the FP32
  // compute type (the kernels read them as they are)
  float rho0_f, omega_f_f, omega_g_f, wg_axis_f, inv_cs2g_f, k_decay_f, c_shift_f, kpad_f;
  // collision constants, FP64 and FP32 (make_collk)
  CollK<double> ck;
  CollK<float> ck_f;
  // segments, index id - GG_FIRST_SEGMENT
  int32_t seg_kind[GG_MAX_SEGMENTS];
  int32_t seg_nx[GG_MAX_SEGMENTS];
  int32_t seg_ny[GG_MAX_SEGMENTS];
  int32_t seg_pad;
  double seg_umax[GG_MAX_SEGMENTS];
  double seg_s0[GG_MAX_SEGMENTS];
  double seg_s1[GG_MAX_SEGMENTS];
  double seg_inv_w2[GG_MAX_SEGMENTS];
  // schedule: phase k starts at phase_start[k] within a period; the c_in
  // table already merges per-phase overrides with the segment defaults.
  int64_t period, t_origin;
  int64_t phase_start[GG_MAX_PHASES];
  uint32_t phase_open[GG_MAX_PHASES];
  double phase_cin[GG_MAX_PHASES][GG_MAX_SEGMENTS];
  double seg_cin[GG_MAX_SEGMENTS];  // used when there is no schedule
  // the same inlet parameters rounded to FP32 for the FP32 compute type:
  // 4 u_max, s0, s1, 1/(s1 - s0)^2 per segment, C_in per phase and segment
  float seg_umax4_f[GG_MAX_SEGMENTS];
  float seg_s0_f[GG_MAX_SEGMENTS];
  float seg_s1_f[GG_MAX_SEGMENTS];
  float seg_inv_w2_f[GG_MAX_SEGMENTS];
  float phase_cin_f[GG_MAX_PHASES][GG_MAX_SEGMENTS];
  float seg_cin_f[GG_MAX_SEGMENTS];
  // pressure segments: density held (and in FP32), compound held at C_in
  double seg_rho[GG_MAX_SEGMENTS];
  float seg_rho_f[GG_MAX_SEGMENTS];
  int32_t seg_holdc[GG_MAX_SEGMENTS];
  // frozen velocity fields of the compound-only step, in the compute type:
  // component c (0: u_x, 1: u_y) of slot k is the plane starting at element
  // (2 k + c) * plane of ufield; phase_field[k]: slot used in phase k
  void *ufield;
  int32_t n_ufield, ufield_pad;
  int8_t phase_field[GG_MAX_PHASES];
};

// Address spaces: the descriptor and tile lists are read-only while a
// kernel runs and are read through the constant space (scalar loads); the
// population planes live in the global space (global_load / global_store
// rather than flat accesses).
#define GG_GLOBAL __attribute__((address_space(1)))
#define GG_CONST __attribute__((address_space(4)))

template <class V> __device__ __forceinline__ V gload(const GG_GLOBAL V *p) { return *p; }
template <class V> __device__ __forceinline__ void gstore(GG_GLOBAL V *p, V v) { *p = v; }

// Storage traits: load into the compute type, store with rounding. W is the
// raw storage word that sits in the planes. Every storage type holds the
// deviations df_i = f_i - w_i rho0 and dg_i = g_i - w_i C_s (the rest state
// subtracted), and the step computes on the deviations directly, so the
// rounding of the stored and of the computed values is relative to the
// departure from rest rather than to w_i rho0.
template <class S> struct Pop;
template <> struct Pop<double> {
  using T = double;
  using W = double;
  static __device__ __forceinline__ T ld(const GG_GLOBAL W *p) { return gload(p); }
  static __device__ __forceinline__ void st(GG_GLOBAL W *p, T v) { gstore(p, v); }
  // two stores at once (one conversion for both where the storage is packed)
  static __device__ __forceinline__ void st2(GG_GLOBAL W *p, GG_GLOBAL W *q, T a, T b) {
    gstore(p, a);
    gstore(q, b);
  }
  // the value a store followed by a load gives back (of one, of two values)
  static __device__ __forceinline__ T rt(T v) { return v; }
  static __device__ __forceinline__ void rt2(T &, T &) {}
  // two adjacent elements (f_i, g_i of the paired layout) in one access
  using W2 = double __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ void ld_pair(const GG_GLOBAL W *p, T &a, T &b) {
    const W2 v = *(const GG_GLOBAL W2 *)p;
    a = v[0];
    b = v[1];
  }
  static __device__ __forceinline__ void st_pair(GG_GLOBAL W *p, T a, T b) {
    W2 v;
    v[0] = a;
    v[1] = b;
    *(GG_GLOBAL W2 *)p = v;
  }
};
template <> struct Pop<float> {
  using T = float;
  using W = float;
  static __device__ __forceinline__ T ld(const GG_GLOBAL W *p) { return gload(p); }
  static __device__ __forceinline__ void st(GG_GLOBAL W *p, T v) { gstore(p, v); }
  static __device__ __forceinline__ void st2(GG_GLOBAL W *p, GG_GLOBAL W *q, T a, T b) {
    gstore(p, a);
    gstore(q, b);
  }
  static __device__ __forceinline__ T rt(T v) { return v; }
  static __device__ __forceinline__ void rt2(T &, T &) {}
  using W2 = float __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ void ld_pair(const GG_GLOBAL W *p, T &a, T &b) {
    const W2 v = *(const GG_GLOBAL W2 *)p;
    a = v[0];
    b = v[1];
  }
  static __device__ __forceinline__ void st_pair(GG_GLOBAL W *p, T a, T b) {
    W2 v;
    v[0] = a;
    v[1] = b;
    *(GG_GLOBAL W2 *)p = v;
  }
};
template <> struct Pop<__half> {
  using T = float;
  using W = unsigned short;
  // FP32 result first, then round to nearest-even binary16. The empty asm
  // keeps the compiler from folding the conversion into the arithmetic that
  // produced v (a mixed-precision FMA with one rounding), which it would do
  // in some kernels and not in others.
  static __device__ __forceinline__ __half to_half(T v) {
    asm("" : "+v"(v));
    return __float2half_rn(v);
  }
  static __device__ __forceinline__ T ld(const GG_GLOBAL W *p) {
    return __half2float(__ushort_as_half(gload(p)));
  }
  static __device__ __forceinline__ void st(GG_GLOBAL W *p, T v) {
    gstore(p, __half_as_ushort(to_half(v)));
  }
  // the value a store followed by a load gives back
  static __device__ __forceinline__ T rt(T v) { return __half2float(to_half(v)); }
  // Two values rounded by one packed conversion (v_cvt_pk_f16_f32: round to
  // nearest even, as the single conversion). A packed conversion is never
  // folded into the arithmetic before it, so it needs no barrier.
  using H2 = _Float16 __attribute__((ext_vector_type(2)));
  using F2 = float __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ H2 to_half2(T a, T b) {
    F2 v;
    v[0] = a;
    v[1] = b;
    return __builtin_convertvector(v, H2);
  }
  static __device__ __forceinline__ void st2(GG_GLOBAL W *p, GG_GLOBAL W *q, T a, T b) {
    const H2 h = to_half2(a, b);
    const _Float16 h0 = h[0], h1 = h[1];
    gstore(p, __builtin_bit_cast(W, h0));
    gstore(q, __builtin_bit_cast(W, h1));
  }
  static __device__ __forceinline__ void rt2(T &a, T &b) {
    const H2 h = to_half2(a, b);
    a = (T)h[0];
    b = (T)h[1];
  }
  // two adjacent elements in one 32-bit access; the store rounds both with
  // one packed conversion, as st2
  static __device__ __forceinline__ void ld_pair(const GG_GLOBAL W *p, T &a, T &b) {
    const uint32_t v = gload((const GG_GLOBAL uint32_t *)p);
    a = __half2float(__ushort_as_half((unsigned short)(v & 0xffffu)));
    b = __half2float(__ushort_as_half((unsigned short)(v >> 16)));
  }
  static __device__ __forceinline__ void st_pair(GG_GLOBAL W *p, T a, T b) {
    gstore((GG_GLOBAL H2 *)p, to_half2(a, b));
  }
};

using CDesc = const GG_CONST LatDesc;

// The population planes of one plane set: uniform base pointers, elements
// reached through a 32-bit byte offset (a plane pair is smaller than
// 4 GiB), which maps onto the scalar-base + vector-offset form of global
// memory access. Two layouts:
//   plane-major: population i of node n at element i * plane + n;
//   paired: f_i and g_i (i = 0..4, the two populations that move along
//     the same velocity) side by side, at elements 2i * plane + 2n and
//     2i * plane + 2n + 1, and f5..f8 plane-major in planes 10..13,
//     so that a pass reads and writes (f_i, g_i) of a node with one access.
__host__ __device__ constexpr bool paired_slot(int i) { return i < 5 || i >= 9; }
template <class W> struct Planes {
  GG_GLOBAL W *p[NPOP];
  bool pairs;
  __device__ __forceinline__ Planes(CDesc &L) : Planes(L.pop, L.plane, L.pairs != 0) {}
  __device__ __forceinline__ Planes(void *pop, int64_t plane, bool paired) : pairs(paired) {
    GG_GLOBAL W *base = (GG_GLOBAL W *)pop;
    // (every pointer a select between two constants' products, so that the
    // array stays in scalar registers when the layout is a run-time value)
#pragma unroll
    for (int i = 0; i < NPOP; ++i) {
      const int k = i < 5 ? 2 * i : (i >= 9 ? 2 * (i - 9) : i + 5);
      p[i] = base + (int64_t)(paired ? k : i) * plane + (paired && i >= 9 ? 1 : 0);
    }
  }
  __device__ __forceinline__ GG_GLOBAL W *at(int i, uint32_t idx) const {
    const uint32_t stride = (pairs && paired_slot(i) ? 2u : 1u) * (uint32_t)sizeof(W);
    return (GG_GLOBAL W *)((GG_GLOBAL char *)p[i] + idx * stride);
  }
  // element idx + drow + dcol of plane i, with the uniform row offset drow
  // (a multiple of the pitch) added to the scalar base and the column offset
  // dcol (-1, 0 or 1) left constant, for the instruction's immediate offset
  __device__ __forceinline__ GG_GLOBAL W *at_nb(int i, uint32_t idx, int drow, int dcol) const {
    const int stride = (pairs && paired_slot(i) ? 2 : 1) * (int)sizeof(W);
    GG_GLOBAL char *row = (GG_GLOBAL char *)p[i] + (int64_t)drow * stride;
    return (GG_GLOBAL W *)(row + idx * (uint32_t)stride + dcol * stride);
  }
};

// Plane-major arrays of other per-node records (the adjoint's tapes).
template <class W> struct TapePlanes {
  GG_GLOBAL W *p[NPOP];
  __device__ __forceinline__ TapePlanes(void *base_, int64_t plane) {
    GG_GLOBAL W *base = (GG_GLOBAL W *)base_;
#pragma unroll
    for (int i = 0; i < NPOP; ++i) p[i] = base + (int64_t)i * plane;
  }
  __device__ __forceinline__ GG_GLOBAL W *at(int i, uint32_t idx) const {
    return (GG_GLOBAL W *)((GG_GLOBAL char *)p[i] + idx * (uint32_t)sizeof(W));
  }
};

}  // namespace gg
