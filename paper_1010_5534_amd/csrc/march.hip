// Ray march kernels for adaptive image ray-tracing on gfx950.
//
// A block of S waves traces a tile of 64 work-queue entries, one ray per
// lane (section 2 step ii): wave k walks the k-th of S equal parameter
// sub-intervals of every ray, and wave 0 folds the S partials in order.  In
// forest-Morton order a tile is a patch of neighbouring pixels, so at each
// step the 64 lanes read neighbouring cells.  Tiles are dealt to the XCDs in
// chunks (static split, or per-XCD tickets when a block has many); on the
// coarse levels, where a launch holds few tiles whose rays lie cells apart,
// each (tile, sub-interval) runs as its own wave job and a second launch
// folds the partials in the same order (split tiles).
//
// Along each ray the exact solution for cell-constant j, kappa, rho is
// accumulated front to back:
//   I_b += exp(-tau_b) j_b ds (1 - exp(-kappa_b ds)) / (kappa_b ds),
//   tau_b += kappa_b ds,  N += rho ds,
// in float32 with Kahan-compensated sums.  Ray-box entry, the sub-interval
// bounds and each axis's first crossing and spacing (relative to the
// sub-interval start) are formed in float64 and rounded once; the k-th
// crossing is rebuilt as fma(k, dt, t_first), so no rounding accumulates
// along the ray and every segment length is a difference of two freshly
// rounded values.
#include "air_common.h"

namespace air {

namespace {

constexpr float LOG2E_F = 1.4426950408889634f;
#ifndef AIR_KB
#define AIR_KB 4
#endif
constexpr int KB = AIR_KB;  // cells per load batch in the march

__device__ __forceinline__ void kadd(float& s, float& c, float x) {
#pragma clang fp contract(off)
  float y = x - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

// (1 - e^-x)/x for 0 <= x < 1/4 by its Taylor series (truncation < 2e-9
// relative); thicker cells use the transmission difference instead (see
// AIR_INTEGRATE)
constexpr float THICK = 0.25f;
__device__ __forceinline__ float seg_weight_series(float x) {
  const float y = -x;
  float p = 1.0f / 5040.0f;
  p = __builtin_fmaf(p, y, 1.0f / 720.0f);
  p = __builtin_fmaf(p, y, 1.0f / 120.0f);
  p = __builtin_fmaf(p, y, 1.0f / 24.0f);
  p = __builtin_fmaf(p, y, 1.0f / 6.0f);
  p = __builtin_fmaf(p, y, 0.5f);
  p = __builtin_fmaf(p, y, 1.0f);
  return p;
}

// field kinds of the march: the ABI's two, and (rho, T) with a band ladder
// (Fld::ladder: s_b = s0 + b ds, one q), whose optics share work across bands
constexpr int FK_LADDER = 2;

// raw cell data: (rho, j, kappa) or (rho, T)
template <int FK>
struct Raw {
  float rho, a, b, c;  // (rho, j, kappa, 1/kappa) or (rho, T, -, -)
};

// The packed field (air_field_pack): one 16-byte (rho, j, kappa, 1/kappa) record
// per cell (one-band (rho, T) fields get their j, kappa evaluated once when
// packing: three transcendentals fewer per visit) or 8-byte (rho, T) for
// several bands, in 2x2x2 bricks.  Loads go through a
// buffer resource: a 32-bit byte offset, and 0 past num_records, so an index
// can never leave the array.  The loads are bound to the LLVM buffer-load
// intrinsics directly (the vector-returning clang builtins shrink to one
// dword with this toolchain).
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ f32x4 buffer_load_f32x4(i32x4 rsrc, int voffset, int soffset, int aux) __asm("llvm.amdgcn.raw.buffer.load.v4f32");

__device__ f32x2 buffer_load_f32x2(i32x4 rsrc, int voffset, int soffset, int aux) __asm("llvm.amdgcn.raw.buffer.load.v2f32");

constexpr int RSRC_WORD3 = 0x00020000;  // raw 32-bit buffer on gfx9-class GPUs

__device__ __forceinline__ i32x4 field_rsrc(const Fld& f) {
  const uint64_t a = (uint64_t)f.packed;
  i32x4 r;
  r[0] = (int)(uint32_t)a;
  r[1] = (int)((uint32_t)(a >> 32) & 0xffffu);  // stride 0
  r[2] = (int)f.packed_bytes;                   // num_records in bytes
  r[3] = RSRC_WORD3;
  return r;
}

template <int FK>
__device__ __forceinline__ Raw<FK> load_raw(i32x4 R, int cell) {
  Raw<FK> r;
  if constexpr (FK == AIR_FIELD_RHO_J_KAPPA) {
    const f32x4 q = buffer_load_f32x4(R, (int)((unsigned)cell * 16u), 0, 0);
    r.rho = q[0];
    r.a = q[1];
    r.b = q[2];
    r.c = q[3];
  } else {
    const f32x2 q = buffer_load_f32x2(R, (int)((unsigned)cell * 8u), 0, 0);
    r.rho = q[0];
    r.a = q[1];
    r.b = 0.0f;
    r.c = 0.0f;
  }
  return r;
}

// emissivity and opacity of each band from the raw cell data
// (and 1/kappa: the packed one-band record carries it)
template <int NB, int FK>
__device__ __forceinline__ void optics(const Fld& f, const Raw<FK>& r, float* j, float* k, float* rk) {
  if constexpr (FK == AIR_FIELD_RHO_J_KAPPA) {
    j[0] = r.a;
    k[0] = r.b;
    rk[0] = r.c;
  } else {
    const float lt = __builtin_amdgcn_logf(r.a);  // log2 T
    const float r2 = r.rho * r.rho;
    if constexpr (FK == FK_LADDER) {
      const float jj = r2 * __builtin_amdgcn_exp2f(f.q0 * lt);
      const float base = r.rho * __builtin_amdgcn_exp2f(-f.s0 * lt);  // rho T^-s0
      const float step = __builtin_amdgcn_exp2f(-f.ds * lt);          // T^-ds
      const float rbase = __builtin_amdgcn_rcpf(base), rstep = __builtin_amdgcn_rcpf(step);
      float e = base, re = rbase;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        k[b] = f.k0[b] * e;
        rk[b] = f.rk0[b] * re;
        j[b] = jj;
        e *= step;
        re *= rstep;
      }
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        k[b] = f.k0[b] * r.rho * __builtin_amdgcn_exp2f(-f.s[b] * lt);
        j[b] = r2 * __builtin_amdgcn_exp2f(f.q[b] * lt);
        rk[b] = __builtin_amdgcn_rcpf(k[b]);
      }
    }
  }
}

// partial result of one sub-interval of a ray, optical depth counted from
// the sub-interval's start
template <int NB>
struct Seg {
  float I[NB], tau[NB];
  float N;
  float rmin, rmax;
  int nvis, lmax;  // block AMR: cells walked and finest level met
};

// entry / exit of the grid box, float64; false if the ray misses
__device__ __forceinline__ bool slab(const Geo& g, const double o[3], const double d[3],
                                     const double inv_d[3], double& t0, double& t1) {
  t0 = -__builtin_huge_val();
  t1 = __builtin_huge_val();
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0) {
      const double ta = (g.lo[a] - o[a]) * inv_d[a], tb = (g.hi[a] - o[a]) * inv_d[a];
      t0 = fmax(t0, fmin(ta, tb));
      t1 = fmin(t1, fmax(ta, tb));
    } else if (!(o[a] >= g.lo[a] && o[a] < g.hi[a])) {
      inside = false;
    }
  }
  return inside && t0 < t1;
}

// cell of axis a just after (after = true) or just before parameter t
__device__ __forceinline__ int cell_at(const Geo& g, const double o[3], const double d[3], int a, double t,
                                       bool after) {
  const double u = (o[a] + t * d[a] - g.lo[a]) * g.inv_h[a];
  int k;
  if (d[a] > 0.0)
    k = after ? (int)floor(u) : (int)ceil(u) - 1;
  else if (d[a] < 0.0)
    k = after ? (int)ceil(u) - 1 : (int)floor(u);
  else
    k = (int)floor(u);
  return min(max(k, 0), g.n[a] - 1);
}

// cells crossed between ta and tb (both inside the box)
__device__ __forceinline__ int cells_between(const Geo& g, const double o[3], const double d[3], double ta,
                                             double tb) {
  int n = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) n += abs(cell_at(g, o, d, a, tb, false) - cell_at(g, o, d, a, ta, true));
  return n;
}

// The cell walk shared by the uniform and block-AMR marches, written as
// macros over named arrays so that every index is static and the batches
// stay in registers.  They expect in scope: the walk state idx, cx, cy, cz,
// t0, t1, t2, k0, k1, k2, tc; the per-axis constants T00..T02, D0..D2,
// s0..s2, the clamp bounds nx, ny, nz, the end S1 and cell count nvis; the
// accumulators I, cI, tau, ctau, N, cN, rmin, rmax; the resource R, the
// field f; and AIR_CELL_INDEX() giving the packed record of (cx, cy, cz).
// AIR_DDA_BATCH takes one DDA step per cell of a batch of KB (the cell's
// record offset and segment length; past the last cell ds = 0 and the cell
// repeats), then issues the batch's loads.
#define AIR_DDA_BATCH(V0, OFF, DS, RAW)                                   \
  _Pragma("unroll") for (int q = 0; q < KB; ++q) {                        \
    OFF[q] = idx;                                                         \
    const bool last = (V0) + q >= nvis - 1;                               \
    const float tm = fminf(fminf(t0, t1), t2);                            \
    const float tn = last ? S1 : tm;                                      \
    const bool a0 = !last && tm == t0;                                    \
    const bool a1 = !last && !a0 && tm == t1;                             \
    const bool a2 = !last && !a0 && !a1;                                  \
    DS[q] = tn - tc;                                                      \
    tc = tn;                                                              \
    if constexpr (BF) { /* the three axis updates computed and selected */ \
      k0 += a0 ? 1.0f : 0.0f;                                             \
      k1 += a1 ? 1.0f : 0.0f;                                             \
      k2 += a2 ? 1.0f : 0.0f;                                             \
      t0 = a0 ? __builtin_fmaf(k0, D0, T00) : t0;                         \
      t1 = a1 ? __builtin_fmaf(k1, D1, T01) : t1;                         \
      t2 = a2 ? __builtin_fmaf(k2, D2, T02) : t2;                         \
      cx = a0 ? min(max(cx + s0, 0), nx - 1) : cx;                        \
      cy = a1 ? min(max(cy + s1, 0), ny - 1) : cy;                        \
      cz = a2 ? min(max(cz + s2, 0), nz - 1) : cz;                        \
    } else if (a0) { /* one update, a uniform branch for coherent rays */ \
      k0 += 1.0f;                                                         \
      t0 = __builtin_fmaf(k0, D0, T00);                                   \
      cx = min(max(cx + s0, 0), nx - 1);                                  \
    } else if (a1) {                                                      \
      k1 += 1.0f;                                                         \
      t1 = __builtin_fmaf(k1, D1, T01);                                   \
      cy = min(max(cy + s1, 0), ny - 1);                                  \
    } else if (a2) {                                                      \
      k2 += 1.0f;                                                         \
      t2 = __builtin_fmaf(k2, D2, T02);                                   \
      cz = min(max(cz + s2, 0), nz - 1);                                  \
    }                                                                     \
    idx = AIR_CELL_INDEX();                                              \
  }                                                                       \
  _Pragma("unroll") for (int q = 0; q < KB; ++q) RAW[q] = load_raw<FK>(R, OFF[q]); \
  /* the batch's loads go out before the older batch is integrated */     \
  __builtin_amdgcn_sched_barrier(0);

// One batch of up to KB cells: plain float32 sums inside the batch (at most
// KB terms), one Kahan step per batch into the running I, tau, N.  Each
// cell's exit transmission Ta = exp(-tau) comes from the compensated optical
// depth at the batch start plus the batch's partial sum and is the next
// cell's entry transmission Tb, so a cell costs one exp.  A cell adds
// Tb j ds (1 - e^-x)/x, x = kappa ds: by the series for x < 1/4, else as
// (Tb - Ta) j / kappa (cancellation at most a factor 4.5 there).
#define AIR_INTEGRATE(V0, DS, RAW)                                        \
  {                                                                       \
    float bI[NB], bT[NB], t0b[NB], Tb[NB], bN = 0.0f;                     \
    _Pragma("unroll") for (int b = 0; b < NB; ++b) {                      \
      bI[b] = 0.0f;                                                       \
      bT[b] = 0.0f;                                                       \
      t0b[b] = tau[b] - ctau[b];                                          \
      Tb[b] = __builtin_amdgcn_exp2f(-t0b[b] * LOG2E_F);                  \
    }                                                                     \
    /* past the last cell ds = 0 (the walk repeats that cell), so a cell  \
       there adds exact zeros: the branch-free walk integrates it */      \
    _Pragma("unroll") for (int q = 0; q < KB; ++q) {                      \
      if (!BF && (V0) + q >= nvis) continue;                              \
      const float ds = DS[q];                                             \
      float jb[NB], kb[NB], rkb[NB];                                      \
      optics<NB, FK>(f, RAW[q], jb, kb, rkb);                             \
      _Pragma("unroll") for (int b = 0; b < NB; ++b) {                    \
        const float dtau = kb[b] * ds;                                    \
        bT[b] += dtau;                                                    \
        const float Ta = __builtin_amdgcn_exp2f(-(t0b[b] + bT[b]) * LOG2E_F); \
        const float thin = Tb[b] * (jb[b] * ds) * seg_weight_series(dtau); \
        const float thick = (Tb[b] - Ta) * jb[b] * rkb[b];               \
        bI[b] += dtau < THICK ? thin : thick;                             \
        Tb[b] = Ta;                                                       \
      }                                                                   \
      bN += RAW[q].rho * ds;                                              \
      if constexpr (RANGE) {                                              \
        const bool in = (V0) + q < nvis;                                  \
        rmin = in ? fminf(rmin, RAW[q].rho) : rmin;                       \
        rmax = in ? fmaxf(rmax, RAW[q].rho) : rmax;                       \
      }                                                                   \
    }                                                                     \
    _Pragma("unroll") for (int b = 0; b < NB; ++b) {                      \
      kadd(I[b], cI[b], bI[b]);                                           \
      kadd(tau[b], ctau[b], bT[b]);                                       \
    }                                                                     \
    kadd(N, cN, bN);                                                      \
  }

// the whole cell walk, two batches in flight: walk and load batch n+1, then
// integrate batch n.  The next batch is issued unconditionally (past the
// last cell the walk stays on it), so every iteration has the same loads in
// flight and the waits count only the older batch.
#define AIR_MARCH_CELLS_WITH(DDA)                                         \
  {                                                                       \
    int offA[KB], offB[KB];                                               \
    float dsA[KB], dsB[KB];                                               \
    Raw<FK> rawA[KB], rawB[KB];                                           \
    DDA(0, offA, dsA, rawA)                                               \
    for (int v0 = 0;;) {                                                  \
      DDA(v0 + KB, offB, dsB, rawB)                                       \
      AIR_INTEGRATE(v0, dsA, rawA)                                        \
      v0 += KB;                                                           \
      if (v0 >= nvis) break;                                              \
      DDA(v0 + KB, offA, dsA, rawA)                                       \
      AIR_INTEGRATE(v0, dsB, rawB)                                        \
      v0 += KB;                                                           \
      if (v0 >= nvis) break;                                              \
      DDA(v0 + KB, offB, dsB, rawB)                                       \
      AIR_INTEGRATE(v0, dsA, rawA)                                        \
      v0 += KB;                                                           \
      if (v0 >= nvis) break;                                              \
      DDA(v0 + KB, offA, dsA, rawA)                                       \
      AIR_INTEGRATE(v0, dsB, rawB)                                        \
      v0 += KB;                                                           \
      if (v0 >= nvis) break;                                              \
    }                                                                     \
  }
#define AIR_MARCH_CELLS() AIR_MARCH_CELLS_WITH(AIR_DDA_BATCH)

// The walk of a ray that moves along one axis only (the other two direction
// components zero, the axis the same for the whole wave): the general walk's
// minimum of the three crossings is then always this axis's, so the same
// crossings, lengths and cells come from one axis update per step, with the
// record index updated along that axis (bitwise the same values).  Expects
// in scope tA, kA, DA, TA0 (the axis's crossing state and constants), cA, sA,
// nA (its cell, step and clamp bound), ibase, istr, ibit (the record index
// without this axis's part, the brick stride and bit position along it) and
// the general walk's idx, tc, S1, nvis.
#define AIR_DDA_BATCH1(V0, OFF, DS, RAW)                                  \
  _Pragma("unroll") for (int q = 0; q < KB; ++q) {                        \
    OFF[q] = idx;                                                         \
    const bool last = (V0) + q >= nvis - 1;                               \
    const float tn = last ? S1 : tA;                                      \
    DS[q] = tn - tc;                                                      \
    tc = tn;                                                              \
    if (!last) {                                                          \
      kA += 1.0f;                                                         \
      tA = __builtin_fmaf(kA, DA, TA0);                                   \
      cA = min(max(cA + sA, 0), nA - 1);                                  \
      idx = ibase + (cA >> 1) * istr + ((cA & 1) << ibit);                \
    }                                                                     \
  }                                                                       \
  _Pragma("unroll") for (int q = 0; q < KB; ++q) RAW[q] = load_raw<FK>(R, OFF[q]); \
  __builtin_amdgcn_sched_barrier(0);

// March the sub-interval [ta, tb] of the ray x(t) = o + t d (d unit) through
// the uniform grid: DDA from the cell just after ta to the cell just before
// tb, optical depth from 0 at ta.  Crossing parameters are measured from ta
// (a sub-interval is at most ~1/S of the chord, ~32 cells): the first
// crossing of each axis and the per-axis spacing come from float64, and the
// k-th crossing is the single-rounding t_a(k) = fma(k, dt_a, t_a(0)), so no
// rounding accumulates and each segment length is a difference of two
// freshly rounded values.
// BF: branch-free cell walk (rays of a wave step different axes: coarse
// levels) or one uniform branch per step (coherent rays); same arithmetic
template <int NB, int FK, bool RANGE, bool BF, bool AX1 = true>
__device__ void march_interval(const Geo& g, const Fld& f, const double o[3], const double d[3],
                               const double inv_d[3], double ta, double tb, Seg<NB>& r) {
  int c[3], st[3], nvis = 1;
  float T0[3], D[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int k0 = cell_at(g, o, d, a, ta, true), k1 = cell_at(g, o, d, a, tb, false);
    c[a] = k0;
    nvis += abs(k1 - k0);
    if (d[a] != 0.0) {
      const int m = d[a] > 0.0 ? k0 + 1 : k0;
      T0[a] = (float)((g.lo[a] + (double)m * g.h[a] - o[a]) * inv_d[a] - ta);
      D[a] = (float)(g.h[a] * fabs(inv_d[a]));
      st[a] = d[a] > 0.0 ? 1 : -1;
    } else {
      T0[a] = __builtin_huge_valf();
      D[a] = 0.0f;
      st[a] = 0;
    }
  }
  const float S1 = (float)(tb - ta);
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const i32x4 R = field_rsrc(f);
  const int bnx = f.bnx, bny = f.bny;

  float I[NB], cI[NB], tau[NB], ctau[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) I[b] = cI[b] = tau[b] = ctau[b] = 0.0f;
  float N = 0.0f, cN = 0.0f;
  float rmin = __builtin_huge_valf(), rmax = -__builtin_huge_valf();

  int cx = c[0], cy = c[1], cz = c[2];
  const int s0 = st[0], s1 = st[1], s2 = st[2];
  const float T00 = T0[0], T01 = T0[1], T02 = T0[2], D0 = D[0], D1 = D[1], D2 = D[2];
  float k0 = 0.0f, k1 = 0.0f, k2 = 0.0f;  // crossings done per axis (exact small integers)
  float t0 = T00, t1 = T01, t2 = T02;
  float tc = 0.0f;
#define AIR_CELL_INDEX() brick_index(cx, cy, cz, bnx, bny)
  int idx = AIR_CELL_INDEX();
  // rays along one axis, the same for every lane of the wave: one axis update per step
  const int nz_axes = (d[0] != 0.0) + (d[1] != 0.0) + (d[2] != 0.0);
  const int ax = d[0] != 0.0 ? 0 : (d[1] != 0.0 ? 1 : 2);
  const int ax0 = __builtin_amdgcn_readfirstlane(ax);
  if (AX1 && __all(nz_axes == 1 && ax == ax0)) {
    float tA, DA, TA0, kA = 0.0f;
    int cA, sA, nA, istr;
    if (ax0 == 0) {
      tA = t0, DA = D0, TA0 = T00, cA = cx, sA = s0, nA = nx, istr = 8;
    } else if (ax0 == 1) {
      tA = t1, DA = D1, TA0 = T01, cA = cy, sA = s1, nA = ny, istr = 8 * bnx;
    } else {
      tA = t2, DA = D2, TA0 = T02, cA = cz, sA = s2, nA = nz, istr = 8 * bnx * bny;
    }
    const int ibit = ax0;
    const int ibase = idx - ((cA >> 1) * istr + ((cA & 1) << ibit));
    AIR_MARCH_CELLS_WITH(AIR_DDA_BATCH1)
  } else {
    AIR_MARCH_CELLS()
  }
#undef AIR_CELL_INDEX
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    r.I[b] = I[b] - cI[b];
    r.tau[b] = tau[b] - ctau[b];
  }
  r.N = N - cN;
  r.rmin = rmin;
  r.rmax = rmax;
}


// finest-level cell of axis a just after (after = true) or just before t
__device__ __forceinline__ int fine_at(const Geo& g, const double o[3], const double d[3], int a, double t,
                                       bool after) {
  const double u = (o[a] + t * d[a] - g.lo[a]) * g.inv_hf[a];
  int k;
  if (d[a] > 0.0)
    k = after ? (int)floor(u) : (int)ceil(u) - 1;
  else if (d[a] < 0.0)
    k = after ? (int)ceil(u) - 1 : (int)floor(u);
  else
    k = (int)floor(u);
  return min(max(k, 0), g.nf[a] - 1);
}

// Leaf block of finest-level block position (fx, fy, fz) and its level:
// descent through the child table from the base block.  A child's
// coordinate is twice its parent's plus its offset bit (the tables were
// checked for it), so the offset at level l is the low bit of the
// position's level-l block coordinate and no coordinate has to be read.
__device__ __forceinline__ int leaf_of(const Geo& g, int fx, int fy, int fz, int& l) {
  const int mL = g.max_level;
  int b = ((fz >> mL) * g.n[1] + (fy >> mL)) * g.n[0] + (fx >> mL);
  l = 0;
  for (int ch = g.bchild[b]; ch >= 0 && l < mL; ch = g.bchild[b]) {
    ++l;
    const int off = ((fx >> (mL - l)) & 1) | (((fy >> (mL - l)) & 1) << 1) | (((fz >> (mL - l)) & 1) << 2);
    b = min(ch + off, g.n_blocks - 1);  // the host checked the tables; this only bounds the reads
  }
  return b;
}

// March [ta, tb] through a block-AMR grid: locate the leaf block just after
// the current parameter (integer fine coordinates, descent through the child
// table), walk its cells at its level's spacing up to the block exit, and
// continue from there.  Crossing parameters restart at every block entry.
// At most g.max_blocks blocks are visited, so every lane terminates; the
// block after an exit is the one across the face the ray leaves by (also
// for a block entered, by rounding, at or past its exit).
template <int NB, int FK, bool RANGE, bool BF>
__device__ void march_amr_interval(const Geo& g, const Fld& f, const double o[3], const double d[3],
                                   const double inv_d[3], double ta, double tb, Seg<NB>& r) {
  const i32x4 R = field_rsrc(f);
  const int bs = g.bs, lbs = g.bs_shift, mL = g.max_level, hb = bs >> 1;
  const int nx = bs, ny = bs, nz = bs;
  float I[NB], cI[NB], tau[NB], ctau[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) I[b] = cI[b] = tau[b] = ctau[b] = 0.0f;
  float N = 0.0f, cN = 0.0f;
  float rmin = __builtin_huge_valf(), rmax = -__builtin_huge_valf();
  int nvis_total = 0, lmax = -1;
  double t = ta;
  int F[3];  // finest-lattice cell of the point just after t
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] = fine_at(g, o, d, a, t, true);
  for (int it = 0; it < g.max_blocks && t < tb; ++it) {
    int b, l;
    if (f.leaf_map) {  // the leaf of the point's finest-level block position
      const uint32_t* lm = reinterpret_cast<const uint32_t*>(static_cast<const char*>(f.packed) + f.leaf_off);
      const int nfx = g.n[0] << mL, nfy = g.n[1] << mL;
      const uint32_t m = lm[((int64_t)(F[2] >> lbs) * nfy + (F[1] >> lbs)) * nfx + (F[0] >> lbs)];
      b = (int)(m >> 4);
      l = (int)(m & 15u);
    } else {
      b = leaf_of(g, F[0] >> lbs, F[1] >> lbs, F[2] >> lbs, l);
    }
    int bc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) bc[a] = (F[a] >> (mL - l)) >> lbs;
    const double scale = 1.0 / (double)(1 << l);
    double t_exit = __builtin_huge_val(), te[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double hl = g.h[a] * scale;
      te[a] = __builtin_huge_val();
      if (d[a] > 0.0)
        te[a] = (g.lo[a] + (double)((bc[a] + 1) * bs) * hl - o[a]) * inv_d[a];
      else if (d[a] < 0.0)
        te[a] = (g.lo[a] + (double)(bc[a] * bs) * hl - o[a]) * inv_d[a];
      t_exit = fmin(t_exit, te[a]);
    }
    const double t_end = fmin(t_exit, tb);
    // the next block's cell: across each face the ray leaves by, the first
    // cell past the face (not the rounded position at the exit, which can
    // fall back into this block, and for a ray that nearly grazes the face
    // would take many one-ulp retries); along the other axes the cell at the
    // exit.  A block entered at (by rounding, past) its exit is left at once
    // across the faces already passed.
    const bool passed = !(t_end > t);
    int Fn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (te[a] <= t_end)  // finite: d[a] != 0 and the ray leaves by this face at t_end
        Fn[a] = d[a] > 0.0 ? ((bc[a] + 1) * bs) << (mL - l) : ((bc[a] * bs) << (mL - l)) - 1;
      else
        Fn[a] = passed ? F[a] : fine_at(g, o, d, a, t_end, true);
      Fn[a] = min(max(Fn[a], 0), g.nf[a] - 1);
    }
    if (passed) {
#pragma unroll
      for (int a = 0; a < 3; ++a) F[a] = Fn[a];
      continue;
    }
    // cells of the block between t and t_end, and the DDA constants
    int c[3], st[3], nvis = 1;
    float T0[3], D[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int k0 = min(max((F[a] >> (mL - l)) - bs * bc[a], 0), bs - 1);
      const int k1 = min(max((fine_at(g, o, d, a, t_end, false) >> (mL - l)) - bs * bc[a], 0), bs - 1);
      c[a] = k0;
      nvis += abs(k1 - k0);
      const double hl = g.h[a] * scale;
      if (d[a] != 0.0) {
        const int m = bs * bc[a] + k0 + (d[a] > 0.0 ? 1 : 0);
        T0[a] = (float)((g.lo[a] + (double)m * hl - o[a]) * inv_d[a] - t);
        D[a] = (float)(hl * fabs(inv_d[a]));
        st[a] = d[a] > 0.0 ? 1 : -1;
      } else {
        T0[a] = __builtin_huge_valf();
        D[a] = 0.0f;
        st[a] = 0;
      }
    }
    const float S1 = (float)(t_end - t);
    int cx = c[0], cy = c[1], cz = c[2];
    const int s0 = st[0], s1 = st[1], s2 = st[2];
    const float T00 = T0[0], T01 = T0[1], T02 = T0[2], D0 = D[0], D1 = D[1], D2 = D[2];
    float k0 = 0.0f, k1 = 0.0f, k2 = 0.0f;
    float t0 = T00, t1 = T01, t2 = T02;
    float tc = 0.0f;
    const int bbase = b * (bs * bs * bs);
#define AIR_CELL_INDEX() (bbase + brick_index(cx, cy, cz, hb, hb))
    int idx = AIR_CELL_INDEX();
    AIR_MARCH_CELLS()
#undef AIR_CELL_INDEX
    nvis_total += nvis;
    lmax = max(lmax, l);
    t = t_end;
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = Fn[a];
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    r.I[b] = I[b] - cI[b];
    r.tau[b] = tau[b] - ctau[b];
  }
  r.N = N - cN;
  r.rmin = rmin;
  r.rmax = rmax;
  r.nvis = nvis_total;
  r.lmax = lmax;
}

__device__ __forceinline__ void pixel_ray(const DevView& V, int N0, int L, uint32_t i, uint32_t j,
                                          double o[3]) {
  const double s = V.width / (double)((int64_t)N0 << L);
  const double au = -0.5 * V.width + ((double)i + 0.5) * s;
  const double av = -0.5 * V.width + ((double)j + 0.5) * s;
#pragma unroll
  for (int a = 0; a < 3; ++a) o[a] = V.c[a] + au * V.eu[a] + av * V.ev[a];
}

template <int NB>
struct RayRes {
  float I[NB];
  float N;
  int nvis;
  int lmax;  // finest grid level crossed, -1 for a miss
  bool hit;
  float rmin, rmax;
};

// LDS staging of the per-segment partials of one 64-ray tile:
// [segment][field][lane], fields I[NB], tau[NB], N, rmin, rmax
template <int NB>
struct TileLds {
  float v[MAX_SEG][2 * NB + 3][WAVE];
  int cnt[MAX_SEG][2][WAVE];  // cells walked, finest level (block AMR)
  int nvis[WAVE];
  int hit[WAVE];
};

// Sub-interval k of the S = 2^sh equal parameter sub-intervals of the chord
// of pixel (i, j)'s ray at level L (S a power of two: k/S is exact, so the
// split depends only on the ray and S, fixed per grid).  Returns whether the
// ray meets the grid; nvis = its uniform-grid cell count when k == 0.
template <int NB, int FK, int GK, bool RANGE, bool BF, bool AX1 = true>
__device__ __forceinline__ bool march_lane(const MarchArgs& A, bool live, uint32_t v, int L, uint32_t i, uint32_t j,
                                           int k, int sh, Seg<NB>& sg, int& nvis) {
  const int S = 1 << sh;
#pragma unroll
  for (int b = 0; b < NB; ++b) sg.I[b] = sg.tau[b] = 0.0f;
  sg.N = 0.0f;
  sg.rmin = __builtin_huge_valf();
  sg.rmax = -__builtin_huge_valf();
  sg.nvis = 0;
  sg.lmax = -1;
  bool hit = false;
  nvis = 0;
  if (live) {
    const DevView& V = A.views[v];
    double o[3], t0, t1;
    pixel_ray(V, A.img.N0, L, i, j, o);
    hit = slab(A.g, o, V.d, V.inv_d, t0, t1);
    if (hit) {
      if (GK == AIR_GRID_UNIFORM && k == 0) nvis = cells_between(A.g, o, V.d, t0, t1);  // frees t0, t1 early
      const double len = t1 - t0, inv_s = 1.0 / (double)S;
      const double ta = k == 0 ? t0 : t0 + len * ((double)k * inv_s);
      const double tb = k == S - 1 ? t1 : t0 + len * ((double)(k + 1) * inv_s);
      if constexpr (GK == AIR_GRID_UNIFORM)
        march_interval<NB, FK, RANGE, BF, AX1>(A.g, A.f, o, V.d, V.inv_d, ta, tb, sg);
      else
        march_amr_interval<NB, FK, RANGE, BF>(A.g, A.f, o, V.d, V.inv_d, ta, tb, sg);
    }
  }
  return hit;
}

// A block of S = 2^sh waves traces a tile of 64 rays (one per lane): wave
// k marches the k-th of S equal parameter sub-intervals of every ray's
// chord, so at each step the 64 lanes of a wave read the cells of 64
// neighbouring rays at a similar depth.  The partials meet in LDS and wave 0
// folds them in order,
//   I = sum_k exp(-tau_0 - ... - tau_{k-1}) I_k,
// which is exact for piecewise-constant cells; a ray's result does not
// depend on which block or kernel traced it.  Every thread of the block
// calls this; the result is valid in wave 0.
template <int NB, int FK, int GK, bool RANGE, bool BF, bool AX1 = true>
__device__ __forceinline__ void trace_tile(const MarchArgs& A, TileLds<NB>& T, bool live, uint32_t v, int L,
                                           uint32_t i, uint32_t j, int sh, RayRes<NB>& r) {
  const int S = 1 << sh, lane = threadIdx.x & (WAVE - 1), k = threadIdx.x / WAVE;
  Seg<NB> sg;
  int nvis;
  const bool hit = march_lane<NB, FK, GK, RANGE, BF, AX1>(A, live, v, L, i, j, k, sh, sg, nvis);
  __syncthreads();  // the previous tile's fold has read the staging area
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    T.v[k][b][lane] = sg.I[b];
    T.v[k][NB + b][lane] = sg.tau[b];
  }
  T.v[k][2 * NB][lane] = sg.N;
  if constexpr (RANGE) {
    T.v[k][2 * NB + 1][lane] = sg.rmin;
    T.v[k][2 * NB + 2][lane] = sg.rmax;
  }
  if constexpr (GK == AIR_GRID_BLOCK_AMR) {
    T.cnt[k][0][lane] = sg.nvis;
    T.cnt[k][1][lane] = sg.lmax;
  }
  if (k == 0) {
    T.nvis[lane] = nvis;
    T.hit[lane] = hit;
  }
  __syncthreads();
  if (k != 0) return;
  float accI[NB], accT[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    accI[b] = T.v[0][b][lane];
    accT[b] = T.v[0][NB + b][lane];
  }
  float accN = T.v[0][2 * NB][lane];
  float mn = sg.rmin, mx = sg.rmax;
  int cells = sg.nvis, lm = sg.lmax;
  for (int q = 1; q < S; ++q) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      accI[b] += __builtin_amdgcn_exp2f(-accT[b] * LOG2E_F) * T.v[q][b][lane];
      accT[b] += T.v[q][NB + b][lane];
    }
    accN += T.v[q][2 * NB][lane];
    if constexpr (RANGE) {
      mn = fminf(mn, T.v[q][2 * NB + 1][lane]);
      mx = fmaxf(mx, T.v[q][2 * NB + 2][lane]);
    }
    if constexpr (GK == AIR_GRID_BLOCK_AMR) {
      cells += T.cnt[q][0][lane];
      lm = max(lm, T.cnt[q][1][lane]);
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) r.I[b] = accI[b];
  r.N = accN;
  r.hit = T.hit[lane] != 0;
  if constexpr (GK == AIR_GRID_BLOCK_AMR) {
    // a cell cut by a sub-interval boundary counts once per part
    r.nvis = cells;
    r.lmax = r.hit ? lm : -1;
  } else {
    r.nvis = T.nvis[lane];
    r.lmax = r.hit ? 0 : -1;
  }
  if constexpr (RANGE) {
    r.rmin = r.hit ? mn : 0.0f;
    r.rmax = r.hit ? mx : 0.0f;
  }
}

// Static, XCD-aware split of n tiles over the blocks of the grid.  Blocks
// are dispatched round-robin over the 8 XCDs (block b on XCD b % 8); tiles
// are dealt to the XCDs in chunks of TCHUNK consecutive tiles (neighbouring
// pixels, whose rays read neighbouring cells, then share an L2), and each
// XCD's blocks stride over its chunks.  No work counter: same-address
// atomics from thousands of waves serialise.  The grid is a multiple of 8.
constexpr long long TCHUNK = 4;
struct Split {
  long long k, step, n, x;
  __device__ long long tile() const {  // k-th item of XCD x
    return ((k / TCHUNK) * 8 + x) * TCHUNK + (k % TCHUNK);
  }
  __device__ bool ok() const { return tile() < n; }
};
__device__ __forceinline__ Split xcd_split(long long n) {
  Split sp;
  sp.x = blockIdx.x & 7;
  sp.k = blockIdx.x >> 3;
  sp.step = gridDim.x >> 3;
  sp.n = n;
  return sp;
}
// number of items of XCD x (upper bound on k), uniform per block
__device__ __forceinline__ long long xcd_items(long long n) { return (n + 7) / 8 + TCHUNK; }

// add the block's hit and visit counts (held by wave 0) into a spread slot
__device__ __forceinline__ void block_stats(unsigned long long* ctr, unsigned long long hit,
                                            unsigned long long vis) {
  if (threadIdx.x >= WAVE) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    hit += __shfl_xor(hit, o);
    vis += __shfl_xor(vis, o);
  }
  if (threadIdx.x == 0) {
    const int slot = blockIdx.x & (CTR_SLOTS - 1);
    if (hit) atomicAdd(&ctr[CTR_HITS + slot], hit);
    if (vis) atomicAdd(&ctr[CTR_VISITS + slot], vis);
  }
}

// add one wave's hit and visit counts into a spread slot
__device__ __forceinline__ void wave_stats(unsigned long long* ctr, unsigned long long hit, unsigned long long vis) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    hit += __shfl_xor(hit, o);
    vis += __shfl_xor(vis, o);
  }
  if ((threadIdx.x & (WAVE - 1)) == 0) {
    const int slot = (blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE) & (CTR_SLOTS - 1);
    if (hit) atomicAdd(&ctr[CTR_HITS + slot], hit);
    if (vis) atomicAdd(&ctr[CTR_VISITS + slot], vis);
  }
}

// ------------------------------------------------------------ kernels
// packing modes: copy (rho, j, kappa); evaluate one band's (j, kappa) from
// (rho, T) with the march's own optics; copy (rho, T).  One-band records
// carry 1/kappa (v_rcp_f32, as the march would take it) in their fourth word
enum { PACK_RJK = 0, PACK_RT_TO_RJK = 1, PACK_RT = 2 };

template <int PM>
__device__ __forceinline__ void pack_cell(const Fld& f, int64_t src, bool in, int64_t dst) {
  if constexpr (PM == PACK_RT) {
    const float2 v = in ? make_float2(f.rho[src], f.temp[src]) : make_float2(0.f, 0.f);
    reinterpret_cast<float2*>(const_cast<void*>(f.packed))[dst] = v;
  } else {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (in) {
      if constexpr (PM == PACK_RJK) {
        const float kap = f.kappa[src];
        v = make_float4(f.rho[src], f.emis[src], kap, __builtin_amdgcn_rcpf(kap));
      } else {
        Raw<AIR_FIELD_RHO_T> r;
        r.rho = f.rho[src];
        r.a = f.temp[src];
        r.b = r.c = 0.0f;
        float j[1], k[1], rk[1];
        optics<1, AIR_FIELD_RHO_T>(f, r, j, k, rk);
        v = make_float4(r.rho, j[0], k[0], rk[0]);
      }
    }
    reinterpret_cast<float4*>(const_cast<void*>(f.packed))[dst] = v;
    if (PM == PACK_RT_TO_RJK && f.rt_bytes) {  // the (rho, T) copy
      char* rt = static_cast<char*>(const_cast<void*>(f.packed)) + f.rt_off;
      reinterpret_cast<float2*>(rt)[dst] = in ? make_float2(f.rho[src], f.temp[src]) : make_float2(0.f, 0.f);
    }
  }
}

// packed layout, written slot by slot (padding cells of odd sizes get 0)
template <int PM>
__global__ __launch_bounds__(256) void k_pack(Geo g, Fld f) {
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int64_t slots = 8ll * f.bnx * f.bny * f.bnz;
  for (int64_t sl = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; sl < slots; sl += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = sl >> 3;
    const int x = (int)(2 * (b % f.bnx)) + (int)(sl & 1);
    const int y = (int)(2 * ((b / f.bnx) % f.bny)) + (int)((sl >> 1) & 1);
    const int z = (int)(2 * (b / ((int64_t)f.bnx * f.bny))) + (int)((sl >> 2) & 1);
    const bool in = x < nx && y < ny && z < nz;
    const int64_t src = in ? x + (int64_t)nx * (y + (int64_t)ny * z) : 0;
    pack_cell<PM>(f, src, in, sl);
  }
}

// block-AMR packed layout: inside each block of bs^3 cells, 2x2x2 bricks
template <int PM>
__global__ __launch_bounds__(256) void k_pack_amr(Geo g, Fld f) {
  const int bs = g.bs, hb = bs >> 1;
  const int64_t cells = (int64_t)g.n_blocks * bs * bs * bs;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < cells; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = q / ((int64_t)bs * bs * bs);
    const int loc = (int)(q - b * bs * bs * bs);
    const int x = loc % bs, y = (loc / bs) % bs, z = loc / (bs * bs);
    pack_cell<PM>(f, q, true, b * bs * bs * bs + brick_index(x, y, z, hb, hb));
  }
}

// the leaf map of a packed block-AMR field: one entry per finest-level block
// position, x fastest
__global__ __launch_bounds__(256) void k_leaf_map(Geo g, Fld f) {
  const int mL = g.max_level, nfx = g.n[0] << mL, nfy = g.n[1] << mL, nfz = g.n[2] << mL;
  uint32_t* lm = reinterpret_cast<uint32_t*>(static_cast<char*>(const_cast<void*>(f.packed)) + f.leaf_off);
  const int64_t total = (int64_t)nfx * nfy * nfz;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int fx = (int)(q % nfx), fy = (int)((q / nfx) % nfy), fz = (int)(q / ((int64_t)nfx * nfy));
    int l;
    const int b = leaf_of(g, fx, fy, fz, l);
    lm[q] = ((uint32_t)b << 4) | (uint32_t)l;
  }
}

// zero the state maps (grid.y = view) with the base image marked existing and
// tested, seed the queue with the base pixels, clear the counters
__global__ void k_init(MarchArgs A) {
  const int64_t S = A.img.S, n0sq = (int64_t)A.img.N0 * A.img.N0;
  const int v = blockIdx.y;
  // S is a multiple of CHUNK bytes: 16-byte stores
  uint4* st = reinterpret_cast<uint4*>(A.w.state + (int64_t)v * S);
  const uint32_t base_bits = AIR_NODE_EXIST | AIR_NODE_TESTED;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < S / 16; w += (int64_t)gridDim.x * blockDim.x) {
    uint32_t word[4] = {0u, 0u, 0u, 0u};
    if (16 * w < n0sq) {  // level 0 occupies [0, N0^2) of the view
#pragma unroll
      for (int b = 0; b < 16; ++b)
        if (16 * w + b < n0sq) word[b >> 2] |= base_bits << (8 * (b & 3));
    }
    st[w] = uint4{word[0], word[1], word[2], word[3]};
  }
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n0sq; e += (int64_t)gridDim.x * blockDim.x)
    A.w.queue[(int64_t)v * n0sq + e] = qentry((uint32_t)v, 0, (uint32_t)e);
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int k = threadIdx.x; k < CTR_COUNT; k += blockDim.x)
      A.w.ctr[k] = k == CTR_CURSOR ? (unsigned long long)(A.img.V * n0sq) : 0ull;
}

// Queue march of level L: tiles of 64 consecutive entries, one tile per
// block at a time (S waves per block).  Tiles differ in cost (chord lengths,
// misses); when a block has many to do it takes them from a ticket counter
// of its XCD, in the XCD's chunk order of the static split.
template <int NB, int FK, int GK, bool BF>
__global__ __launch_bounds__(64 * MAX_SEG) void k_march_queue(MarchArgs A, int L) {
  __shared__ TileLds<NB> T;
  unsigned long long* ctr = A.w.ctr;
  const unsigned long long qs = ctr[CTR_LSTART + L];
  // appends past the capacity are dropped (and flagged), never read
  const unsigned long long qe = min(ctr[CTR_CURSOR], (unsigned long long)A.w.qcap);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[CTR_LSTART + L + 1] = qe;
  const int lane = threadIdx.x & (WAVE - 1), sh = A.g.seg_shift;
  const int64_t SV = A.img.S, VS = (int64_t)A.img.V * SV;
  const bool range = L == 0 && A.w.rmin != nullptr;  // uniform: level 0 holds only level-0 nodes
  unsigned long long hit = 0, vis = 0;
  const long long ntiles = (long long)((qe - qs + WAVE - 1) / WAVE);
  __shared__ unsigned long long s_ticket;
  Split sp = xcd_split(ntiles);
  unsigned long long* ticket = ctr + CTR_TILE + 8 * L + sp.x;
  // trace the tile and store its rays' values (every thread of the block)
  auto trace_and_store = [&](bool trace, bool live, uint32_t v, uint32_t lev, uint32_t key, uint32_t i, uint32_t j) {
    RayRes<NB> r;
    if (range)
      trace_tile<NB, FK, GK, true, BF>(A, T, trace, v, (int)lev, i, j, sh, r);
    else
      trace_tile<NB, FK, GK, false, BF>(A, T, trace, v, (int)lev, i, j, sh, r);
    if (threadIdx.x < WAVE && live && !trace) {
      const int64_t pos = (int64_t)v * SV + A.img.off[lev] + key;
      A.w.state[pos] = A.w.state[pos] | ST_TRACED;
    }
    if (threadIdx.x < WAVE && trace) {
      const int64_t pos = (int64_t)v * SV + A.img.off[lev] + key;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b < A.f.nb) A.w.valI[b * VS + pos] = r.I[b];
      A.w.valN[pos] = r.N;
      A.w.visits[pos] = r.nvis;
      A.w.state[pos] = A.w.state[pos] | ST_TRACED;
      if (range) {
        const int64_t q0 = (int64_t)v * A.img.N0 * A.img.N0 + key;
        A.w.rmin[q0] = r.rmin;
        A.w.rmax[q0] = r.rmax;
        A.w.lmax0[q0] = r.lmax;
      }
      hit += r.hit;
      vis += (unsigned long long)r.nvis;
    }
  };
  // many tiles per block: take them from the XCD's ticket counter (one
  // atomic per tile); few: the static split (a ticket's round trip would sit
  // on every tile's path)
  const bool dyn = ntiles > 4 * (long long)gridDim.x;
  const long long kend = xcd_items(ntiles);
  for (;; sp.k += dyn ? 0 : sp.step) {
    if (dyn) {
      if (threadIdx.x == 0) s_ticket = atomicAdd(ticket, 1ull);
      __syncthreads();
      sp.k = (long long)s_ticket;
      __syncthreads();  // s_ticket is rewritten by the next iteration
      if (!sp.ok()) break;  // an XCD's tiles grow with k
    } else {
      if (sp.k >= kend) break;
      if (!sp.ok()) continue;
    }
    const unsigned long long e = qs + (unsigned long long)sp.tile() * WAVE + lane;
    const bool live = e < qe;
    uint32_t v = 0, lev = 0, key = 0, i = 0, j = 0;
    bool trace = live;
    if (live) {
      qdecode(A.w.queue[e], v, lev, key);
      coords_of(key, (int)lev, A.img.N0, i, j);
      // learned mode: a speculatively traced node already holds its values
      if (A.w.skip_spec) trace = !(A.w.state[(int64_t)v * SV + A.img.off[lev] + key] & ST_SPEC);
    }
    if (__ballot(trace)) {  // the same 64 entries in every wave: uniform per block
      trace_and_store(trace, live, v, lev, key, i, j);
    } else if (threadIdx.x < WAVE && live) {
      const int64_t pos = (int64_t)v * SV + A.img.off[lev] + key;
      A.w.state[pos] = A.w.state[pos] | ST_TRACED;
    }
  }
  block_stats(ctr, hit, vis);
}

// Split tiles.  At the coarse levels a launch holds few tiles and their
// rays lie cells apart, so the lanes of a wave read distinct cache lines
// and a tile's time is set by how fast its one compute unit pulls lines
// from L2.  There each (tile, sub-interval) march runs as its own wave job
// (the jobs of one tile land in different blocks), the partials go to
// A.w.parts, and k_fold_parts folds each tile's S partials in the order of
// the LDS fold, so the results are bit-identical to trace_tile's.  The host
// picks this form only when the launch cannot hold more than split_tiles
// tiles; a larger count (impossible) is flagged as an overflow.
template <int NB>
__device__ __forceinline__ float* part_rec(const MarchArgs& A, long long t, int k, int sh) {
  return A.w.parts + (((t << sh) + k) * split_fields(NB)) * WAVE + (threadIdx.x & (WAVE - 1));
}

template <int NB, int FK, int GK, bool RANGE>
__global__ __launch_bounds__(256) void k_march_parts(MarchArgs A, int L) {
  unsigned long long* ctr = A.w.ctr;
  const unsigned long long qs = ctr[CTR_LSTART + L];
  const unsigned long long qe = min(ctr[CTR_CURSOR], (unsigned long long)A.w.qcap);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[CTR_LSTART + L + 1] = qe;
  const long long ntiles = (long long)((qe - qs + WAVE - 1) / WAVE);
  if (ntiles > A.w.split_tiles) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctr[CTR_OVERFLOW], 1ull);
    return;
  }
  const int lane = threadIdx.x & (WAVE - 1), sh = A.g.seg_shift, wpb = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
  const int64_t SV = A.img.S;
  // job = k * ntiles + t: the waves of a block march neighbouring tiles, the
  // S parts of a tile go to S different blocks
  const long long njobs = ntiles << sh, nblk = (njobs + wpb - 1) / wpb;
  Split sp = xcd_split(nblk);
  const long long kend = xcd_items(nblk);
  for (; sp.k < kend; sp.k += sp.step) {
    if (!sp.ok()) continue;
    const long long job = sp.tile() * wpb + wv;
    if (job >= njobs) continue;  // uniform per wave
    const int k = (int)(job / ntiles);
    const long long t = job - (long long)k * ntiles;
    const unsigned long long e = qs + (unsigned long long)t * WAVE + lane;
    const bool live = e < qe;
    uint32_t v = 0, lev = 0, key = 0, i = 0, j = 0;
    bool trace = live;
    if (live) {
      qdecode(A.w.queue[e], v, lev, key);
      coords_of(key, (int)lev, A.img.N0, i, j);
      if (A.w.skip_spec) trace = !(A.w.state[(int64_t)v * SV + A.img.off[lev] + key] & ST_SPEC);
    }
    if (!__ballot(trace)) continue;  // the fold marks the tile
    Seg<NB> sg;
    int nvis;
    const bool hit = march_lane<NB, FK, GK, RANGE, true>(A, trace, v, (int)lev, i, j, k, sh, sg, nvis);
    float* P = part_rec<NB>(A, t, k, sh);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      P[b * WAVE] = sg.I[b];
      P[(NB + b) * WAVE] = sg.tau[b];
    }
    P[2 * NB * WAVE] = sg.N;
    if constexpr (RANGE) {
      P[(2 * NB + 1) * WAVE] = sg.rmin;
      P[(2 * NB + 2) * WAVE] = sg.rmax;
    }
    if constexpr (GK == AIR_GRID_BLOCK_AMR) {
      P[(2 * NB + 3) * WAVE] = __int_as_float(sg.nvis);
      P[(2 * NB + 4) * WAVE] = __int_as_float(sg.lmax);
    }
    if (k == 0) {
      P[(2 * NB + 5) * WAVE] = __int_as_float(nvis);
      P[(2 * NB + 6) * WAVE] = hit ? 1.0f : 0.0f;
    }
  }
}

// one wave per tile: fold the tile's S partials (the arithmetic of
// trace_tile's fold), then store like k_march_queue
template <int NB, int GK, bool RANGE>
__global__ __launch_bounds__(256) void k_fold_parts(MarchArgs A, int L) {
  unsigned long long* ctr = A.w.ctr;
  const unsigned long long qs = ctr[CTR_LSTART + L], qe = ctr[CTR_LSTART + L + 1];
  const long long ntiles = (long long)((qe - qs + WAVE - 1) / WAVE);
  if (ntiles > A.w.split_tiles) return;  // flagged by k_march_parts
  const int lane = threadIdx.x & (WAVE - 1), sh = A.g.seg_shift, S = 1 << sh, wpb = blockDim.x / WAVE;
  const int64_t SV = A.img.S, VS = (int64_t)A.img.V * SV;
  unsigned long long hit = 0, vis = 0;
  for (long long t = (long long)blockIdx.x * wpb + threadIdx.x / WAVE; t < ntiles; t += (long long)gridDim.x * wpb) {
    const unsigned long long e = qs + (unsigned long long)t * WAVE + lane;
    const bool live = e < qe;
    uint32_t v = 0, lev = 0, key = 0;
    bool trace = live;
    if (live) {
      qdecode(A.w.queue[e], v, lev, key);
      if (A.w.skip_spec) trace = !(A.w.state[(int64_t)v * SV + A.img.off[lev] + key] & ST_SPEC);
    }
    const int64_t pos = (int64_t)v * SV + A.img.off[lev] + key;
    if (live && !trace) A.w.state[pos] = A.w.state[pos] | ST_TRACED;
    if (!trace) continue;  // no shuffles below: lanes may leave
    const float* P0 = part_rec<NB>(A, t, 0, sh);
    float accI[NB], accT[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      accI[b] = P0[b * WAVE];
      accT[b] = P0[(NB + b) * WAVE];
    }
    float accN = P0[2 * NB * WAVE];
    float mn = 0.0f, mx = 0.0f;
    if constexpr (RANGE) {
      mn = P0[(2 * NB + 1) * WAVE];
      mx = P0[(2 * NB + 2) * WAVE];
    }
    int cells = 0, lm = -1;
    if constexpr (GK == AIR_GRID_BLOCK_AMR) {
      cells = __float_as_int(P0[(2 * NB + 3) * WAVE]);
      lm = __float_as_int(P0[(2 * NB + 4) * WAVE]);
    }
    for (int q = 1; q < S; ++q) {
      const float* P = part_rec<NB>(A, t, q, sh);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        accI[b] += __builtin_amdgcn_exp2f(-accT[b] * LOG2E_F) * P[b * WAVE];
        accT[b] += P[(NB + b) * WAVE];
      }
      accN += P[2 * NB * WAVE];
      if constexpr (RANGE) {
        mn = fminf(mn, P[(2 * NB + 1) * WAVE]);
        mx = fmaxf(mx, P[(2 * NB + 2) * WAVE]);
      }
      if constexpr (GK == AIR_GRID_BLOCK_AMR) {
        cells += __float_as_int(P[(2 * NB + 3) * WAVE]);
        lm = max(lm, __float_as_int(P[(2 * NB + 4) * WAVE]));
      }
    }
    const bool rhit = P0[(2 * NB + 6) * WAVE] != 0.0f;
    const int rnvis = GK == AIR_GRID_BLOCK_AMR ? cells : __float_as_int(P0[(2 * NB + 5) * WAVE]);
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b < A.f.nb) A.w.valI[b * VS + pos] = accI[b];
    A.w.valN[pos] = accN;
    A.w.visits[pos] = rnvis;
    A.w.state[pos] = A.w.state[pos] | ST_TRACED;
    if constexpr (RANGE) {
      const int64_t q0 = (int64_t)v * A.img.N0 * A.img.N0 + key;
      A.w.rmin[q0] = rhit ? mn : 0.0f;
      A.w.rmax[q0] = rhit ? mx : 0.0f;
      A.w.lmax0[q0] = rhit ? (GK == AIR_GRID_BLOCK_AMR ? lm : 0) : -1;
    }
    hit += rhit;
    vis += (unsigned long long)rnvis;
  }
  wave_stats(ctr, hit, vis);
}

// Speculative march of the learned proposal: the entries of spec, of any
// level; values land in the level maps as in the level march, marked
// ST_SPEC (not ST_TRACED: the refinement test of a level sees a node only
// once the level loop has reached it).
template <int NB, int FK, int GK>
__global__ __launch_bounds__(64 * MAX_SEG) void k_march_spec(MarchArgs A, const uint64_t* spec,
                                                             const unsigned long long* count) {
  __shared__ TileLds<NB> T;
  const unsigned long long n = *count;
  const int lane = threadIdx.x & (WAVE - 1), sh = A.g.seg_shift;
  const int64_t SV = A.img.S, VS = (int64_t)A.img.V * SV;
  unsigned long long hit = 0, vis = 0;
  const long long ntiles = (long long)((n + WAVE - 1) / WAVE);
  Split sp = xcd_split(ntiles);
  const long long kend = xcd_items(ntiles);
  for (; sp.k < kend; sp.k += sp.step) {
    if (!sp.ok()) continue;
    const unsigned long long e = (unsigned long long)sp.tile() * WAVE + lane;
    const bool live = e < n;
    uint32_t v = 0, lev = 0, key = 0, i = 0, j = 0;
    if (live) {
      qdecode(spec[e], v, lev, key);
      coords_of(key, (int)lev, A.img.N0, i, j);
    }
    RayRes<NB> r;
    trace_tile<NB, FK, GK, false, false>(A, T, live, v, (int)lev, i, j, sh, r);
    if (threadIdx.x < WAVE && live) {
      const int64_t pos = (int64_t)v * SV + A.img.off[lev] + key;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b < A.f.nb) A.w.valI[b * VS + pos] = r.I[b];
      A.w.valN[pos] = r.N;
      A.w.visits[pos] = r.nvis;
      A.w.state[pos] = A.w.state[pos] | ST_SPEC;
      hit += r.hit;
      vis += (unsigned long long)r.nvis;
    }
  }
  block_stats(A.w.ctr, hit, vis);
}

// fixed raster: entry e = view * R^2 + key, key in forest-Morton order
template <int NB, int FK, int GK>
__global__ __launch_bounds__(64 * MAX_SEG) void k_march_fixed(MarchArgs A, int L, float* images) {
  __shared__ TileLds<NB> T;
  const int64_t R = (int64_t)A.img.N0 << L, R2 = R * R;
  const unsigned long long total = (unsigned long long)A.img.V * R2;
  const int lane = threadIdx.x & (WAVE - 1), sh = A.g.seg_shift;
  unsigned long long hit = 0, vis = 0;
  const long long ntiles = (long long)((total + WAVE - 1) / WAVE);
  Split sp = xcd_split(ntiles);
  const long long kend = xcd_items(ntiles);
  for (; sp.k < kend; sp.k += sp.step) {
    if (!sp.ok()) continue;
    const unsigned long long e = (unsigned long long)sp.tile() * WAVE + lane;
    const bool live = e < total;
    uint32_t v = 0, key = 0, i = 0, j = 0;
    if (live) {
      v = (uint32_t)(e / R2);
      key = (uint32_t)(e % R2);
      coords_of(key, L, A.img.N0, i, j);
    }
    RayRes<NB> r;
    // the fixed image keeps the one general walk (its register budget holds
    // four waves per SIMD only without the single-axis copy)
    trace_tile<NB, FK, GK, false, false, false>(A, T, live, v, L, i, j, sh, r);
    if (threadIdx.x < WAVE && live) {
      if (images) {
        float* img = images + (int64_t)v * (A.f.nb + 1) * R2 + (int64_t)j * R + i;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b < A.f.nb) __builtin_nontemporal_store(r.I[b], img + b * R2);  // write-once output
        __builtin_nontemporal_store(r.N, img + A.f.nb * R2);
      }
      hit += r.hit;
      vis += (unsigned long long)r.nvis;
    }
  }
  block_stats(A.w.ctr, hit, vis);
}

template <int NB, int FK, int GK>
__global__ __launch_bounds__(64 * MAX_SEG) void k_trace_pixels(MarchArgs A, int64_t n, const int32_t* level,
                                                               const int32_t* ix, const int32_t* iy, float* I,
                                                               float* N, int32_t* visits) {
  __shared__ TileLds<NB> T;
  const int lane = threadIdx.x & (WAVE - 1), sh = A.g.seg_shift;
  for (int64_t b0 = (int64_t)blockIdx.x * WAVE; b0 < n; b0 += (int64_t)gridDim.x * WAVE) {  // uniform per block
    const int64_t k = b0 + lane;
    const bool live = k < n;
    RayRes<NB> r;
    trace_tile<NB, FK, GK, false, false>(A, T, live, 0, live ? level[k] : 0, live ? (uint32_t)ix[k] : 0u,
                                  live ? (uint32_t)iy[k] : 0u, sh, r);
    if (threadIdx.x < WAVE && live) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b < A.f.nb) I[b * n + k] = r.I[b];
      if (N) N[k] = r.N;
      if (visits) visits[k] = r.nvis;
    }
  }
}

}  // namespace

// ----------------------------------------------------------- dispatch
#define AIR_DISPATCH_NB(NBV, FKV, GKV, ...)                                      \
  do {                                                                           \
    if (FKV == AIR_FIELD_RHO_J_KAPPA || NBV == 1) {                              \
      constexpr int NB_ = 1, FK_ = AIR_FIELD_RHO_J_KAPPA, GK_ = GKV;             \
      __VA_ARGS__;                                                               \
    } else if (FKV == FK_LADDER) {                                               \
      if (NBV == 2) {                                                            \
        constexpr int NB_ = 2, FK_ = FK_LADDER, GK_ = GKV;                       \
        __VA_ARGS__;                                                             \
      } else if (NBV <= 4) {                                                     \
        constexpr int NB_ = 4, FK_ = FK_LADDER, GK_ = GKV;                       \
        __VA_ARGS__;                                                             \
      } else {                                                                   \
        constexpr int NB_ = 8, FK_ = FK_LADDER, GK_ = GKV;                       \
        __VA_ARGS__;                                                             \
      }                                                                          \
    } else if (NBV == 2) {                                                       \
      constexpr int NB_ = 2, FK_ = AIR_FIELD_RHO_T, GK_ = GKV;                   \
      __VA_ARGS__;                                                               \
    } else if (NBV <= 4) {                                                       \
      constexpr int NB_ = 4, FK_ = AIR_FIELD_RHO_T, GK_ = GKV;                   \
      __VA_ARGS__;                                                               \
    } else {                                                                     \
      constexpr int NB_ = 8, FK_ = AIR_FIELD_RHO_T, GK_ = GKV;                   \
      __VA_ARGS__;                                                               \
    }                                                                            \
  } while (0)
#define AIR_DISPATCH(A_, ...)                                                    \
  do {                                                                           \
    const int fk_ = (A_).f.ladder ? FK_LADDER : (A_).f.kind;                     \
    if ((A_).g.kind == AIR_GRID_BLOCK_AMR)                                       \
      AIR_DISPATCH_NB((A_).f.nb, fk_, AIR_GRID_BLOCK_AMR, __VA_ARGS__);           \
    else                                                                         \
      AIR_DISPATCH_NB((A_).f.nb, fk_, AIR_GRID_UNIFORM, __VA_ARGS__);             \
  } while (0)

hipError_t launch_march_spec(const MarchArgs& a, const uint64_t* spec, const unsigned long long* count,
                             int grid_blocks, hipStream_t s) {
  const dim3 blk(WAVE << a.g.seg_shift);
  AIR_DISPATCH(a, hipLaunchKernelGGL((k_march_spec<NB_, FK_, GK_>), dim3(grid_blocks), blk, 0, s, a, spec, count));
  return hipGetLastError();
}

int pack_mode(const Fld& f) {
  if (f.kind == AIR_FIELD_RHO_J_KAPPA) return PACK_RJK;
  return f.nb == 1 ? PACK_RT_TO_RJK : PACK_RT;
}

hipError_t launch_pack_amr(const Geo& g, const Fld& f, void* packed, hipStream_t s) {
  Fld F = f;
  F.packed = packed;
  switch (pack_mode(f)) {
    case PACK_RJK: hipLaunchKernelGGL(k_pack_amr<PACK_RJK>, dim3(4096), dim3(256), 0, s, g, F); break;
    case PACK_RT_TO_RJK: hipLaunchKernelGGL(k_pack_amr<PACK_RT_TO_RJK>, dim3(4096), dim3(256), 0, s, g, F); break;
    default: hipLaunchKernelGGL(k_pack_amr<PACK_RT>, dim3(4096), dim3(256), 0, s, g, F);
  }
  return hipGetLastError();
}

hipError_t launch_leaf_map(const Geo& g, const Fld& f, void* packed, hipStream_t s) {
  Fld F = f;
  F.packed = packed;
  hipLaunchKernelGGL(k_leaf_map, dim3(1024), dim3(256), 0, s, g, F);
  return hipGetLastError();
}

hipError_t launch_pack(const Geo& g, const Fld& f, void* packed, hipStream_t s) {
  Fld F = f;
  F.packed = packed;
  switch (pack_mode(f)) {
    case PACK_RJK: hipLaunchKernelGGL(k_pack<PACK_RJK>, dim3(4096), dim3(256), 0, s, g, F); break;
    case PACK_RT_TO_RJK: hipLaunchKernelGGL(k_pack<PACK_RT_TO_RJK>, dim3(4096), dim3(256), 0, s, g, F); break;
    default: hipLaunchKernelGGL(k_pack<PACK_RT>, dim3(4096), dim3(256), 0, s, g, F);
  }
  return hipGetLastError();
}

hipError_t launch_init(const MarchArgs& a, hipStream_t s) {
  const int64_t per_view = std::max<int64_t>(1, std::min<int64_t>(2048, (a.img.S / 16 + 255) / 256));
  hipLaunchKernelGGL(k_init, dim3((unsigned)per_view, (unsigned)a.img.V), dim3(256), 0, s, a);
  return hipGetLastError();
}

// tiles a queue launch of level L can hold: the level's nodes and balance
// nodes of coarser levels, at most every position of levels 0..L
int64_t queue_tile_bound(const MarchArgs& a, int L) {
  int64_t bound = 0;
  for (int l = 0; l <= L; ++l) bound += ((int64_t)a.img.N0 * a.img.N0) << (2 * l);
  return (bound * a.img.V + WAVE - 1) / WAVE;
}

// rays of level L at least one (coarsest-level) cell apart in every view:
// the lanes of a wave step different axes, so the walk goes branch-free
bool coarse_level(const MarchArgs& a, int L) {
  double h = a.g.h[0];
  for (int ax = 1; ax < 3; ++ax) h = std::max(h, a.g.h[ax]);
  return a.img.min_width / (double)((int64_t)a.img.N0 << L) >= h;
}

bool split_level(const MarchArgs& a, int L) {
  // level 0 reads the field cold and is bound by DRAM in either form
  return L >= 1 && a.w.split_tiles > 0 && queue_tile_bound(a, L) <= a.w.split_tiles;
}

// rays of level L at least half a (coarsest-level) cell apart in every view
bool sparse_level(const MarchArgs& a, int L) {
  double h = a.g.h[0];
  for (int ax = 1; ax < 3; ++ax) h = std::max(h, a.g.h[ax]);
  return a.img.min_width / (double)((int64_t)a.img.N0 << L) >= 0.5 * h;
}

template <int NB, int FK, int GK>
hipError_t queue_launch(const MarchArgs& a, int L, int grid_blocks, hipStream_t s) {
  if (!split_level(a, L)) {
    const dim3 blk(WAVE << a.g.seg_shift);
    if (coarse_level(a, L))
      hipLaunchKernelGGL((k_march_queue<NB, FK, GK, true>), dim3(grid_blocks), blk, 0, s, a, L);
    else
      hipLaunchKernelGGL((k_march_queue<NB, FK, GK, false>), dim3(grid_blocks), blk, 0, s, a, L);
    return hipGetLastError();
  }
  const int64_t tiles = queue_tile_bound(a, L), jobs = tiles << a.g.seg_shift;
  const int pg = (int)std::min<int64_t>(std::max<int64_t>((jobs + 4 * 8 - 1) / (4 * 8) * 8, 8), 8192);
  const int fg = (int)std::min<int64_t>((tiles + 3) / 4, 4096);
  hipLaunchKernelGGL((k_march_parts<NB, FK, GK, false>), dim3(pg), dim3(256), 0, s, a, L);
  hipLaunchKernelGGL((k_fold_parts<NB, GK, false>), dim3(fg), dim3(256), 0, s, a, L);
  return hipGetLastError();
}

hipError_t launch_march_queue(const MarchArgs& a, int L, int grid_blocks, hipStream_t s) {
  if (a.f.rt_bytes && a.f.packed && sparse_level(a, L)) {  // the (rho, T) copy
    MarchArgs b = a;
    b.f.packed = static_cast<const char*>(a.f.packed) + a.f.rt_off;
    b.f.packed_bytes = a.f.rt_bytes;
    return queue_launch<1, AIR_FIELD_RHO_T, AIR_GRID_UNIFORM>(b, L, grid_blocks, s);
  }
  AIR_DISPATCH(a, return (queue_launch<NB_, FK_, GK_>(a, L, grid_blocks, s)));
  return hipSuccess;
}

hipError_t launch_march_fixed(const MarchArgs& a, int level, float* images, int grid_blocks, hipStream_t s) {
  const dim3 blk(WAVE << a.g.seg_shift);
  AIR_DISPATCH(a, hipLaunchKernelGGL((k_march_fixed<NB_, FK_, GK_>), dim3(grid_blocks), blk, 0, s, a, level, images));
  return hipGetLastError();
}

hipError_t launch_trace_pixels(const MarchArgs& a, int64_t n, const int32_t* level, const int32_t* ix,
                               const int32_t* iy, float* I, float* N, int32_t* visits, hipStream_t s) {
  int blocks = (int)std::min<int64_t>((n + WAVE - 1) / WAVE, 4096);
  if (blocks < 1) blocks = 1;
  const dim3 blk(WAVE << a.g.seg_shift);
  AIR_DISPATCH(a, hipLaunchKernelGGL((k_trace_pixels<NB_, FK_, GK_>), dim3(blocks), blk, 0, s, a, n, level, ix, iy, I,
                                      N, visits));
  return hipGetLastError();
}

}  // namespace air
