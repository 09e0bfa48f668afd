// Ray march kernels for adaptive image ray-tracing on gfx950.
//
// One lane traces one pixel's ray (section 2 step ii); a wavefront takes 64
// consecutive work-queue entries, which in forest-Morton order are an 8x8
// pixel tile of a complete subtree, so its lanes walk neighbouring cell
// columns and their field loads share cache lines.  Waves pull tiles from a
// per-level ticket counter, so the grid is sized to the machine, not to the
// (data-dependent) queue length.
//
// Along each ray the exact solution for cell-constant j, kappa, rho is
// accumulated front to back:
//   I_b += exp(-tau_b) j_b ds (1 - exp(-kappa_b ds)) / (kappa_b ds),
//   tau_b += kappa_b ds,  N += rho ds,
// in float32 with Kahan-compensated sums.  Ray-box entry and the DDA's
// per-axis crossing parameters are formed in float64 and carried as
// float-float pairs; each crossing time is rebuilt from its integer count
// (t = t_first + k dt), so no rounding accumulates along the ray and every
// segment length is a difference of two correctly rounded values.
#include "air_common.h"

namespace air {

namespace {

constexpr float LOG2E_F = 1.4426950408889634f;

struct ff {
  float hi, lo;
};

__device__ __forceinline__ ff ff_of(double x) {
  float h = (float)x;
  return {h, (float)(x - (double)h)};
}

// T0 + k*D, float-float, k a crossing count (exact in float)
__device__ __forceinline__ ff ff_axpy(int k, ff D, ff T0) {
#pragma clang fp contract(off)
  float kf = (float)k;
  float p = kf * D.hi;
  float pe = __builtin_fmaf(kf, D.hi, -p);  // exact error of the product
  float pl = __builtin_fmaf(kf, D.lo, pe);
  float s = T0.hi + p;  // two-sum of T0.hi and p
  float z = s - T0.hi;
  float se = (T0.hi - (s - z)) + (p - z);
  return {s, (se + pl) + T0.lo};
}

__device__ __forceinline__ void kadd(float& s, float& c, float x) {
#pragma clang fp contract(off)
  float y = x - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

// (1 - e^-x)/x: Taylor series below 1/4 (truncation < 2e-9 relative),
// direct form above (cancellation at most a factor 4.5)
__device__ __forceinline__ float seg_weight(float x) {
  if (x < 0.25f) {
    float y = -x;
    float p = 1.0f / 5040.0f;
    p = __builtin_fmaf(p, y, 1.0f / 720.0f);
    p = __builtin_fmaf(p, y, 1.0f / 120.0f);
    p = __builtin_fmaf(p, y, 1.0f / 24.0f);
    p = __builtin_fmaf(p, y, 1.0f / 6.0f);
    p = __builtin_fmaf(p, y, 0.5f);
    p = __builtin_fmaf(p, y, 1.0f);
    return p;
  }
  float e = __builtin_amdgcn_exp2f(-x * LOG2E_F);
  return (1.0f - e) * __builtin_amdgcn_rcpf(x);
}

template <int NB>
struct RayRes {
  float I[NB];
  float N;
  int nvis;
  bool hit;
  float rmin, rmax;
};

// per-cell optics of band b
template <int NB, int FK>
struct Optics {
  float rho;
  float j[NB], k[NB];
};

template <int NB, int FK>
__device__ __forceinline__ void load_optics(const Fld& f, int idx, Optics<NB, FK>& o) {
  if constexpr (FK == AIR_FIELD_RHO_J_KAPPA) {
    o.rho = f.rho[idx];
    o.j[0] = f.emis[idx];
    o.k[0] = f.kappa[idx];
  } else {
    float r = f.rho[idx];
    float T = f.temp[idx];
    o.rho = r;
    float lt = __builtin_amdgcn_logf(T);  // log2 T
    float r2 = r * r;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      o.k[b] = f.k0[b] * r * __builtin_amdgcn_exp2f(-f.s[b] * lt);
      o.j[b] = r2 * __builtin_amdgcn_exp2f(f.q[b] * lt);
    }
  }
}

// Ray x(t) = o + t d (d unit) through the uniform grid, DDA from the entry.
template <int NB, int FK, bool RANGE>
__device__ void march_uniform(const Geo& g, const Fld& f, const double o[3], const double d[3],
                              RayRes<NB>& r) {
#pragma unroll
  for (int b = 0; b < NB; ++b) r.I[b] = 0.0f;
  r.N = 0.0f;
  r.nvis = 0;
  r.hit = false;
  r.rmin = 0.0f;
  r.rmax = 0.0f;

  // slab entry / exit, float64
  double t0 = -__builtin_huge_val(), t1 = __builtin_huge_val();
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0) {
      double ta = (g.lo[a] - o[a]) / d[a], tb = (g.hi[a] - o[a]) / d[a];
      t0 = fmax(t0, fmin(ta, tb));
      t1 = fmin(t1, fmax(ta, tb));
    } else if (!(o[a] >= g.lo[a] && o[a] < g.hi[a])) {
      inside = false;
    }
  }
  if (!inside || !(t0 < t1)) return;

  // entry and exit cells (the cell just after t0 / just before t1), the
  // number of cells crossed, and the first crossing of each axis relative
  // to the entry, all from float64
  int c[3], st[3], nvis = 1;
  ff T0[3], D[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int n = g.n[a];
    double u0 = (o[a] + t0 * d[a] - g.lo[a]) / g.h[a];
    double u1 = (o[a] + t1 * d[a] - g.lo[a]) / g.h[a];
    int k0, k1;
    if (d[a] > 0.0) {
      k0 = (int)floor(u0);
      k1 = (int)ceil(u1) - 1;
    } else if (d[a] < 0.0) {
      k0 = (int)ceil(u0) - 1;
      k1 = (int)floor(u1);
    } else {
      k0 = k1 = (int)floor(u0);
    }
    k0 = min(max(k0, 0), n - 1);
    k1 = min(max(k1, 0), n - 1);
    c[a] = k0;
    nvis += abs(k1 - k0);
    if (d[a] != 0.0) {
      int m = d[a] > 0.0 ? k0 + 1 : k0;
      double tf = (g.lo[a] + (double)m * g.h[a] - o[a]) / d[a] - t0;
      T0[a] = ff_of(tf);
      D[a] = ff_of(g.h[a] / fabs(d[a]));
      st[a] = d[a] > 0.0 ? 1 : -1;
    } else {
      T0[a] = {__builtin_huge_valf(), 0.0f};
      D[a] = {0.0f, 0.0f};
      st[a] = 0;
    }
  }
  const ff S1 = ff_of(t1 - t0);
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];

  float I[NB], cI[NB], tau[NB], ctau[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) I[b] = cI[b] = tau[b] = ctau[b] = 0.0f;
  float N = 0.0f, cN = 0.0f;
  float rmin = __builtin_huge_valf(), rmax = -__builtin_huge_valf();

  int cx = c[0], cy = c[1], cz = c[2];
  int k0 = 0, k1 = 0, k2 = 0;
  ff ta0 = T0[0], ta1 = T0[1], ta2 = T0[2];
  ff tc = {0.0f, 0.0f};
  int idx = cx + nx * (cy + ny * cz);
  Optics<NB, FK> op;
  load_optics<NB, FK>(f, idx, op);
  for (int v = 0; v < nvis; ++v) {
    ff tn;
    int ax;
    if (v == nvis - 1) {
      tn = S1;
      ax = 3;
    } else {
      ax = (ta0.hi <= ta1.hi) ? (ta0.hi <= ta2.hi ? 0 : 2) : (ta1.hi <= ta2.hi ? 1 : 2);
      tn = ax == 0 ? ta0 : (ax == 1 ? ta1 : ta2);
    }
    const float ds = (tn.hi - tc.hi) + (tn.lo - tc.lo);
    tc = tn;
    // step the DDA and start the next cell's loads before integrating this one
    if (ax == 0) {
      ++k0;
      ta0 = ff_axpy(k0, D[0], T0[0]);
      cx = min(max(cx + st[0], 0), nx - 1);
    } else if (ax == 1) {
      ++k1;
      ta1 = ff_axpy(k1, D[1], T0[1]);
      cy = min(max(cy + st[1], 0), ny - 1);
    } else if (ax == 2) {
      ++k2;
      ta2 = ff_axpy(k2, D[2], T0[2]);
      cz = min(max(cz + st[2], 0), nz - 1);
    }
    const Optics<NB, FK> cur = op;
    if (ax != 3) {
      idx = cx + nx * (cy + ny * cz);
      load_optics<NB, FK>(f, idx, op);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float dtau = cur.k[b] * ds;
      const float T = __builtin_amdgcn_exp2f(-(tau[b] - ctau[b]) * LOG2E_F);
      kadd(I[b], cI[b], T * (cur.j[b] * ds) * seg_weight(dtau));
      kadd(tau[b], ctau[b], dtau);
    }
    kadd(N, cN, cur.rho * ds);
    if constexpr (RANGE) {
      rmin = fminf(rmin, cur.rho);
      rmax = fmaxf(rmax, cur.rho);
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) r.I[b] = I[b] - cI[b];
  r.N = N - cN;
  r.nvis = nvis;
  r.hit = true;
  if constexpr (RANGE) {
    r.rmin = rmin;
    r.rmax = rmax;
  }
}

__device__ __forceinline__ void pixel_ray(const DevView& V, int N0, int L, uint32_t i, uint32_t j,
                                          double o[3]) {
  const double s = V.width / (double)((int64_t)N0 << L);
  const double au = -0.5 * V.width + ((double)i + 0.5) * s;
  const double av = -0.5 * V.width + ((double)j + 0.5) * s;
#pragma unroll
  for (int a = 0; a < 3; ++a) o[a] = V.c[a] + au * V.eu[a] + av * V.ev[a];
}

template <int NB, int FK, bool RANGE>
__device__ __forceinline__ void trace_pixel(const MarchArgs& A, uint32_t v, int L, uint32_t i, uint32_t j,
                                            RayRes<NB>& r) {
  const DevView& V = A.views[v];
  double o[3];
  pixel_ray(V, A.img.N0, L, i, j, o);
  march_uniform<NB, FK, RANGE>(A.g, A.f, o, V.d, r);
}

__device__ __forceinline__ void wave_add(unsigned long long* p, unsigned long long x) {
  // one atomic per wave
  unsigned long long s = x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(p, s);
}

// ------------------------------------------------------------ kernels
__global__ void k_init(MarchArgs A) {
  const int64_t V = A.img.V, S = A.img.S, n0sq = (int64_t)A.img.N0 * A.img.N0;
  const int64_t words = V * S / 4;
  uint32_t* st = reinterpret_cast<uint32_t*>(A.w.state);
  const uint32_t base_bits = AIR_NODE_EXIST | AIR_NODE_TESTED;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < words;
       w += (int64_t)gridDim.x * blockDim.x) {
    int64_t local = (4 * w) % S;  // level 0 occupies [0, N0^2) of every view
    uint32_t word = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (local + b < n0sq) word |= base_bits << (8 * b);
    st[w] = word;
  }
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < V * n0sq;
       e += (int64_t)gridDim.x * blockDim.x)
    A.w.queue[e] = qentry((uint32_t)(e / n0sq), 0, (uint32_t)(e % n0sq));
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < CTR_COUNT; k += blockDim.x)
      A.w.ctr[k] = k == CTR_CURSOR ? (unsigned long long)(V * n0sq) : 0ull;
}

template <int NB, int FK>
__global__ __launch_bounds__(256) void k_march_queue(MarchArgs A, int L) {
  unsigned long long* ctr = A.w.ctr;
  const unsigned long long qs = ctr[CTR_LSTART + L];
  // appends past the capacity are dropped (and flagged), never read
  const unsigned long long qe = min(ctr[CTR_CURSOR], (unsigned long long)A.w.qcap);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[CTR_LSTART + L + 1] = qe;
  const unsigned long long ntiles = (qe - qs + WAVE - 1) / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t S = A.img.S;
  for (;;) {
    unsigned long long t = 0;
    if (lane == 0) t = atomicAdd(&ctr[CTR_TILE + L], 1ull);
    t = __shfl(t, 0);
    if (t >= ntiles) break;
    const unsigned long long e = qs + t * WAVE + lane;
    unsigned long long hit = 0, vis = 0;
    if (e < qe) {
      uint32_t v, lev, key;
      qdecode(A.w.queue[e], v, lev, key);
      uint32_t i, j;
      coords_of(key, (int)lev, A.img.N0, i, j);
      RayRes<NB> r;
      if (lev == 0 && A.w.rmin) {
        trace_pixel<NB, FK, true>(A, v, (int)lev, i, j, r);
        A.w.rmin[(int64_t)v * A.img.N0 * A.img.N0 + key] = r.rmin;
        A.w.rmax[(int64_t)v * A.img.N0 * A.img.N0 + key] = r.rmax;
      } else {
        trace_pixel<NB, FK, false>(A, v, (int)lev, i, j, r);
      }
      const int64_t pos = (int64_t)v * S + A.img.off[lev] + key;
      const int64_t VS = (int64_t)A.img.V * S;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b < A.f.nb) A.w.valI[b * VS + pos] = r.I[b];
      A.w.valN[pos] = r.N;
      A.w.visits[pos] = r.nvis;
      A.w.state[pos] = A.w.state[pos] | ST_TRACED;
      hit = r.hit;
      vis = (unsigned long long)r.nvis;
    }
    wave_add(&ctr[CTR_HITS], hit);
    wave_add(&ctr[CTR_VISITS], vis);
  }
}

// fixed raster: entry e = view * R^2 + key, key in forest-Morton order
template <int NB, int FK>
__global__ __launch_bounds__(256) void k_march_fixed(MarchArgs A, int L, float* images) {
  unsigned long long* ctr = A.w.ctr;
  const int64_t R = (int64_t)A.img.N0 << L, R2 = R * R;
  const unsigned long long total = (unsigned long long)A.img.V * R2;
  const unsigned long long ntiles = (total + WAVE - 1) / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  for (;;) {
    unsigned long long t = 0;
    if (lane == 0) t = atomicAdd(&ctr[CTR_TILE], 1ull);
    t = __shfl(t, 0);
    if (t >= ntiles) break;
    const unsigned long long e = t * WAVE + lane;
    unsigned long long hit = 0, vis = 0;
    if (e < total) {
      const uint32_t v = (uint32_t)(e / R2), key = (uint32_t)(e % R2);
      uint32_t i, j;
      coords_of(key, L, A.img.N0, i, j);
      RayRes<NB> r;
      trace_pixel<NB, FK, false>(A, v, L, i, j, r);
      if (images) {
        float* img = images + (int64_t)v * (NB + 1) * R2 + (int64_t)j * R + i;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b < A.f.nb) img[b * R2] = r.I[b];
        img[A.f.nb * R2] = r.N;
      }
      hit = r.hit;
      vis = (unsigned long long)r.nvis;
    }
    wave_add(&ctr[CTR_HITS], hit);
    wave_add(&ctr[CTR_VISITS], vis);
  }
}

template <int NB, int FK>
__global__ __launch_bounds__(256) void k_trace_pixels(MarchArgs A, int64_t n, const int32_t* level,
                                                      const int32_t* ix, const int32_t* iy, float* I,
                                                      float* N, int32_t* visits) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    RayRes<NB> r;
    trace_pixel<NB, FK, false>(A, 0, level[k], (uint32_t)ix[k], (uint32_t)iy[k], r);
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b < A.f.nb) I[b * n + k] = r.I[b];
    if (N) N[k] = r.N;
    if (visits) visits[k] = r.nvis;
  }
}

}  // namespace

// ----------------------------------------------------------- dispatch
#define AIR_DISPATCH(NBV, FKV, CALL)                                             \
  do {                                                                           \
    if (FKV == AIR_FIELD_RHO_J_KAPPA) {                                          \
      constexpr int NB_ = 1, FK_ = AIR_FIELD_RHO_J_KAPPA;                        \
      CALL;                                                                      \
    } else if (NBV == 1) {                                                       \
      constexpr int NB_ = 1, FK_ = AIR_FIELD_RHO_T;                              \
      CALL;                                                                      \
    } else if (NBV == 2) {                                                       \
      constexpr int NB_ = 2, FK_ = AIR_FIELD_RHO_T;                              \
      CALL;                                                                      \
    } else if (NBV <= 4) {                                                       \
      constexpr int NB_ = 4, FK_ = AIR_FIELD_RHO_T;                              \
      CALL;                                                                      \
    } else {                                                                     \
      constexpr int NB_ = 8, FK_ = AIR_FIELD_RHO_T;                              \
      CALL;                                                                      \
    }                                                                            \
  } while (0)

hipError_t launch_init(const MarchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(2048), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_march_queue(const MarchArgs& a, int L, int grid_blocks, hipStream_t s) {
  AIR_DISPATCH(a.f.nb, a.f.kind,
               hipLaunchKernelGGL((k_march_queue<NB_, FK_>), dim3(grid_blocks), dim3(256), 0, s, a, L));
  return hipGetLastError();
}

hipError_t launch_march_fixed(const MarchArgs& a, int level, float* images, int grid_blocks, hipStream_t s) {
  AIR_DISPATCH(a.f.nb, a.f.kind,
               hipLaunchKernelGGL((k_march_fixed<NB_, FK_>), dim3(grid_blocks), dim3(256), 0, s, a, level,
                                  images));
  return hipGetLastError();
}

hipError_t launch_trace_pixels(const MarchArgs& a, int64_t n, const int32_t* level, const int32_t* ix,
                               const int32_t* iy, float* I, float* N, int32_t* visits, hipStream_t s) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  AIR_DISPATCH(a.f.nb, a.f.kind,
               hipLaunchKernelGGL((k_trace_pixels<NB_, FK_>), dim3(blocks), dim3(256), 0, s, a, n, level, ix, iy,
                                  I, N, visits));
  return hipGetLastError();
}

}  // namespace air
