// Per-pixel spectra with many energy bins (section 2 step vi: integrated
// quantities such as broadband images, and the note that an integrated
// spectrum needs every pixel's spectrum kept until the image is final).
//
// The spectral march gives one wave to one ray and one lane to each bin
// (four bins per lane and pass, 256 per pass, passes for more): every lane
// walks the same cells, so the (rho, T) loads are one address per wave and
// the work per visit is the bins' optics and exponentials, spread over the
// lanes.  Each traced ray leaves its spectrum in a store indexed by its work
// queue position and its broadband value sum_b w_b I_b (reduced over the
// lanes in a fixed order) in the level maps, where the refinement test reads
// it.  Once the tree is final the spectra are gathered into canonical node
// order and the leaves' spectra integrated into the image's spectrum.
#include "air_common.h"

namespace air {

namespace {

constexpr float LOG2E = 1.4426950408889634f;
constexpr float THICK_X = 0.25f;
constexpr int BPL = 4;              // bins per lane and pass
constexpr int PASS = BPL * WAVE;    // bins per pass

__device__ __forceinline__ void kahan(float& s, float& c, float x) {
#pragma clang fp contract(off)
  const float y = x - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// (1 - e^-x)/x for 0 <= x < 1/4 (Taylor series, truncation < 2e-9 relative)
__device__ __forceinline__ float weight_series(float x) {
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

// box entry and exit along the ray (float64); false if it misses
__device__ bool box_chord(const Geo& g, const double o[3], const DevView& V, double& t0, double& t1) {
  t0 = -__builtin_huge_val();
  t1 = __builtin_huge_val();
  bool inside = true;
  for (int a = 0; a < 3; ++a) {
    if (V.d[a] != 0.0) {
      const double ta = (g.lo[a] - o[a]) * V.inv_d[a], tb = (g.hi[a] - o[a]) * V.inv_d[a];
      t0 = fmax(t0, fmin(ta, tb));
      t1 = fmin(t1, fmax(ta, tb));
    } else if (!(o[a] >= g.lo[a] && o[a] < g.hi[a])) {
      inside = false;
    }
  }
  return inside && t0 < t1;
}

// half-open cell of axis a holding the point just after (after) or just
// before parameter t
__device__ int axis_cell(const Geo& g, const double o[3], const double d[3], int a, double t, bool after) {
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

__device__ __forceinline__ float wave_sum(float x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

}  // namespace

// Spectral march of the level-L queue entries: one wave per ray.
__global__ __launch_bounds__(256) void k_march_spectra(MarchArgs A, SpecArgs S, int L) {
  unsigned long long* ctr = A.w.ctr;
  const unsigned long long qs = ctr[CTR_LSTART + L];
  const unsigned long long qe = min(ctr[CTR_CURSOR], (unsigned long long)A.w.qcap);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[CTR_LSTART + L + 1] = qe;
  const int lane = threadIdx.x & (WAVE - 1);
  const unsigned long long wid = ((unsigned long long)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const unsigned long long nw = (unsigned long long)gridDim.x * blockDim.x / WAVE;
  const int64_t SV = A.img.S;
  const int nbins = S.nbins;
  const Geo& g = A.g;
  unsigned long long hits = 0, visits = 0;
  for (unsigned long long e = qs + wid; e < qe; e += nw) {
    uint32_t v, lev, key, i, j;
    qdecode(A.w.queue[e], v, lev, key);
    coords_of(key, (int)lev, A.img.N0, i, j);
    const DevView& V = A.views[v];
    double o[3];
    const double px = V.width / (double)((int64_t)A.img.N0 << lev);
    const double au = -0.5 * V.width + ((double)i + 0.5) * px, av = -0.5 * V.width + ((double)j + 0.5) * px;
    for (int a = 0; a < 3; ++a) o[a] = V.c[a] + au * V.eu[a] + av * V.ev[a];
    double ta, tb;
    const bool hit = box_chord(g, o, V, ta, tb);
    // the walk, in float64: every lane takes the same step, so its cost is
    // shared by the ray's bins, and a short segment (a ray grazing a cell of
    // the thin shocked shell, where the high-energy bins get most of their
    // emission) keeps its length to float64 rounding of the chord, not to
    // float32's.  The k-th crossing of an axis is fma(k, D, T0) from the
    // entry.
    int c0[3], st[3], nvis = 0;
    double T0[3], D[3];
    double S1 = 0.0;
    if (hit) {
      nvis = 1;
      for (int a = 0; a < 3; ++a) {
        const int k0 = axis_cell(g, o, V.d, a, ta, true), k1 = axis_cell(g, o, V.d, a, tb, false);
        c0[a] = k0;
        nvis += abs(k1 - k0);
        if (V.d[a] != 0.0) {
          const int m = V.d[a] > 0.0 ? k0 + 1 : k0;
          T0[a] = (g.lo[a] + (double)m * g.h[a] - o[a]) * V.inv_d[a] - ta;
          D[a] = g.h[a] * fabs(V.inv_d[a]);
          st[a] = V.d[a] > 0.0 ? 1 : -1;
        } else {
          T0[a] = __builtin_huge_val();
          D[a] = 0.0;
          st[a] = 0;
        }
      }
      S1 = tb - ta;
    }
    float N = 0.0f, cN = 0.0f, broad = 0.0f;
    for (int p0 = 0; p0 < nbins; p0 += PASS) {
      float k0b[BPL], msb[BPL], qb[BPL], eLb[BPL], e0b[BPL];
      float I[BPL], cI[BPL], tau[BPL], ctau[BPL], Tb[BPL];
      bool on[BPL];
#pragma unroll
      for (int q = 0; q < BPL; ++q) {
        const int b = p0 + q * WAVE + lane;
        on[q] = b < nbins;
        const int bc = on[q] ? b : 0;
        k0b[q] = S.tab[0 * S.stride + bc];
        msb[q] = S.tab[1 * S.stride + bc];
        qb[q] = S.tab[2 * S.stride + bc];
        eLb[q] = S.tab[3 * S.stride + bc];
        e0b[q] = S.tab[4 * S.stride + bc];
        I[q] = cI[q] = tau[q] = ctau[q] = 0.0f;
        Tb[q] = 1.0f;
      }
      int cx = c0[0], cy = c0[1], cz = c0[2];
      double k0 = 0.0, k1 = 0.0, k2 = 0.0, tc = 0.0;
      double t0 = hit ? T0[0] : 0.0, t1 = hit ? T0[1] : 0.0, t2 = hit ? T0[2] : 0.0;
      for (int n = 0; n < nvis; ++n) {  // nvis is the same in every lane
        const bool last = n == nvis - 1;
        const double tm = fmin(fmin(t0, t1), t2);
        const double tn = last ? S1 : tm;
        const float ds = (float)(tn - tc);
        const int64_t cell = cx + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz);
        const float rho = A.f.rho[cell], T = A.f.temp[cell];
        if (!last) {
          tc = tn;
          if (tm == t0) {
            k0 += 1.0;
            t0 = fma(k0, D[0], T0[0]);
            cx = min(max(cx + st[0], 0), g.n[0] - 1);
          } else if (tm == t1) {
            k1 += 1.0;
            t1 = fma(k1, D[1], T0[1]);
            cy = min(max(cy + st[1], 0), g.n[1] - 1);
          } else {
            k2 += 1.0;
            t2 = fma(k2, D[2], T0[2]);
            cz = min(max(cz + st[2], 0), g.n[2] - 1);
          }
        }
        const float lt = __builtin_amdgcn_logf(T);  // log2 T
        const float iT = __builtin_amdgcn_rcpf(T);
        const float r2 = rho * rho;
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
          const float kap = k0b[q] * rho * __builtin_amdgcn_exp2f(msb[q] * lt);
          const float jem = e0b[q] * r2 * __builtin_amdgcn_exp2f(__builtin_fmaf(qb[q], lt, eLb[q] * iT));
          const float dtau = kap * ds;
          kahan(tau[q], ctau[q], dtau);
          const float Ta = __builtin_amdgcn_exp2f(-(tau[q] - ctau[q]) * LOG2E);
          const float thin = Tb[q] * (jem * ds) * weight_series(dtau);
          const float thick = (Tb[q] - Ta) * jem * __builtin_amdgcn_rcpf(kap);
          kahan(I[q], cI[q], dtau < THICK_X ? thin : thick);
          Tb[q] = Ta;
        }
        if (p0 == 0) kahan(N, cN, rho * ds);
      }
#pragma unroll
      for (int q = 0; q < BPL; ++q) {
        const int b = p0 + q * WAVE + lane;
        const float val = I[q] - cI[q];
        if (on[q]) {
          if (e < S.cap) __builtin_nontemporal_store(val, S.store + e * (unsigned long long)nbins + b);
          broad += S.tab[5 * S.stride + b] * val;
        }
      }
    }
    broad = wave_sum(broad);
    if (lane == 0) {
      const int64_t pos = (int64_t)v * SV + A.img.off[lev] + key;
      A.w.valI[pos] = broad;
      A.w.valN[pos] = N - cN;
      A.w.visits[pos] = nvis;
      A.w.state[pos] = A.w.state[pos] | ST_TRACED;
      S.qpos[pos] = (uint32_t)min(e, (unsigned long long)0xffffffffu);
      if (e >= S.cap) atomicOr(S.overflow, 1u);
      hits += hit ? 1 : 0;
      visits += (unsigned long long)nvis;
    }
  }
  if (lane == 0) {
    const int slot = (int)(wid & (CTR_SLOTS - 1));
    if (hits) atomicAdd(&ctr[CTR_HITS + slot], hits);
    if (visits) atomicAdd(&ctr[CTR_VISITS + slot], visits);
  }
}

// Spectra into canonical node order: one wave per node, lanes over bins.
// Rows of view v start at out_row[v]; a node beyond its view's capacity or a
// store row beyond the store's is skipped (the call then reports the
// capacity error).
__global__ __launch_bounds__(256) void k_spectra_gather(MarchArgs A, SpecArgs S, const unsigned long long* chunk_off,
                                                        int64_t n_chunks, const uint64_t* node_pos, SpecOut O) {
  const unsigned long long total = chunk_off[n_chunks];
  const int64_t SV = A.img.S, cpv = SV / CHUNK;
  const int lane = threadIdx.x & (WAVE - 1);
  const unsigned long long nw = (unsigned long long)gridDim.x * blockDim.x / WAVE;
  for (unsigned long long gi = ((unsigned long long)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; gi < total;
       gi += nw) {
    const int64_t p = (int64_t)node_pos[gi];
    const int v = (int)(p / SV);
    const int64_t id = (int64_t)gi - (int64_t)chunk_off[v * cpv];
    const unsigned long long q = S.qpos[p];
    if (id >= O.cap[v] || q >= S.cap) continue;  // reported as a capacity error
    float* dst = O.spectra + (O.row0[v] + id) * (int64_t)S.nbins;
    const float* src = S.store + q * (unsigned long long)S.nbins;
    for (int b = lane; b < S.nbins; b += WAVE) __builtin_nontemporal_store(src[b], dst + b);
  }
}

// The image's spectrum: per (view, chunk of SPEC_CHUNK canonical nodes, bin)
// the sum over the chunk's leaves of pixel area times I_b in node order
// (float64), then per (view, bin) the chunks in order.  Block = one wave over
// 64 bins of one (view, chunk); the chunk's node data are staged in LDS first.
__global__ __launch_bounds__(64) void k_spectra_partial(MarchArgs A, SpecArgs S, const unsigned long long* chunk_off,
                                                        const uint64_t* node_pos, int64_t chunks_per_view,
                                                        double* partial) {
  __shared__ unsigned long long sq[SPEC_CHUNK];
  __shared__ double sa[SPEC_CHUNK];
  const int64_t SV = A.img.S, cpv = SV / CHUNK;
  const int nbg = (S.nbins + WAVE - 1) / WAVE;
  const int64_t blk = blockIdx.x;
  const int bg = (int)(blk % nbg);
  const int64_t vc = blk / nbg;
  const int v = (int)(vc / chunks_per_view);
  const int64_t c = vc % chunks_per_view;
  const int64_t base = (int64_t)chunk_off[v * cpv], end = (int64_t)chunk_off[(v + 1) * cpv];
  const int64_t lo = base + c * SPEC_CHUNK, hi = min(lo + SPEC_CHUNK, end);
  const double w = A.views[v].width;
  for (int k = threadIdx.x; k < SPEC_CHUNK; k += WAVE) {
    const int64_t gi = lo + k;
    double area = 0.0;
    unsigned long long q = 0;
    if (gi < hi) {
      const int64_t p = (int64_t)node_pos[gi];
      const uint8_t s = A.w.state[p];
      if ((s & AIR_NODE_EXIST) && !(s & AIR_NODE_REFINED)) {
        q = S.qpos[p];
        if (q < S.cap) {
          const int64_t local = p - (int64_t)v * SV;
          int L = 0;
          while (L < A.img.Lmax && local >= A.img.off[L + 1]) ++L;
          const double px = w / (double)((int64_t)A.img.N0 << L);
          area = px * px;
        }
      }
    }
    sq[k] = q;
    sa[k] = area;
  }
  __syncthreads();
  const int b = bg * WAVE + (int)threadIdx.x;
  if (b >= S.nbins) return;
  double acc = 0.0;
  const int n = hi > lo ? (int)(hi - lo) : 0;
  for (int k = 0; k < n; ++k)
    if (sa[k] != 0.0) acc += sa[k] * (double)S.store[sq[k] * (unsigned long long)S.nbins + b];
  partial[((int64_t)v * chunks_per_view + c) * S.nbins + b] = acc;
}

__global__ __launch_bounds__(256) void k_spectra_final(int V, int nbins, int64_t chunks_per_view,
                                                      const double* partial, double* flux) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < (int64_t)V * nbins;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = k / nbins, b = k % nbins;
    double s = 0.0;
    for (int64_t c = 0; c < chunks_per_view; ++c) s += partial[(v * chunks_per_view + c) * nbins + b];
    flux[k] = s;
  }
}

hipError_t launch_march_spectra(const MarchArgs& a, const SpecArgs& s, int L, int grid_blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_march_spectra, dim3(grid_blocks), dim3(256), 0, st, a, s, L);
  return hipGetLastError();
}

hipError_t launch_spectra_out(const MarchArgs& a, const SpecArgs& s, const unsigned long long* chunk_off,
                              int64_t n_chunks, const uint64_t* node_pos, const SpecOut& o, int64_t chunks_per_view,
                              double* partial, double* flux_dev, int grid_blocks, hipStream_t st) {
  if (o.spectra)
    hipLaunchKernelGGL(k_spectra_gather, dim3(grid_blocks), dim3(256), 0, st, a, s, chunk_off, n_chunks, node_pos, o);
  if (flux_dev) {
    const int nbg = (s.nbins + WAVE - 1) / WAVE;
    const int64_t blocks = (int64_t)a.img.V * chunks_per_view * nbg;
    hipLaunchKernelGGL(k_spectra_partial, dim3((unsigned)blocks), dim3(64), 0, st, a, s, chunk_off, node_pos,
                       chunks_per_view, partial);
    const int64_t n = (int64_t)a.img.V * s.nbins;
    hipLaunchKernelGGL(k_spectra_final, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st,
                       a.img.V, s.nbins, chunks_per_view, partial, flux_dev);
  }
  return hipGetLastError();
}

}  // namespace air
