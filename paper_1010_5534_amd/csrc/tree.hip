// Image-tree kernels: refinement test, 2:1 closure and work-queue
// compaction for one level (section 2 steps iii-iv), then the canonical node
// list, the quadtree-to-raster assembler and the flux (step vi).
//
// The pixel tree of every view lives in dense per-level maps indexed by the
// forest-Morton key (parent = key >> 2, children = 4 key + 0..3), one state
// byte per position.  A node is "traced" once its ray's values are written;
// the test at level L reads only traced values, so nodes created while the
// test runs (children, balance nodes) never leak into it, and the test, the
// closure and the compaction run as one pass per level.
#include "air_common.h"

namespace air {

namespace {

constexpr int RB = 128;             // refine block size
constexpr int STK = 2 * MAXL + 2;   // closure stack depth bound (2L + 1)

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t state_or(uint8_t* state, int64_t p, uint32_t bits) {
  const uint32_t sh = 8u * (uint32_t)(p & 3);
  uint32_t old = atomicOr(reinterpret_cast<uint32_t*>(state + (p - (p & 3))), bits << sh);
  return (old >> sh) & 0xffu;
}

// Eq. 3 on a 3x3 stencil p[(b+1)*3 + (a+1)], a along u, b along v:
// squared second differences (the mixed one for both orderings) over the
// squared sums of absolute first differences; the mixed denominator uses
// the first differences along one direction at the two offsets of the other
// (scaled like the mixed numerator), so each term is bounded and xi <= 1.
// A direction without both neighbours drops its terms and the mixed ones;
// a zero denominator gives 0.
__device__ __forceinline__ float xi_of(const float* p, bool hx, bool hy) {
  float num = 0.0f, den = 0.0f;
  if (hx) {
    const float n = (p[5] - p[4]) - (p[4] - p[3]);
    const float d = fabsf(p[5] - p[4]) + fabsf(p[4] - p[3]);
    num += n * n;
    den += d * d;
  }
  if (hy) {
    const float n = (p[7] - p[4]) - (p[4] - p[1]);
    const float d = fabsf(p[7] - p[4]) + fabsf(p[4] - p[1]);
    num += n * n;
    den += d * d;
  }
  if (hx && hy) {
    const float a = p[8] - p[6], b = p[2] - p[0];  // u-differences at v = +1, -1
    const float c = p[8] - p[2], e = p[6] - p[0];  // v-differences at u = +1, -1
    const float nxy = 0.25f * (a - b);
    const float dxy = 0.25f * (fabsf(a) + fabsf(b));
    const float dyx = 0.25f * (fabsf(c) + fabsf(e));
    num += 2.0f * nxy * nxy;
    den += dxy * dxy + dyx * dyx;
  }
  if (den == 0.0f) return 0.0f;
  return sqrtf(num / den);
}

struct BandW {
  float w[MAXB];
};

__global__ __launch_bounds__(RB) void k_refine(MarchArgs A, int L, float xcI, float xcN, BandW W) {
  __shared__ uint64_t stk[STK][RB];
  unsigned long long* ctr = A.w.ctr;
  const unsigned long long qs = ctr[CTR_LSTART + L], qe = ctr[CTR_LSTART + L + 1];
  const int N0 = A.img.N0, nb = A.f.nb;
  const int64_t S = A.img.S, VS = (int64_t)A.img.V * S;
  const uint32_t R = (uint32_t)N0 << L;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1);
  const uint64_t qcap = A.w.qcap;
  for (unsigned long long base = (unsigned long long)blockIdx.x * RB; base < qe - qs;
       base += (unsigned long long)gridDim.x * RB) {
    const unsigned long long e = qs + base + tid;
    bool live = e < qe, flag = false;
    uint32_t v = 0, lev = 0, key = 0, i = 0, j = 0;
    int64_t vb = 0;
    if (live) {
      qdecode(A.w.queue[e], v, lev, key);
      live = (int)lev == L;  // balance nodes of lower levels are never tested
    }
    if (live) {
      coords_of(key, L, N0, i, j);
      vb = (int64_t)v * S;
      float pI[9], pN[9];
#pragma unroll
      for (int b = -1; b <= 1; ++b)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
          const int k = (b + 1) * 3 + (a + 1);
          const int qi = (int)i + a, qj = (int)j + b;
          if (qi < 0 || qj < 0 || qi >= (int)R || qj >= (int)R) {
            pI[k] = pN[k] = 0.0f;
            continue;
          }
          const uint32_t kq = key_of((uint32_t)qi, (uint32_t)qj, L, N0);
          int64_t p = vb + A.img.off[L] + kq;
          if (!(A.w.state[p] & ST_TRACED)) p = vb + A.img.off[L - 1] + (kq >> 2);  // covering coarser node
          float s = 0.0f;
          for (int bb = 0; bb < nb; ++bb) s += W.w[bb] * A.w.valI[bb * VS + p];
          pI[k] = s;
          pN[k] = A.w.valN[p];
        }
      const bool hx = i > 0 && i + 1 < R, hy = j > 0 && j + 1 < R;
      const float xI = xi_of(pI, hx, hy), xN = xi_of(pN, hx, hy);
      const int64_t pos = vb + A.img.off[L] + key;
      A.w.xiI[pos] = xI;
      A.w.xiN[pos] = xN;
      flag = (xI >= xcI) || (xN >= xcN);
      state_or(A.w.state, pos,
               AIR_NODE_EVALUATED | (flag ? (AIR_NODE_FLAGGED | AIR_NODE_REFINED) : 0u));
      if (flag)  // four tested children (4-byte aligned: offsets are multiples of 256)
        atomicOr(reinterpret_cast<uint32_t*>(A.w.state + vb + A.img.off[L + 1] + 4ll * key),
                 0x01010101u * (AIR_NODE_EXIST | AIR_NODE_TESTED));
    }
    // children of the flagged nodes of this wave: one queue reservation
    const uint64_t mask = __ballot(flag);
    if (mask) {
      const int leader = __builtin_ctzll(mask);
      unsigned long long dst = 0;
      if (lane == leader) dst = atomicAdd(&ctr[CTR_CURSOR], 4ull * (unsigned long long)__popcll(mask));
      dst = __shfl(dst, leader);
      if (flag) {
        dst += 4ull * lanes_below(mask);
        if (dst + 4 <= qcap) {
#pragma unroll
          for (uint32_t c = 0; c < 4; ++c) A.w.queue[dst + c] = qentry(v, L + 1, 4u * key + c);
        } else {
          atomicOr(&ctr[CTR_OVERFLOW], 1ull);
        }
      }
    }
    // 2:1 closure: every edge/corner neighbour of a flagged node must exist
    // before its children do.  A missing neighbour's parent is refined, after
    // making that parent's own neighbours exist, recursively down the levels.
    // The REFINED bit is claimed atomically, so each refinement is done once
    // and the result is the unique minimal closure whatever the order.
    if (flag && L >= 1) {
      int sp = 0;
      auto request = [&](int l, uint32_t qi, uint32_t qj) {
        const uint32_t kq = key_of(qi, qj, l, N0);
        const uint32_t old = state_or(A.w.state, vb + A.img.off[l] + kq, AIR_NODE_REFINED);
        if (!(old & AIR_NODE_REFINED)) stk[sp++][tid] = ((uint64_t)l << 32) | kq;
      };
      // the parents of the 8 neighbours of (l, ni, nj), other than its own
      auto around = [&](int l, uint32_t ni, uint32_t nj) {
        const int pi = (int)(ni >> 1), pj = (int)(nj >> 1);
        const int ai = pi + ((ni & 1) ? 1 : -1), aj = pj + ((nj & 1) ? 1 : -1);
        const int R1 = N0 << (l - 1);
        const bool okx = ai >= 0 && ai < R1, oky = aj >= 0 && aj < R1;
        if (okx) request(l - 1, (uint32_t)ai, (uint32_t)pj);
        if (oky) request(l - 1, (uint32_t)pi, (uint32_t)aj);
        if (okx && oky) request(l - 1, (uint32_t)ai, (uint32_t)aj);
      };
      around(L, i, j);
      while (sp > 0) {
        const uint64_t t = stk[--sp][tid];
        const int l = (int)(t >> 32);
        const uint32_t kq = (uint32_t)t;
        if (l >= 1) {
          uint32_t qi, qj;
          coords_of(kq, l, N0, qi, qj);
          around(l, qi, qj);
        }
        atomicOr(reinterpret_cast<uint32_t*>(A.w.state + vb + A.img.off[l + 1] + 4ll * kq),
                 0x01010101u * (AIR_NODE_EXIST | AIR_NODE_BALANCE));
        const unsigned long long d = atomicAdd(&ctr[CTR_CURSOR], 4ull);
        if (d + 4 <= qcap) {
          for (uint32_t c = 0; c < 4; ++c) A.w.queue[d + c] = qentry(v, l + 1, 4u * kq + c);
        } else {
          atomicOr(&ctr[CTR_OVERFLOW], 1ull);
        }
      }
    }
  }
}

// level of a position inside a view
__device__ __forceinline__ int level_of(const Img& img, int64_t local) {
  int L = 0;
  while (L < img.Lmax && local >= img.off[L + 1]) ++L;
  return L;
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long x, unsigned long long* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  unsigned long long t = 0;
  for (int k = 0; k < nw; ++k) t += sh[k];
  return t;
}

// per chunk of CHUNK positions: existing nodes; plus the tree counters
__global__ __launch_bounds__(256) void k_count(MarchArgs A, unsigned long long* chunk_counts,
                                               unsigned long long* vstat) {
  __shared__ unsigned long long sh[4];
  __shared__ unsigned long long lv[MAXL];
  const int64_t c = blockIdx.x;
  const int64_t S = A.img.S;
  const int64_t v = (c * CHUNK) / S;  // S is a multiple of CHUNK
  if (threadIdx.x < MAXL) lv[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long n = 0, leaves = 0, tested = 0, flagged = 0, bal = 0;
  for (int k = 0; k < CHUNK / 256; ++k) {
    const int64_t p = c * CHUNK + k * 256 + threadIdx.x;
    const uint8_t s = A.w.state[p];
    if (s & AIR_NODE_EXIST) {
      ++n;
      leaves += !(s & AIR_NODE_REFINED);
      tested += (s & AIR_NODE_EVALUATED) != 0;
      flagged += (s & AIR_NODE_FLAGGED) != 0;
      bal += (s & AIR_NODE_BALANCE) != 0;
      atomicAdd(&lv[level_of(A.img, p % S)], 1ull);
    }
  }
  const unsigned long long tot = block_sum_u64(n, sh);
  const unsigned long long tl = block_sum_u64(leaves, sh);
  const unsigned long long tt = block_sum_u64(tested, sh);
  const unsigned long long tf = block_sum_u64(flagged, sh);
  const unsigned long long tb = block_sum_u64(bal, sh);
  if (threadIdx.x == 0) {
    chunk_counts[c] = tot;
    unsigned long long* ctr = A.w.ctr;
    if (tl) atomicAdd(&ctr[CTR_LEAVES], tl);
    if (tl) atomicAdd(&vstat[v * (MAXL + 1) + MAXL], tl);
    if (tt) atomicAdd(&ctr[CTR_TESTED], tt);
    if (tf) atomicAdd(&ctr[CTR_FLAGGED], tf);
    if (tb) atomicAdd(&ctr[CTR_BALANCE], tb);
  }
  if (threadIdx.x < MAXL && lv[threadIdx.x]) {
    atomicAdd(&A.w.ctr[CTR_NODES + threadIdx.x], lv[threadIdx.x]);
    atomicAdd(&vstat[v * (MAXL + 1) + threadIdx.x], lv[threadIdx.x]);
  }
}

// exclusive scan of the chunk counts (one block; n_chunks is modest)
__global__ __launch_bounds__(1024) void k_scan(unsigned long long* a, int64_t n) {
  __shared__ unsigned long long part[1024];
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = threadIdx.x * per, e = min<int64_t>(b + per, n);
  unsigned long long s = 0;
  for (int64_t k = b; k < e; ++k) s += a[k];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int k = 0; k < 1024; ++k) {
      unsigned long long t = part[k];
      part[k] = run;
      run += t;
    }
  }
  __syncthreads();
  unsigned long long run = part[threadIdx.x];
  for (int64_t k = b; k < e; ++k) {
    unsigned long long t = a[k];
    a[k] = run;
    run += t;
  }
  if (e == n && b < e) a[n] = run;  // total after the last element
  if (n == 0 && threadIdx.x == 0) a[0] = 0;
}

// node ids: exclusive prefix of existing positions in canonical order
__global__ __launch_bounds__(256) void k_emit(MarchArgs A, const unsigned long long* chunk_off, int32_t* id_map) {
  __shared__ unsigned long long sh[4];
  const int64_t c = blockIdx.x;
  unsigned long long run = chunk_off[c];
  for (int k = 0; k < CHUNK / 256; ++k) {
    const int64_t p = c * CHUNK + k * 256 + threadIdx.x;
    const bool ex = (A.w.state[p] & AIR_NODE_EXIST) != 0;
    const uint64_t m = __ballot(ex);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = __popcll(m);
    __syncthreads();
    unsigned long long before = 0, tot = 0;
    for (int q = 0; q < 4; ++q) {
      if (q < w) before += sh[q];
      tot += sh[q];
    }
    if (ex) id_map[p] = (int32_t)(run + before + lanes_below(m));
    run += tot;
  }
}

__global__ __launch_bounds__(256) void k_write_tree(MarchArgs A, const unsigned long long* chunk_off,
                                                    const int32_t* id_map, const TreeOut* outs) {
  const int64_t S = A.img.S, VS = (int64_t)A.img.V * S, cpv = S / CHUNK;
  const int N0 = A.img.N0, nb = A.f.nb;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < VS; p += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t s = A.w.state[p];
    if (!(s & AIR_NODE_EXIST)) continue;
    const int v = (int)(p / S);
    const int64_t local = p - (int64_t)v * S;
    const int L = level_of(A.img, local);
    const uint32_t key = (uint32_t)(local - A.img.off[L]);
    const TreeOut& T = outs[v];
    const int64_t base = (int64_t)chunk_off[v * cpv];
    const int64_t id = (int64_t)id_map[p] - base;
    if (id >= T.capacity) continue;
    uint32_t i, j;
    coords_of(key, L, N0, i, j);
    if (T.level) T.level[id] = (int8_t)L;
    if (T.ix) T.ix[id] = (int32_t)i;
    if (T.iy) T.iy[id] = (int32_t)j;
    if (T.parent)
      T.parent[id] = L == 0 ? -1 : (int32_t)(id_map[(int64_t)v * S + A.img.off[L - 1] + (key >> 2)] - base);
    if (T.first_child)
      T.first_child[id] = (s & AIR_NODE_REFINED)
                              ? (int32_t)(id_map[(int64_t)v * S + A.img.off[L + 1] + 4ll * key] - base)
                              : -1;
    if (T.state) T.state[id] = s & (uint8_t)~ST_TRACED;
    if (T.I)
      for (int b = 0; b < nb; ++b) T.I[b * T.capacity + id] = A.w.valI[b * VS + p];
    if (T.N) T.N[id] = A.w.valN[p];
    const bool ev = (s & AIR_NODE_EVALUATED) != 0;
    if (T.xi_I) T.xi_I[id] = ev ? A.w.xiI[p] : __builtin_nanf("");
    if (T.xi_N) T.xi_N[id] = ev ? A.w.xiN[p] : __builtin_nanf("");
    if (T.visits) T.visits[id] = A.w.visits[p];
  }
}

// raster of the leaves: each finest pixel descends from its coarse pixel
__global__ __launch_bounds__(256) void k_assemble(MarchArgs A, float* images) {
  const int N0 = A.img.N0, Lm = A.img.Lmax, nb = A.f.nb;
  const int64_t R = (int64_t)N0 << Lm, R2 = R * R, S = A.img.S, VS = (int64_t)A.img.V * S;
  const int64_t total = (int64_t)A.img.V * R2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int v = (int)(e / R2);
    const int64_t r = e - (int64_t)v * R2;
    const uint32_t i = (uint32_t)(r % R), j = (uint32_t)(r / R);
    const int64_t vb = (int64_t)v * S;
    uint32_t key = (j >> Lm) * (uint32_t)N0 + (i >> Lm);
    int L = 0;
    int64_t p = vb + key;
    while (L < Lm && (A.w.state[p] & AIR_NODE_REFINED)) {
      ++L;
      const int sh = Lm - L;
      key = 4u * key + (((i >> sh) & 1u) | (((j >> sh) & 1u) << 1));
      p = vb + A.img.off[L] + key;
    }
    float* img = images + (int64_t)v * (nb + 1) * R2 + r;
    for (int b = 0; b < nb; ++b) img[b * R2] = A.w.valI[b * VS + p];
    img[nb * R2] = A.w.valN[p];
  }
}

// flux partials per chunk and band: sum over leaves of (pixel area) I_b,
// float64, fixed reduction order
__global__ __launch_bounds__(256) void k_flux_partial(MarchArgs A, const DevView* views, double* partial) {
  __shared__ double sh[256];
  const int64_t c = blockIdx.x, S = A.img.S, VS = (int64_t)A.img.V * S;
  const int nb = A.f.nb;
  for (int b = 0; b < nb; ++b) {
    double s = 0.0;
    for (int k = 0; k < CHUNK / 256; ++k) {
      const int64_t p = c * CHUNK + k * 256 + threadIdx.x;
      const uint8_t st = A.w.state[p];
      if ((st & AIR_NODE_EXIST) && !(st & AIR_NODE_REFINED)) {
        const int v = (int)(p / S);
        const int L = level_of(A.img, p - (int64_t)v * S);
        const double px = views[v].width / (double)((int64_t)A.img.N0 << L);
        s += px * px * (double)A.w.valI[b * VS + p];
      }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[c * nb + b] = sh[0];
    __syncthreads();
  }
}

// per (view, band): sum the view's chunk partials in order
__global__ void k_flux_final(const double* partial, int64_t chunks_per_view, int V, int nb, double* flux) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V * nb) return;
  const int v = t / nb, b = t % nb;
  double s = 0.0;
  for (int64_t c = 0; c < chunks_per_view; ++c) s += partial[((int64_t)v * chunks_per_view + c) * nb + b];
  flux[t] = s;
}

// fixed image flux: per (view, band, chunk of raster) partials
__global__ __launch_bounds__(256) void k_fixed_partial(const float* images, int nb, int64_t R2, double area,
                                                       int64_t chunks_per_plane, double* partial) {
  __shared__ double sh[256];
  const int64_t c = blockIdx.x;                 // over V * nb * chunks_per_plane
  const int64_t plane = c / chunks_per_plane;   // v * (nb + 1) + b  mapped below
  const int64_t v = plane / nb, b = plane % nb;
  const float* img = images + (v * (nb + 1) + b) * R2;
  const int64_t beg = (c % chunks_per_plane) * CHUNK;
  double s = 0.0;
  for (int k = 0; k < CHUNK / 256; ++k) {
    const int64_t q = beg + k * 256 + threadIdx.x;
    if (q < R2) s += area * (double)img[q];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[c] = sh[0];
}

__global__ void k_fixed_final(const double* partial, int64_t chunks_per_plane, int n_planes, double* flux) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_planes) return;
  double s = 0.0;
  for (int64_t c = 0; c < chunks_per_plane; ++c) s += partial[(int64_t)t * chunks_per_plane + c];
  flux[t] = s;
}

}  // namespace

hipError_t launch_refine(const MarchArgs& a, int L, float xcI, float xcN, const float* w, int grid_blocks,
                         hipStream_t s) {
  BandW W;
  for (int b = 0; b < MAXB; ++b) W.w[b] = w[b];
  hipLaunchKernelGGL(k_refine, dim3(grid_blocks), dim3(RB), 0, s, a, L, xcI, xcN, W);
  return hipGetLastError();
}

hipError_t launch_count(const MarchArgs& a, unsigned long long* chunk_counts, int64_t n_chunks,
                        unsigned long long* vstat, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3((unsigned)n_chunks), dim3(256), 0, s, a, chunk_counts, vstat);
  return hipGetLastError();
}

hipError_t launch_scan(unsigned long long* chunk_counts, int64_t n_chunks, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, chunk_counts, n_chunks);
  return hipGetLastError();
}

hipError_t launch_emit(const MarchArgs& a, const unsigned long long* chunk_offsets, int64_t n_chunks,
                       int32_t* id_map, hipStream_t s) {
  hipLaunchKernelGGL(k_emit, dim3((unsigned)n_chunks), dim3(256), 0, s, a, chunk_offsets, id_map);
  return hipGetLastError();
}

hipError_t launch_write_tree(const MarchArgs& a, const unsigned long long* chunk_offsets, const int32_t* id_map,
                             const TreeOut* outs, hipStream_t s) {
  hipLaunchKernelGGL(k_write_tree, dim3(4096), dim3(256), 0, s, a, chunk_offsets, id_map, outs);
  return hipGetLastError();
}

hipError_t launch_assemble(const MarchArgs& a, float* images, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble, dim3(8192), dim3(256), 0, s, a, images);
  return hipGetLastError();
}

hipError_t launch_flux(const MarchArgs& a, double* partial, int64_t n_chunks, double* flux_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_flux_partial, dim3((unsigned)n_chunks), dim3(256), 0, s, a, a.views, partial);
  const int n = a.img.V * a.f.nb;
  hipLaunchKernelGGL(k_flux_final, dim3((n + 63) / 64), dim3(64), 0, s, partial, n_chunks / a.img.V, a.img.V,
                     a.f.nb, flux_dev);
  return hipGetLastError();
}

hipError_t launch_fixed_flux(const float* images, int V, int nb, int64_t R, double pix_area, double* partial,
                             double* flux_dev, hipStream_t s) {
  const int64_t R2 = R * R, cpp = (R2 + CHUNK - 1) / CHUNK;
  const int64_t n = (int64_t)V * nb * cpp;
  hipLaunchKernelGGL(k_fixed_partial, dim3((unsigned)n), dim3(256), 0, s, images, nb, R2, pix_area, cpp, partial);
  hipLaunchKernelGGL(k_fixed_final, dim3((V * nb + 63) / 64), dim3(64), 0, s, partial, cpp, V * nb, flux_dev);
  return hipGetLastError();
}

}  // namespace air
