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

constexpr int RB = 256;             // refine block size
constexpr int STK = 2 * MAXL;       // closure stack depth bound: 2L + 1 with L <= MAXL - 2
constexpr int BALQ = 16;            // closure refinements listed per thread (more go out directly)

__device__ __forceinline__ uint32_t state_or(uint8_t* state, int64_t p, uint32_t bits) {
  const uint32_t sh = 8u * (uint32_t)(p & 3);
  uint32_t old = atomicOr(reinterpret_cast<uint32_t*>(state + (p - (p & 3))), bits << sh);
  return (old >> sh) & 0xffu;
}
// state_or where on is true; elsewhere an OR of nothing (p must still be a
// valid position) that returns `bits`, as if already set.  Issued without a
// branch, so several claims can be in flight together.
__device__ __forceinline__ uint32_t state_or_if(uint8_t* state, int64_t p, bool on, uint32_t bits) {
  const uint32_t sh = 8u * (uint32_t)(p & 3);
  const uint32_t old = atomicOr(reinterpret_cast<uint32_t*>(state + (p - (p & 3))), on ? bits << sh : 0u);
  return on ? (old >> sh) & 0xffu : bits;
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
  __shared__ uint32_t stk_key[STK][RB];
  __shared__ uint8_t stk_lev[STK][RB];
  __shared__ uint32_t bal_key[BALQ][RB];  // closure refinements awaiting their queue entries
  __shared__ uint8_t bal_lev[BALQ][RB];
  __shared__ unsigned wcnt[RB / WAVE];
  __shared__ unsigned long long bbase;
  // level offsets for the closure, whose levels differ per thread (read
  // from the kernel arguments that would be one memory round trip each)
  __shared__ int64_t s_off[MAXL + 1];
  if (threadIdx.x <= MAXL) s_off[threadIdx.x] = A.img.off[threadIdx.x];
  __syncthreads();
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
      // the 3x3 stencil: the nine state bytes go out together, then the
      // nine positions' values (a neighbour not yet traced takes the
      // covering coarser node's; one outside the image is 0)
      const int64_t lb = vb + A.img.off[L], cb = vb + (L > 0 ? A.img.off[L - 1] : 0);
      uint32_t kq[9];
      bool in[9];
      uint8_t sq[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int qi = (int)i + k % 3 - 1, qj = (int)j + k / 3 - 1;
        in[k] = qi >= 0 && qj >= 0 && qi < (int)R && qj < (int)R;
        kq[k] = in[k] ? key_of((uint32_t)qi, (uint32_t)qj, L, N0) : key;  // outside: a valid stand-in
        sq[k] = A.w.state[lb + kq[k]];
      }
      int64_t pp[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) pp[k] = (sq[k] & ST_TRACED) ? lb + kq[k] : cb + (kq[k] >> 2);
      float pI[9], pN[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        pN[k] = A.w.valN[pp[k]];  // in flight with the first band's values
        pI[k] = 0.0f;
      }
      for (int bb = 0; bb < nb; ++bb) {
        const float wb = W.w[bb];
        const float* src = A.w.valI + bb * VS;
#pragma unroll
        for (int k = 0; k < 9; ++k) pI[k] += wb * src[pp[k]];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (!in[k]) pI[k] = pN[k] = 0.0f;
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
    // 2:1 closure: every edge/corner neighbour of a flagged node must exist
    // before its children do.  A missing neighbour's parent is refined, after
    // making that parent's own neighbours exist, recursively down the levels.
    // The REFINED bit is claimed atomically, so each refinement is done once
    // and the result is the unique minimal closure whatever the order.  The
    // refinements a thread claims are listed in LDS and their children queued
    // with the block's flagged children below.
    int nbal = 0;
    if (flag && L >= 1) {
      int sp = 0;
      // the parents of the 8 neighbours of (l, ni, nj), other than its own:
      // the three claims go out together
      auto around = [&](int l, uint32_t ni, uint32_t nj) {
        const int pi = (int)(ni >> 1), pj = (int)(nj >> 1);
        const int ai = pi + ((ni & 1) ? 1 : -1), aj = pj + ((nj & 1) ? 1 : -1);
        const int R1 = N0 << (l - 1);
        const bool okx = ai >= 0 && ai < R1, oky = aj >= 0 && aj < R1;
        const int64_t lb = vb + s_off[l - 1];
        const uint32_t k0 = okx ? key_of((uint32_t)ai, (uint32_t)pj, l - 1, N0) : 0u;
        const uint32_t k1 = oky ? key_of((uint32_t)pi, (uint32_t)aj, l - 1, N0) : 0u;
        const uint32_t k2 = okx && oky ? key_of((uint32_t)ai, (uint32_t)aj, l - 1, N0) : 0u;
        // a neighbour off the image claims nothing (at key 0, a valid position)
        const uint32_t o0 = state_or_if(A.w.state, lb + k0, okx, AIR_NODE_REFINED);
        const uint32_t o1 = state_or_if(A.w.state, lb + k1, oky, AIR_NODE_REFINED);
        const uint32_t o2 = state_or_if(A.w.state, lb + k2, okx && oky, AIR_NODE_REFINED);
        if (!(o0 & AIR_NODE_REFINED)) {
          stk_key[sp][tid] = k0;
          stk_lev[sp][tid] = (uint8_t)(l - 1);
          ++sp;
        }
        if (!(o1 & AIR_NODE_REFINED)) {
          stk_key[sp][tid] = k1;
          stk_lev[sp][tid] = (uint8_t)(l - 1);
          ++sp;
        }
        if (!(o2 & AIR_NODE_REFINED)) {
          stk_key[sp][tid] = k2;
          stk_lev[sp][tid] = (uint8_t)(l - 1);
          ++sp;
        }
      };
      around(L, i, j);
      while (sp > 0) {
        --sp;
        const int l = stk_lev[sp][tid];
        const uint32_t kq = stk_key[sp][tid];
        if (l >= 1) {
          uint32_t qi, qj;
          coords_of(kq, l, N0, qi, qj);
          around(l, qi, qj);
        }
        atomicOr(reinterpret_cast<uint32_t*>(A.w.state + vb + s_off[l + 1] + 4ll * kq),
                 0x01010101u * (AIR_NODE_EXIST | AIR_NODE_BALANCE));
        if (nbal < BALQ) {
          bal_key[nbal][tid] = kq;
          bal_lev[nbal][tid] = (uint8_t)l;
          ++nbal;
        } else {  // list full: queue the four children directly
          const unsigned long long d = atomicAdd(&ctr[CTR_CURSOR], 4ull);
          if (d + 4 <= qcap) {
            for (uint32_t c = 0; c < 4; ++c) A.w.queue[d + c] = qentry(v, l + 1, 4u * kq + c);
          } else {
            atomicOr(&ctr[CTR_OVERFLOW], 1ull);
          }
        }
      }
    }
    // the block's new queue entries (children of its flagged nodes, then of
    // its closure refinements): one reservation per block
    const unsigned mine = (flag ? 1u : 0u) + (unsigned)nbal;  // groups of four
    unsigned x = mine;  // inclusive prefix over the wave
    for (int o = 1; o < WAVE; o <<= 1) {
      const unsigned y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    const int w = tid / WAVE;
    if (lane == WAVE - 1) wcnt[w] = x;
    __syncthreads();
    if (tid == 0) {
      unsigned tot = 0;
      for (int q = 0; q < RB / WAVE; ++q) tot += wcnt[q];
      bbase = tot ? atomicAdd(&ctr[CTR_CURSOR], 4ull * tot) : 0ull;
    }
    __syncthreads();
    {
      unsigned before = x - mine;
      for (int q = 0; q < w; ++q) before += wcnt[q];
      unsigned long long dst = bbase + 4ull * before;
      __syncthreads();  // wcnt and bbase are rewritten by the next iteration
      if (mine && dst + 4ull * mine > qcap) {
        atomicOr(&ctr[CTR_OVERFLOW], 1ull);
      } else {
        if (flag) {
#pragma unroll
          for (uint32_t c = 0; c < 4; ++c) A.w.queue[dst + c] = qentry(v, L + 1, 4u * key + c);
          dst += 4;
        }
        for (int q = 0; q < nbal; ++q) {
          const uint32_t kq = bal_key[q][tid];
          const int l = bal_lev[q][tid];
#pragma unroll
          for (uint32_t c = 0; c < 4; ++c) A.w.queue[dst + c] = qentry(v, l + 1, 4u * kq + c);
          dst += 4;
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

// a counting chunk lies in one (view, level): its view, level and first key
struct ChunkPos {
  int v, L;
  int64_t key0;
};
__device__ __forceinline__ ChunkPos chunk_pos(const Img& img, int64_t c) {
  ChunkPos r;
  const int64_t p = c * CHUNK;
  r.v = (int)(p / img.S);
  const int64_t local = p - (int64_t)r.v * img.S;
  r.L = level_of(img, local);
  r.key0 = local - img.off[r.L];
  return r;
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

// the raster of the leaves: each thread paints QX consecutive pixels of one
// row of view v (block xb of the view's pixels).  An ancestor's key follows
// from the pixel alone, so the state bytes of every level above the pixels
// are loaded together (one round of loads, not one per level), the leaf is
// the shallowest ancestor that is not refined, and its value is gathered.
// QX = 4 (i a multiple of 4): levels up to Lm - 2 are shared by the four
// pixels, level Lm - 1 by pairs; 16-byte stores.
template <int QX>
__device__ __forceinline__ void paint_pixels(const MarchArgs& A, float* images, int v, int64_t xb) {
  const int N0 = A.img.N0, Lm = A.img.Lmax, nb = A.f.nb;
  const uint32_t R = (uint32_t)N0 << Lm;
  const int64_t R2 = (int64_t)R * R, VS = (int64_t)A.img.V * A.img.S;
  const int64_t vb = (int64_t)v * A.img.S;
  const int64_t e = (xb * 256 + threadIdx.x) * QX;
  if (e >= R2) return;
  const uint32_t i = (uint32_t)(e % R), j = (uint32_t)(e / R);
  const uint8_t* state = A.w.state + vb;
  int64_t offm = 0, offm1 = 0;  // offsets of levels Lm and Lm - 1 (selected statically: uniform registers)
#pragma unroll
  for (int L = 0; L <= MAXL; ++L) {
    if (L == Lm) offm = A.img.off[L];
    if (L == Lm - 1) offm1 = A.img.off[L];
  }
  // shared levels 0 .. ng - 1, their keys and state bytes
  const int ng = QX == 4 ? max(Lm - 1, 0) : Lm;
  uint32_t kk[MAXL];
  uint8_t st[MAXL];
  uint32_t key = (j >> Lm) * (uint32_t)N0 + (i >> Lm);
#pragma unroll
  for (int L = 0; L < MAXL; ++L) {
    kk[L] = 0;
    st[L] = 0;
    if (L < ng) {  // uniform
      if (L > 0) {
        const int sh = Lm - L;
        key = 4u * key + (((i >> sh) & 1u) | (((j >> sh) & 1u) << 1));
      }
      kk[L] = key;
      st[L] = state[A.img.off[L] + key];
    }
  }
  // QX = 4: the pairs' level-(Lm - 1) nodes (i0 = 4k, so pair h's bit along u is h)
  uint32_t kp[2] = {0u, 0u};
  uint8_t sp[2] = {0, 0};
  if (QX == 4 && Lm >= 1) {
    const uint32_t base = Lm >= 2 ? 4u * key + (((j >> 1) & 1u) << 1) : (j >> 1) * (uint32_t)N0 + (i >> 1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      kp[h] = base + (uint32_t)h;
      sp[h] = state[offm1 + kp[h]];
    }
  }
  int lf = ng;  // the shallowest shared level whose node is a leaf, ng if none
#pragma unroll
  for (int L = MAXL - 1; L >= 0; --L)
    if (L < ng && !(st[L] & AIR_NODE_REFINED)) lf = L;
  int64_t pg = 0;  // the shared leaf's position
#pragma unroll
  for (int L = 0; L < MAXL; ++L)
    if (L == lf) pg = A.img.off[L] + kk[L];
  int64_t p[QX];
#pragma unroll
  for (int q = 0; q < QX; ++q) {
    const uint32_t bits = ((i + q) & 1u) | ((j & 1u) << 1);
    if (lf < ng) {
      p[q] = pg;
    } else if (QX == 4 && Lm >= 1) {
      const int h = q >> 1;
      p[q] = (sp[h] & AIR_NODE_REFINED) ? offm + 4u * kp[h] + bits : offm1 + kp[h];
    } else {  // every level above the pixels refined, or Lm = 0 (then pixel q is key + q)
      p[q] = Lm > 0 ? offm + 4u * key + bits : offm + key + (uint32_t)q;
    }
    p[q] += vb;
  }
  float* img = images + (int64_t)v * (nb + 1) * R2 + e;
  // a write-once output: streaming stores keep it from evicting the field
  // and the maps from the caches
  typedef float f4 __attribute__((ext_vector_type(4)));
  // two planes per trip: their gathers are in flight together
  for (int b0 = 0; b0 <= nb; b0 += 2) {
    float x[2][QX];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int b = min(b0 + u, nb);
      const float* src = b < nb ? A.w.valI + b * VS : A.w.valN;
#pragma unroll
      for (int q = 0; q < QX; ++q) x[u][q] = src[p[q]];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (b0 + u > nb) break;
      float* dst = img + (int64_t)(b0 + u) * R2;
      if constexpr (QX >= 4) {
#pragma unroll
        for (int g = 0; g < QX; g += 4)
          __builtin_nontemporal_store(f4{x[u][g], x[u][g + 1], x[u][g + 2], x[u][g + 3]}, reinterpret_cast<f4*>(dst + g));
      } else {
        __builtin_nontemporal_store(x[u][0], dst);
      }
    }
  }
}

// Step vi's super-resolution option (reading: the cited interpolation is not
// given): each pixel of the finest raster, lying in a level-L leaf, takes the
// bilinear interpolation at its centre of the level-L point samples around
// it.  A sample is the level-L node's value where that node exists, else the
// value of the level-(L-1) node covering the position (which the 2:1 rule
// makes exist next to a leaf); positions beyond the image edge take the
// nearest edge position.  In level-L units a finest pixel x sits at
// u = (x + 1/2) / 2^(Lmax-L) - 1/2, exactly representable, so the weights are
// exact and a level-Lmax leaf gives its own value bit for bit.
__device__ __forceinline__ int64_t sample_pos(const MarchArgs& A, int64_t vb, int L, int i, int j) {
  const int RL = A.img.N0 << L;
  i = min(max(i, 0), RL - 1);
  j = min(max(j, 0), RL - 1);
  const uint32_t k = key_of((uint32_t)i, (uint32_t)j, L, A.img.N0);
  const int64_t p = vb + A.img.off[L] + k;
  if (L == 0 || (A.w.state[p] & AIR_NODE_EXIST)) return p;
  return vb + A.img.off[L - 1] + (k >> 2);
}

__global__ __launch_bounds__(256) void k_superres(MarchArgs A, float* images) {
  const int N0 = A.img.N0, Lm = A.img.Lmax, nb = A.f.nb;
  const uint32_t R = (uint32_t)N0 << Lm;
  const int64_t R2 = (int64_t)R * R, VS = (int64_t)A.img.V * A.img.S;
  const int64_t total = (int64_t)A.img.V * R2;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int v = (int)(e / R2);
    const int64_t q = e - (int64_t)v * R2;
    const uint32_t x = (uint32_t)(q % R), y = (uint32_t)(q / R);
    const int64_t vb = (int64_t)v * A.img.S;
    // the leaf holding the pixel
    uint32_t key = (y >> Lm) * (uint32_t)N0 + (x >> Lm);
    int L = 0;
    int64_t p = vb + key;
    while (L < Lm && (A.w.state[p] & AIR_NODE_REFINED)) {
      ++L;
      const int sh = Lm - L;
      key = 4u * key + (((x >> sh) & 1u) | (((y >> sh) & 1u) << 1));
      p = vb + A.img.off[L] + key;
    }
    const float inv_s = 1.0f / (float)(1u << (Lm - L));  // a power of two
    const float u = ((float)x + 0.5f) * inv_s - 0.5f, w = ((float)y + 0.5f) * inv_s - 0.5f;
    const float fi = floorf(u), fj = floorf(w);
    const float fu = u - fi, fv = w - fj;
    const int i0 = (int)fi, j0 = (int)fj;
    const int64_t pa = sample_pos(A, vb, L, i0, j0), pb = sample_pos(A, vb, L, i0 + 1, j0);
    const int64_t pc = sample_pos(A, vb, L, i0, j0 + 1), pd = sample_pos(A, vb, L, i0 + 1, j0 + 1);
    const float wa = (1.0f - fu) * (1.0f - fv), wb = fu * (1.0f - fv), wc = (1.0f - fu) * fv, wd = fu * fv;
    float* img = images + (int64_t)v * (nb + 1) * R2 + q;
    for (int b = 0; b <= nb; ++b) {
      const float* src = b < nb ? A.w.valI + b * VS : A.w.valN;
      const float val = wa * src[pa] + wb * src[pb] + wc * src[pc] + wd * src[pd];
      __builtin_nontemporal_store(val, img + b * R2);
    }
  }
}

template <int QX>
__host__ __device__ inline int64_t paint_blocks_per_view(const Img& img) {
  const int64_t R = (int64_t)img.N0 << img.Lmax;
  return (R * R / QX + 255) / 256;
}

// per chunk of CHUNK positions: existing nodes (for the scan), the tree
// counters, written per chunk (no global atomics), and, when flux_partial
// is given, the chunk's leaf flux per band (pixel area x I, float64, each
// thread's 16 positions in order, then a fixed tree).  Each thread reads its
// 16 consecutive state bytes with one load.
constexpr int PPT = CHUNK / 256;  // positions per thread
static_assert(PPT == 16, "one 16-byte state load per thread");

__device__ __forceinline__ uint4 state16(const uint8_t* st, int64_t p) {
  return *reinterpret_cast<const uint4*>(st + p);
}
__device__ __forceinline__ uint8_t byte_of(const uint4& q, int k) {
  const uint32_t w = k < 4 ? q.x : k < 8 ? q.y : k < 12 ? q.z : q.w;
  return (uint8_t)(w >> (8 * (k & 3)));
}

__device__ __forceinline__ double wave_sum_f64(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// QX > 0: the blocks after the n_chunks counting blocks paint the raster
// (paint_pixels<QX>), which does not depend on the counts
template <int QX>
__global__ __launch_bounds__(256) void k_count(MarchArgs A, unsigned long long* chunk_counts, unsigned* chunk_stats,
                                               int64_t n_chunks, double* flux_partial, float* images) {
  __shared__ unsigned sh[VS_N][4];
  __shared__ double shf[MAXB][4];
  const int64_t c = blockIdx.x;
  if constexpr (QX > 0) {
    if (c >= n_chunks) {  // uniform per block
      const int64_t pb = paint_blocks_per_view<QX>(A.img), k = c - n_chunks;
      paint_pixels<QX>(A, images, (int)(k / pb), k % pb);
      return;
    }
  }
  unsigned cnt[VS_N];
#pragma unroll
  for (int q = 0; q < VS_N; ++q) cnt[q] = 0;
  const ChunkPos cp = chunk_pos(A.img, c);
  const bool above0 = cp.L > 0;
  const int64_t p0 = c * CHUNK + threadIdx.x * PPT;
  const uint4 q4 = state16(A.w.state, p0);
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const uint8_t s = byte_of(q4, k);
    const bool spec = (s & ST_SPEC) != 0;
    if (s & AIR_NODE_EXIST) {
      ++cnt[VS_NODES];
      cnt[VS_LEAVES] += !(s & AIR_NODE_REFINED);
      cnt[VS_TESTED] += (s & AIR_NODE_EVALUATED) != 0;
      cnt[VS_FLAGGED] += (s & AIR_NODE_FLAGGED) != 0;
      cnt[VS_BALANCE] += (s & AIR_NODE_BALANCE) != 0;
      cnt[VS_MISSING] += above0 && !spec;
    } else {
      cnt[VS_WASTED] += spec;
    }
    cnt[VS_SPEC] += spec;
  }
  const int w = threadIdx.x / WAVE;
#pragma unroll
  for (int q = 0; q < VS_N; ++q) {
    unsigned x = cnt[q];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[q][w] = x;
  }
  const int nb = A.f.nb;
  if (flux_partial) {  // uniform
    const int64_t VS = (int64_t)A.img.V * A.img.S;
    const double px = A.views[cp.v].width / (double)((int64_t)A.img.N0 << cp.L), area = px * px;
    typedef float f4 __attribute__((ext_vector_type(4)));
    unsigned leaves = 0;  // bit k: position p0 + k is a leaf
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const uint8_t st = byte_of(q4, k);
      leaves |= ((st & AIR_NODE_EXIST) && !(st & AIR_NODE_REFINED)) ? 1u << k : 0u;
    }
    for (int b = 0; b < nb; ++b) {
      // a thread with leaves reads its 16 values in four 16-byte loads issued
      // together (every position of the chunk lies inside the maps), then
      // adds its leaves in position order
      f4 x[PPT / 4];
      if (leaves) {
        const f4* src = reinterpret_cast<const f4*>(A.w.valI + b * VS + p0);
#pragma unroll
        for (int u = 0; u < PPT / 4; ++u) x[u] = src[u];
      }
      double f = 0.0;
#pragma unroll
      for (int k = 0; k < PPT; ++k)
        if (leaves & (1u << k)) f += area * (double)x[k >> 2][k & 3];
      const double t = wave_sum_f64(f);
      if ((threadIdx.x & (WAVE - 1)) == 0) shf[b][w] = t;
    }
  }
  __syncthreads();
  if (threadIdx.x < VS_N) {
    const unsigned t = sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] + sh[threadIdx.x][3];
    chunk_stats[threadIdx.x * n_chunks + c] = t;
    if (threadIdx.x == VS_NODES) chunk_counts[c] = t;
  }
  if (flux_partial && threadIdx.x < nb)
    flux_partial[c * nb + threadIdx.x] =
        ((shf[threadIdx.x][0] + shf[threadIdx.x][1]) + shf[threadIdx.x][2]) + shf[threadIdx.x][3];
}

// exclusive scan of n counts by one block of 1024 threads: each thread sums
// a contiguous run (16 independent loads at a time), the 1024 run sums are
// scanned by wave prefix sums and the 16 wave totals, then each thread
// rewrites its run; the total lands in a[n]
__device__ __forceinline__ void scan_block(unsigned long long* a, int64_t n, unsigned long long* wsum) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = tid * per, e = min<int64_t>(b + per, n);
  unsigned long long s = 0;
  for (int64_t k0 = b; k0 < e; k0 += 16) {
    unsigned long long v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = k0 + k < e ? a[k0 + k] : 0ull;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
  }
  unsigned long long x = s;  // inclusive prefix inside the wave
  for (int o = 1; o < WAVE; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == WAVE - 1) wsum[w] = x;
  __syncthreads();
  unsigned long long before = 0, total = 0;
  for (int q = 0; q < 1024 / WAVE; ++q) {
    before += q < w ? wsum[q] : 0ull;
    total += wsum[q];
  }
  unsigned long long run = before + x - s;  // exclusive prefix of this run
  for (int64_t k0 = b; k0 < e; k0 += 16) {
    unsigned long long v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = k0 + k < e ? a[k0 + k] : 0ull;
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k0 + k < e) {
        a[k0 + k] = run;
        run += v[k];
      }
  }
  if (tid == 0) a[n] = total;
}

// The closing launch of a render, one role per block: block 0 scans the
// chunk counts (when the node list is built) and copies the device
// counters; blocks 1 .. V (Lmax+1) sum the counters of one (view, level)'s
// chunks (levels start on a chunk); the next V nb blocks sum one (view,
// band)'s flux partials (each thread a fixed stride, then a fixed tree).
// Everything goes to the result block res (device memory, or pinned host
// memory that the host reads once the stream has finished).
__global__ __launch_bounds__(1024) void k_finish(MarchArgs A, unsigned long long* chunk_counts, int64_t n_chunks,
                                                 int scan, const unsigned* chunk_stats, const double* flux_partial,
                                                 unsigned long long* res) {
  __shared__ unsigned long long wsum[1024 / WAVE];
  __shared__ unsigned long long sh[VS_N][1024 / WAVE];
  __shared__ double shd[1024];
  const int nL = A.img.Lmax + 1, V = A.img.V, nb = A.f.nb;
  const int role = blockIdx.x;
  if (role == 0) {
    for (int k = threadIdx.x; k < CTR_COUNT; k += 1024) res[k] = A.w.ctr[k];
    __threadfence_system();  // res may be host memory, read once the stream is done
    if (scan) scan_block(chunk_counts, n_chunks, wsum);
    return;
  }
  if (role <= V * nL) {
    const int v = (role - 1) / nL, L = (role - 1) % nL;
    const int64_t c0 = ((int64_t)v * A.img.S + A.img.off[L]) / CHUNK;
    const int64_t c1 = ((int64_t)v * A.img.S + A.img.off[L + 1]) / CHUNK;
    unsigned long long x[VS_N];
#pragma unroll
    for (int q = 0; q < VS_N; ++q) x[q] = 0;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += 1024)
#pragma unroll
      for (int q = 0; q < VS_N; ++q) x[q] += chunk_stats[q * n_chunks + c];
    const int w = threadIdx.x / WAVE;
#pragma unroll
    for (int q = 0; q < VS_N; ++q) {
      unsigned long long y = x[q];
      for (int o = 32; o > 0; o >>= 1) y += __shfl_xor(y, o);
      if ((threadIdx.x & (WAVE - 1)) == 0) sh[q][w] = y;
    }
    __syncthreads();
    if (threadIdx.x < VS_N) {
      unsigned long long t = 0;
      for (int k = 0; k < 1024 / WAVE; ++k) t += sh[threadIdx.x][k];
      res[res_vstat_off() + ((int64_t)v * MAXL + L) * VS_N + threadIdx.x] = t;
      __threadfence_system();
    }
    return;
  }
  const int fb = role - 1 - V * nL;  // (view, band)
  const int v = fb / nb, b = fb % nb;
  const int64_t cpv = n_chunks / V;
  double x = 0.0;
  for (int64_t c = threadIdx.x; c < cpv; c += 1024) x += flux_partial[((int64_t)v * cpv + c) * nb + b];
  shd[threadIdx.x] = x;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) shd[threadIdx.x] += shd[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    reinterpret_cast<double*>(res + res_flux_off(V))[fb] = shd[0];
    __threadfence_system();
  }
}

// node ids: exclusive prefix of existing positions in canonical order; also
// the compact list of the nodes' positions (node_pos[id])
__global__ __launch_bounds__(256) void k_emit(MarchArgs A, const unsigned long long* chunk_off, int32_t* id_map,
                                              uint64_t* node_pos) {
  __shared__ unsigned wsum[4];
  const int64_t c = blockIdx.x;
  if (chunk_off[c + 1] == chunk_off[c]) return;
  const int64_t p0 = c * CHUNK + threadIdx.x * PPT;
  const uint4 q4 = state16(A.w.state, p0);
  unsigned mine = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) mine += (byte_of(q4, k) & AIR_NODE_EXIST) ? 1u : 0u;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  unsigned x = mine;  // inclusive prefix in the wave
  for (int o = 1; o < WAVE; o <<= 1) {
    const unsigned y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == WAVE - 1) wsum[w] = x;
  __syncthreads();
  unsigned before = x - mine;
  for (int q = 0; q < w; ++q) before += wsum[q];
  unsigned long long id = chunk_off[c] + before;
#pragma unroll
  for (int k = 0; k < PPT; ++k)
    if (byte_of(q4, k) & AIR_NODE_EXIST) {
      id_map[p0 + k] = (int32_t)id;
      node_pos[id] = (uint64_t)(p0 + k);
      ++id;
    }
}

// one thread per node (grid-stride up to the total the scan left in
// chunk_off[n_chunks]): ids are consecutive, so every output array is
// written contiguously
__global__ __launch_bounds__(256) void k_write_tree(MarchArgs A, const unsigned long long* chunk_off, int64_t n_chunks,
                                                    const int32_t* id_map, const uint64_t* node_pos,
                                                    const TreeOut* outs) {
  // level offsets for per-thread levels (a kernel-argument read with a
  // per-thread index is a memory round trip)
  __shared__ int64_t s_off[MAXL + 1];
  if (threadIdx.x <= MAXL) s_off[threadIdx.x] = A.img.off[threadIdx.x];
  __syncthreads();
  const unsigned long long total = chunk_off[n_chunks];
  const int64_t S = A.img.S, VS = (int64_t)A.img.V * S, cpv = S / CHUNK;
  const int N0 = A.img.N0, nb = A.f.nb, Lm = A.img.Lmax;
  for (unsigned long long g = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; g < total;
       g += (unsigned long long)gridDim.x * blockDim.x) {
    const int64_t p = (int64_t)node_pos[g];
    const int v = (int)(p / S);
    const int64_t local = p - (int64_t)v * S;
    const int L = level_of(A.img, local);
    const uint32_t key = (uint32_t)(local - A.img.off[L]);
    // Everything this node writes is read first, in one round: the output
    // table entry and the node's values.  (The compiler cannot tell that
    // the outputs alias none of them, so a read placed after a store would
    // wait for the store's turn.)
    const TreeOut T = outs[v];
    const int64_t base = (int64_t)chunk_off[v * cpv];
    const int64_t vb = (int64_t)v * S;
    const uint8_t s = A.w.state[p];
    const int32_t par = L > 0 ? id_map[vb + s_off[L > 0 ? L - 1 : 0] + (key >> 2)] : 0;
    const int32_t fch = L < Lm ? id_map[vb + s_off[L < Lm ? L + 1 : L] + 4ll * key] : 0;
    float vI[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) vI[b] = b < nb ? A.w.valI[b * VS + p] : 0.0f;
    const float vN = A.w.valN[p], xI = A.w.xiI[p], xN = A.w.xiN[p];
    const int32_t vis = A.w.visits[p];
    const int64_t id = (int64_t)g - base;
    if (id >= T.capacity) continue;
    uint32_t i, j;
    coords_of(key, L, N0, i, j);
    // write-once outputs: streaming stores
    if (T.level) __builtin_nontemporal_store((int8_t)L, T.level + id);
    if (T.ix) __builtin_nontemporal_store((int32_t)i, T.ix + id);
    if (T.iy) __builtin_nontemporal_store((int32_t)j, T.iy + id);
    if (T.parent) __builtin_nontemporal_store(L == 0 ? -1 : (int32_t)(par - base), T.parent + id);
    if (T.first_child)
      __builtin_nontemporal_store((s & AIR_NODE_REFINED) ? (int32_t)(fch - base) : -1, T.first_child + id);
    if (T.state) __builtin_nontemporal_store((uint8_t)(s & (uint8_t)~(ST_TRACED | ST_SPEC)), T.state + id);
    if (T.I)
#pragma unroll
      for (int b = 0; b < MAXB; ++b)
        if (b < nb) __builtin_nontemporal_store(vI[b], T.I + b * T.capacity + id);
    if (T.N) __builtin_nontemporal_store(vN, T.N + id);
    const bool ev = (s & AIR_NODE_EVALUATED) != 0;
    if (T.xi_I) __builtin_nontemporal_store(ev ? xI : __builtin_nanf(""), T.xi_I + id);
    if (T.xi_N) __builtin_nontemporal_store(ev ? xN : __builtin_nanf(""), T.xi_N + id);
    if (T.visits) __builtin_nontemporal_store(vis, T.visits + id);
  }
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

__global__ __launch_bounds__(256) void k_fixed_final(const double* partial, int64_t chunks_per_plane,
                                                     double* flux) {
  __shared__ double sh[256];
  double x = 0.0;
  for (int64_t c = threadIdx.x; c < chunks_per_plane; c += 256) x += partial[(int64_t)blockIdx.x * chunks_per_plane + c];
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) flux[blockIdx.x] = sh[0];
}

}  // namespace

hipError_t launch_refine(const MarchArgs& a, int L, float xcI, float xcN, const float* w, int grid_blocks,
                         hipStream_t s) {
  BandW W;
  for (int b = 0; b < MAXB; ++b) W.w[b] = w[b];
  hipLaunchKernelGGL(k_refine, dim3(grid_blocks), dim3(RB), 0, s, a, L, xcI, xcN, W);
  return hipGetLastError();
}

hipError_t launch_count(const MarchArgs& a, unsigned long long* chunk_counts, unsigned* chunk_stats,
                        int64_t n_chunks, double* flux_partial, float* images, hipStream_t s) {
  const int64_t R = (int64_t)a.img.N0 << a.img.Lmax;
  if (!images) {
    hipLaunchKernelGGL(k_count<0>, dim3((unsigned)n_chunks), dim3(256), 0, s, a, chunk_counts, chunk_stats, n_chunks,
                       flux_partial, images);
  } else if (R % 4 == 0 && ((uintptr_t)images & 15) == 0) {
    // rows of a multiple of 4 pixels, 16-byte aligned planes: four pixels per thread
    const int64_t n = n_chunks + a.img.V * paint_blocks_per_view<4>(a.img);
    hipLaunchKernelGGL(k_count<4>, dim3((unsigned)n), dim3(256), 0, s, a, chunk_counts, chunk_stats, n_chunks,
                       flux_partial, images);
  } else {
    const int64_t n = n_chunks + a.img.V * paint_blocks_per_view<1>(a.img);
    hipLaunchKernelGGL(k_count<1>, dim3((unsigned)n), dim3(256), 0, s, a, chunk_counts, chunk_stats, n_chunks,
                       flux_partial, images);
  }
  return hipGetLastError();
}

hipError_t launch_finish(const MarchArgs& a, unsigned long long* chunk_counts, int64_t n_chunks, bool scan,
                         const unsigned* chunk_stats, const double* flux_partial, unsigned long long* res,
                         hipStream_t s) {
  const int blocks = 1 + a.img.V * (a.img.Lmax + 1) + (flux_partial ? a.img.V * a.f.nb : 0);
  hipLaunchKernelGGL(k_finish, dim3(blocks), dim3(1024), 0, s, a, chunk_counts, n_chunks, scan ? 1 : 0, chunk_stats,
                     flux_partial, res);
  return hipGetLastError();
}

hipError_t launch_emit(const MarchArgs& a, const unsigned long long* chunk_offsets, int64_t n_chunks,
                       int32_t* id_map, uint64_t* node_pos, hipStream_t s) {
  hipLaunchKernelGGL(k_emit, dim3((unsigned)n_chunks), dim3(256), 0, s, a, chunk_offsets, id_map, node_pos);
  return hipGetLastError();
}

hipError_t launch_write_tree(const MarchArgs& a, const unsigned long long* chunk_offsets, const int32_t* id_map,
                             const uint64_t* node_pos, const TreeOut* outs, int grid_blocks, hipStream_t s) {
  const int64_t n_chunks = (int64_t)a.img.V * a.img.S / CHUNK;
  hipLaunchKernelGGL(k_write_tree, dim3(grid_blocks), dim3(256), 0, s, a, chunk_offsets, n_chunks, id_map, node_pos,
                     outs);
  return hipGetLastError();
}

hipError_t launch_superres(const MarchArgs& a, float* images, hipStream_t s) {
  const int64_t R = (int64_t)a.img.N0 << a.img.Lmax, total = (int64_t)a.img.V * R * R;
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>((total + 255) / 256, 1), 65536);
  hipLaunchKernelGGL(k_superres, dim3((unsigned)blocks), dim3(256), 0, s, a, images);
  return hipGetLastError();
}

hipError_t launch_fixed_flux(const float* images, int V, int nb, int64_t R, double pix_area, double* partial,
                             double* flux_dev, hipStream_t s) {
  const int64_t R2 = R * R, cpp = (R2 + CHUNK - 1) / CHUNK;
  const int64_t n = (int64_t)V * nb * cpp;
  hipLaunchKernelGGL(k_fixed_partial, dim3((unsigned)n), dim3(256), 0, s, images, nb, R2, pix_area, cpp, partial);
  hipLaunchKernelGGL(k_fixed_final, dim3((unsigned)(V * nb)), dim3(256), 0, s, partial, cpp, flux_dev);
  return hipGetLastError();
}

}  // namespace air
