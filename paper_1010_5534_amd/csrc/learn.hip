// Learned depth proposal around plain AIR: the coarse feature maps, the
// cost-aware depth decision, the speculative work list and the depth labels
// of finished trees.  The network itself is in cnn.hip; the speculative
// march in march.hip.
#include <algorithm>

#include "air_common.h"

namespace air {

namespace {

// raw features of each coarse pixel, raster order [V][N0][N0][4]:
// log10(I_w + 1e-30), log10(N + 1e-30), finest grid level crossed (-1 for a
// miss), log10(rho_max / rho_min) along the ray (0 for a miss or rho_min 0)
__global__ __launch_bounds__(256) void k_features(MarchArgs A, LearnW W, float* feat) {
  const int N0 = A.img.N0, nb = A.f.nb;
  const int64_t n0sq = (int64_t)N0 * N0, total = (int64_t)A.img.V * n0sq, VS = (int64_t)A.img.V * A.img.S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = e / n0sq, key = e % n0sq;  // level 0: key = j * N0 + i
    const int64_t pos = v * A.img.S + key;
    float Iw = 0.0f;
    for (int b = 0; b < nb; ++b) Iw += W.w[b] * A.w.valI[b * VS + pos];
    const float N = A.w.valN[pos];
    const int lm = A.w.lmax0[e];
    const float rmin = A.w.rmin[e], rmax = A.w.rmax[e];
    float4 o;
    o.x = log10f(Iw + 1e-30f);
    o.y = log10f(N + 1e-30f);
    o.z = (float)lm;
    o.w = (lm >= 0 && rmin > 0.0f) ? log10f(rmax / rmin) : 0.0f;
    reinterpret_cast<float4*>(feat)[e] = o;
  }
}

__device__ __forceinline__ unsigned long long subtree_rays(int d) {
  unsigned long long s = 0, q = 1;
  for (int l = 1; l <= d; ++l) {
    q *= 4;
    s += q;
  }
  return s;
}

// depth per coarse pixel: argmin_d c_ray * rays(1..d) + c_sweep * P(depth > d)
__global__ __launch_bounds__(256) void k_decide(const float* z, int64_t total, int dmax, float c_ray, float c_sweep,
                                                uint8_t* depth, unsigned long long* counts) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const float* zp = z + e * LOGIT_STRIDE;
    float m = zp[0];
    for (int c = 1; c < DEPTH_CLASSES; ++c) m = fmaxf(m, zp[c]);
    float p[DEPTH_CLASSES], se = 0.0f;
    for (int c = 0; c < DEPTH_CLASSES; ++c) {
      p[c] = expf(zp[c] - m);
      se += p[c];
    }
    for (int c = 0; c < DEPTH_CLASSES; ++c) p[c] = p[c] / se;
    int best = 0;
    float best_cost = __builtin_huge_valf();
    for (int d = 0; d <= dmax; ++d) {
      float tail = 0.0f;
      for (int c = d + 1; c < DEPTH_CLASSES; ++c) tail += p[c];
      const float cost = c_ray * (float)subtree_rays(d) + c_sweep * tail;
      if (cost < best_cost) {
        best = d;
        best_cost = cost;
      }
    }
    depth[e] = (uint8_t)best;
    counts[e] = subtree_rays(best);
  }
}

// the speculative work list: one wave per coarse pixel writes the keys of its
// levels 1..d, level by level, each level's keys contiguous (Morton order)
__global__ __launch_bounds__(256) void k_spec_emit(const uint8_t* depth, const unsigned long long* offsets,
                                                   int64_t total, int64_t n0sq, uint64_t* spec) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; e < total; e += nw) {
    const int d = depth[e];
    const uint32_t v = (uint32_t)(e / n0sq), key0 = (uint32_t)(e % n0sq);
    unsigned long long at = offsets[e];
    uint32_t cnt = 1;
    for (int l = 1; l <= d; ++l) {
      cnt *= 4;
      for (uint32_t m = lane; m < cnt; m += WAVE) spec[at + m] = qentry(v, (uint32_t)l, (key0 << (2 * l)) + m);
      at += cnt;
    }
  }
}

// deepest level of a finished tree inside each coarse pixel
__global__ __launch_bounds__(256) void k_tree_depth(const int8_t* level, const int32_t* ix, const int32_t* iy,
                                                    int64_t n, int N0, int* depth) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int L = level[k];
    atomicMax(&depth[(int64_t)(iy[k] >> L) * N0 + (ix[k] >> L)], L);
  }
}

int grid_for(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096); }

}  // namespace

hipError_t launch_features(const MarchArgs& a, const LearnW& w, float* feat, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(grid_for((int64_t)a.img.V * a.img.N0 * a.img.N0)), dim3(256), 0, s, a, w, feat);
  return hipGetLastError();
}

hipError_t launch_decide(const float* logits, int64_t total, int dmax, float c_ray, float c_sweep, uint8_t* depth,
                         unsigned long long* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(grid_for(total)), dim3(256), 0, s, logits, total, dmax, c_ray, c_sweep, depth,
                     counts);
  return hipGetLastError();
}

hipError_t launch_spec_emit(const uint8_t* depth, const unsigned long long* offsets, int64_t total, int64_t n0sq,
                            uint64_t* spec, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((total + 3) / 4, 8192);  // 4 waves per block
  hipLaunchKernelGGL(k_spec_emit, dim3(std::max(blocks, 1)), dim3(256), 0, s, depth, offsets, total, n0sq, spec);
  return hipGetLastError();
}

hipError_t launch_tree_depth(const int8_t* level, const int32_t* ix, const int32_t* iy, int64_t n, int N0,
                             int* depth, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_depth, dim3(grid_for(n)), dim3(256), 0, s, level, ix, iy, n, N0, depth);
  return hipGetLastError();
}

}  // namespace air
