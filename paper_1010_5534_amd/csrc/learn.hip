// Learned depth proposal around plain AIR: the coarse feature maps, the
// speculative work list and the depth labels of finished trees.  The network
// and the cost-aware depth choice are in cnn.hip; the speculative march in
// march.hip.
#include <algorithm>

#include "air_common.h"
#include "cnn.h"

namespace air {

namespace {

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);  // nearest, ties to even
  return (uint16_t)(u >> 16);
}

// raw features of each coarse pixel, raster order [V][N0][N0][4]:
// log10(I_w + 1e-30), log10(N + 1e-30), finest grid level crossed (-1 for a
// miss), log10(rho_max / rho_min) along the ray (0 for a miss or rho_min 0)
template <bool BF16>
__global__ __launch_bounds__(256) void k_features(MarchArgs A, LearnW W, float* feat, FeatNorm nm, uint16_t* x0) {
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
    if constexpr (BF16) {
      // the network's input row: standardised, bfloat16, channels 4..7 zero
      uint4 q;
      q.x = (uint32_t)to_bf16((o.x - nm.mean[0]) * nm.inv_std[0]) | ((uint32_t)to_bf16((o.y - nm.mean[1]) * nm.inv_std[1]) << 16);
      q.y = (uint32_t)to_bf16((o.z - nm.mean[2]) * nm.inv_std[2]) | ((uint32_t)to_bf16((o.w - nm.mean[3]) * nm.inv_std[3]) << 16);
      q.z = 0u;
      q.w = 0u;
      reinterpret_cast<uint4*>(x0)[e] = q;
    } else {
      reinterpret_cast<float4*>(feat)[e] = o;
    }
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

// a given speculation depth per coarse pixel (clamped to dmax): its depth
// byte and the start of its speculative rays in the work list, a block's
// range reserved with one atomic on the list's length (the order of the
// ranges changes no traced value)
__global__ __launch_bounds__(256) void k_spec_reserve(const uint8_t* given, int dmax, int64_t total, uint8_t* depth,
                                                      unsigned long long* off, unsigned long long* spec_total) {
  __shared__ unsigned long long wsum[4];
  __shared__ unsigned long long base;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < total; b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = b0 + threadIdx.x;
    int d = 0;
    if (e < total) d = min((int)given[e], dmax);
    const unsigned long long mine = e < total ? cnn::subtree_rays(d) : 0ull;
    unsigned long long x = mine;  // inclusive prefix in the wave
    for (int o = 1; o < WAVE; o <<= 1) {
      const unsigned long long y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) base = atomicAdd(spec_total, wsum[0] + wsum[1] + wsum[2] + wsum[3]);
    __syncthreads();
    unsigned long long before = base + x - mine;
    for (int q = 0; q < w; ++q) before += wsum[q];
    if (e < total) {
      depth[e] = (uint8_t)d;
      off[e] = before;
    }
    __syncthreads();  // wsum and base are rewritten by the next round
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
  hipLaunchKernelGGL(k_features<false>, dim3(grid_for((int64_t)a.img.V * a.img.N0 * a.img.N0)), dim3(256), 0, s, a, w,
                     feat, FeatNorm{}, nullptr);
  return hipGetLastError();
}

hipError_t launch_features_bf16(const MarchArgs& a, const LearnW& w, const FeatNorm& nm, uint16_t* x0, hipStream_t s) {
  hipLaunchKernelGGL(k_features<true>, dim3(grid_for((int64_t)a.img.V * a.img.N0 * a.img.N0)), dim3(256), 0, s, a, w,
                     nullptr, nm, x0);
  return hipGetLastError();
}

hipError_t launch_spec_emit(const uint8_t* depth, const unsigned long long* offsets, int64_t total, int64_t n0sq,
                            uint64_t* spec, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((total + 3) / 4, 8192);  // 4 waves per block
  hipLaunchKernelGGL(k_spec_emit, dim3(std::max(blocks, 1)), dim3(256), 0, s, depth, offsets, total, n0sq, spec);
  return hipGetLastError();
}

hipError_t launch_spec_reserve(const uint8_t* given, int dmax, int64_t total, uint8_t* depth,
                               unsigned long long* off, unsigned long long* spec_total, hipStream_t s) {
  hipLaunchKernelGGL(k_spec_reserve, dim3(grid_for(total)), dim3(256), 0, s, given, dmax, total, depth, off, spec_total);
  return hipGetLastError();
}

hipError_t launch_tree_depth(const int8_t* level, const int32_t* ix, const int32_t* iy, int64_t n, int N0,
                             int* depth, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_depth, dim3(grid_for(n)), dim3(256), 0, s, level, ix, iy, n, N0, depth);
  return hipGetLastError();
}

}  // namespace air
