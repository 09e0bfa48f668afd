// Internal declarations of the depth-proposal network kernels (cnn.hip).
// Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace air {
namespace cnn {

constexpr int LAYERS = 4;
constexpr int FEAT = 4;     // input maps
constexpr int CLASSES = 6;  // depth 0..5
constexpr int HID = 32;
// channels of each layer's input and output (real counts)
constexpr int CIN[LAYERS] = {FEAT, HID, HID, HID};
constexpr int COUT[LAYERS] = {HID, HID, HID, CLASSES};
// stored channels of the bf16 tensors: the input maps and the logit
// gradients are padded to 8 (16-byte rows), hidden maps hold 32
constexpr int XC = 8;   // input maps
constexpr int ZC = 8;   // logits (float32) and their gradient (bf16)
// padded GEMM shapes: rows (output channels, a multiple of 16) and K = 9 *
// stored input channels rounded up to the MFMA depth of 32
constexpr int KPAD(int cin_stored) { return (9 * cin_stored + 31) / 32 * 32; }

// flat parameter offsets (weights [cout][3][3][cin] then bias [cout])
struct Offsets {
  int w[LAYERS], b[LAYERS], total;
};
__host__ __device__ inline Offsets offsets() {
  Offsets o{};
  int p = 0;
  for (int l = 0; l < LAYERS; ++l) {
    o.w[l] = p;
    p += COUT[l] * 9 * CIN[l];
    o.b[l] = p;
    p += COUT[l];
  }
  o.total = p;
  return o;
}

// device buffers of one network
struct Net {
  float* theta = nullptr;  // [P] float32 master parameters
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  float* grad = nullptr;   // [P]
  uint16_t* wf[LAYERS] = {};  // forward operand: [rows][KPAD(cin stored)] bf16
  uint16_t* wt[LAYERS] = {};  // input-gradient operand (layers 1..3): [32][KPAD(cout stored)]
  float mean[FEAT] = {0, 0, 0, 0}, stdv[FEAT] = {1, 1, 1, 1};
  int64_t step = 0;
  bool dirty = true;  // bf16 operands need rebuilding from theta
};

// rays of levels 1..d below one coarse pixel
__host__ __device__ inline unsigned long long subtree_rays(int d) {
  unsigned long long s = 0, q = 1;
  for (int l = 1; l <= d; ++l) {
    q *= 4;
    s += q;
  }
  return s;
}

// cost-aware depth choice from one pixel's six logits: argmin over d <= dmax
// of c_ray * rays(1..d) + c_sweep * P(depth > d), P the softmax; ties go to
// the shallower depth
__device__ inline int depth_choice(const float* z, int dmax, float c_ray, float c_sweep) {
  float m = z[0];
  for (int c = 1; c < CLASSES; ++c) m = fmaxf(m, z[c]);
  float p[CLASSES], se = 0.0f;
  for (int c = 0; c < CLASSES; ++c) {
    p[c] = expf(z[c] - m);
    se += p[c];
  }
  for (int c = 0; c < CLASSES; ++c) p[c] = p[c] / se;
  int best = 0;
  float best_cost = __builtin_huge_valf();
  for (int d = 0; d <= dmax; ++d) {
    float tail = 0.0f;
    for (int c = d + 1; c < CLASSES; ++c) tail += p[c];
    const float cost = c_ray * (float)subtree_rays(d) + c_sweep * tail;
    if (cost < best_cost) {
      best = d;
      best_cost = cost;
    }
  }
  return best;
}

// launchers; every pointer is device memory.  n = maps, h x w pixels each
hipError_t prep_weights(const Net& net, hipStream_t s);
hipError_t input_maps(const float* feat, int64_t P, const float* mean, const float* stdv, uint16_t* x, hipStream_t s);
// forward layer l: x (stored channels of its input) -> y (hidden: bf16
// after bias and ReLU; last: float32 logits + bias)
hipError_t conv_forward(int l, const Net& net, const uint16_t* x, int n, int h, int w, void* y, hipStream_t s);
// input gradient of layer l (1..3): dy -> dx masked by act > 0 (act = the
// layer's input activation), bf16
hipError_t conv_input_grad(int l, const Net& net, const uint16_t* dy, const uint16_t* act, int n, int h, int w,
                           uint16_t* dx, hipStream_t s);
// weight and bias gradient of layer l into net.grad (its slice), through
// per-block partials (partial must hold wgrad_partial_floats() floats)
hipError_t conv_weight_grad(int l, const Net& net, const uint16_t* dy, const uint16_t* x, int n, int h, int w,
                            float* partial, hipStream_t s);
size_t wgrad_partial_floats();
// loss: per-block partials, final reduction into out[0] = sum of weights,
// out[1] = weighted mean loss; then dz (bf16)
hipError_t loss_and_dz(const float* z, const int32_t* labels, int64_t P, const float* class_w, double* partial,
                       double* out, uint16_t* dz, hipStream_t s);
size_t loss_partial_doubles();
hipError_t adam(Net& net, int P, float lr, float beta1, float beta2, float eps, hipStream_t s);
// inference of all four layers on n maps of bf16 input rows x [n*h*w][8]
// (output tiles with their activations kept in LDS) followed by the depth
// choice: depth[p] per pixel, and spec_off[p], the start of pixel p's
// speculative rays in a work list whose length is counted in *spec_total
// (which must hold 0 before the launch; ranges are reserved per block, in
// no fixed order)
hipError_t infer_depth(const Net& net, const uint16_t* x, int n, int h, int w, int dmax, float c_ray, float c_sweep,
                       uint8_t* depth, unsigned long long* spec_off, unsigned long long* spec_total, hipStream_t s);

}  // namespace cnn
}  // namespace air
