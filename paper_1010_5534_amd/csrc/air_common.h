// Internal declarations shared by the HIP kernels and the host API of the
// AIR library.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/air.h"

namespace air {

constexpr int MAXL = AIR_MAX_LEVELS;
constexpr int MAXB = AIR_MAX_BANDS;
constexpr int WAVE = 64;
#ifndef AIR_MAX_SEG
#define AIR_MAX_SEG 8
#endif
constexpr int MAX_SEG = AIR_MAX_SEG;  // at most this many waves (sub-intervals) per ray tile

// node state bits beyond the public ones: set by the march once the node's
// values are written (the refinement test reads only traced values)
constexpr uint8_t ST_TRACED = 64u;
// set by the speculative march of the learned proposal: the node's values
// are already in the maps (it may never become a tree node)
constexpr uint8_t ST_SPEC = 128u;

// learned proposal: depth classes 0..5 and the float32 logit row stride
constexpr int DEPTH_CLASSES = 6;
constexpr int LOGIT_STRIDE = 8;

// view, precomputed on the host in double precision
struct DevView {
  double d[3], eu[3], ev[3], c[3];
  double inv_d[3];  // 1/d per axis (0 where d = 0)
  double width;
};

// grid geometry
struct Geo {
  int kind;
  int n[3];       // uniform: cells per axis; AMR: base blocks per axis
  double lo[3], hi[3];
  double h[3];    // uniform cell size; AMR: base block size
  double inv_h[3];
  int seg_shift;  // rays are traced by 2^seg_shift lanes (equal parameter sub-intervals)
  // block AMR: n = base blocks per axis, h = base cell size, bs = 2^bs_shift
  // cells per block edge, levels 0..max_level; the finest spacing hf and
  // cells per axis nf; max_blocks bounds the blocks one lane may visit
  int bs, bs_shift, max_level, n_blocks;
  int nf[3];
  double hf[3], inv_hf[3];
  int max_blocks;
  const int* bchild;
  const int* bcoord;
  const int* blevel;
};

// cell data
struct Fld {
  int kind, nb;
  const void* packed;  // bricked march layout (see air_field_pack)
  uint32_t packed_bytes;
  // one-band (rho, T) on a uniform grid: the same cells again as 8-byte
  // (rho, T) records, rt_off bytes into the packed buffer (0 bytes: none)
  uint32_t rt_bytes;
  int64_t rt_off;
  // block AMR: the leaf block of every finest-level block position, (id << 4)
  // | level, leaf_off bytes into the packed buffer (leaf_map 0: none, the
  // march descends the child table)
  int leaf_map;
  int64_t leaf_off;
  int bnx, bny, bnz;   // bricks per axis
  const float* rho;
  const float* emis;
  const float* kappa;
  const float* temp;
  float k0[MAXB], s[MAXB], q[MAXB];
  // band ladder: s_b = s0 + b ds and one q for every band (as in the power-law
  // band tables of the workloads): then T^-s_b = T^-s0 (T^-ds)^b and j is
  // shared, so a visit takes 5 transcendentals for its bands instead of 3 per
  // band; rk0[b] = 1 / k0[b]
  int ladder;
  float s0, ds, q0, rk0[MAXB];
};

// image pyramid layout: per view, levels 0..Lmax of dense maps indexed by
// the forest-Morton key (coarse pixel row-major, Morton inside it)
struct Img {
  int N0, Lmax, V;
  int64_t S;              // positions per view (padded)
  int64_t off[MAXL + 1];  // level offsets inside a view (multiples of 256)
  double min_width;       // narrowest view (launch-shape choices on the host)
};

// counters (uint64) in device memory
enum : int {
  CTR_CURSOR = 0,         // queue append cursor
  CTR_OVERFLOW = 1,       // set when an append would pass the capacity
  CTR_LSTART = 2,         // [MAXL + 2] queue start of each level
  CTR_SPEC = CTR_LSTART + MAXL + 2,  // length of the learned proposal's work list
  CTR_TILE = CTR_SPEC + 1,           // [MAXL + 1][8] march tile tickets per level and XCD
  // march statistics, spread over CTR_SLOTS addresses so that concurrent
  // blocks rarely add to the same word (same-address atomics serialise)
  CTR_HITS = CTR_TILE + 8 * (MAXL + 1),
  CTR_VISITS = CTR_HITS + 64,
  CTR_COUNT = CTR_VISITS + 64
};
constexpr int CTR_SLOTS = 64;
// per (view, level) counts; SPEC = speculatively traced positions, WASTED =
// those that are no tree node, MISSING = tree nodes below level 0 traced by
// the level loop instead
enum : int { VS_NODES = 0, VS_LEAVES, VS_TESTED, VS_FLAGGED, VS_BALANCE, VS_SPEC, VS_WASTED, VS_MISSING, VS_N };

struct Work {
  uint8_t* state;   // [V*S]
  float* valI;      // [nb][V*S]
  float* valN;      // [V*S]
  float* xiI;       // [V*S]
  float* xiN;       // [V*S]
  int* visits;      // [V*S]
  float* rmin;      // [V*N0*N0] level-0 density range (feature maps), may be null
  float* rmax;
  int* lmax0;       // [V*N0*N0] level-0 finest grid level crossed (with rmin)
  uint64_t* queue;  // work queue entries
  uint64_t qcap;
  int skip_spec;    // learned mode: the level march skips nodes with ST_SPEC
  unsigned long long* ctr;  // [CTR_COUNT]
  // split tiles: a queue launch of a level >= 1 that can hold at most
  // split_tiles tiles runs its sub-interval marches as separate wave jobs
  // with partials in parts ([tile][sub-interval][split_fields(NB)][64]
  // floats); 0 = never
  float* parts;
  int64_t split_tiles;
};
// fields of one split job's partial record: I[NB], tau[NB], N, rmin, rmax,
// cells walked, finest level, uniform-grid cell count, hit
__host__ __device__ constexpr int split_fields(int nb) { return 2 * nb + 7; }
// the march's band count for a field (1 for one-band records, else 2, 4, 8)
__host__ __device__ inline int march_nb(int kind, int nb) {
  return (kind == AIR_FIELD_RHO_J_KAPPA || nb == 1) ? 1 : nb <= 2 ? 2 : nb <= 4 ? 4 : 8;
}

// ------------------------------------------------------------ Morton keys
__host__ __device__ inline uint32_t spread2(uint32_t x) {
  x &= 0x0000ffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}
__host__ __device__ inline uint32_t squeeze2(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return x;
}
// key of pixel (i, j) at level L: coarse pixel index, then Morton code of
// the position inside it (i in even bits, j in odd bits).  The parent of key
// k is k >> 2 and its children are 4k..4k+3.
__host__ __device__ inline uint32_t key_of(uint32_t i, uint32_t j, int L, int N0) {
  uint32_t mask = (1u << L) - 1u;
  uint32_t root = (j >> L) * (uint32_t)N0 + (i >> L);
  return (root << (2 * L)) | spread2(i & mask) | (spread2(j & mask) << 1);
}
__host__ __device__ inline void coords_of(uint32_t key, int L, int N0, uint32_t& i, uint32_t& j) {
  uint32_t root = key >> (2 * L);
  uint32_t m = key & ((1u << (2 * L)) - 1u);
  i = ((root % (uint32_t)N0) << L) | squeeze2(m);
  j = ((root / (uint32_t)N0) << L) | squeeze2(m >> 1);
}

// queue entry: view (24 bits) | level (8) | key (32)
__host__ __device__ inline uint64_t qentry(uint32_t v, uint32_t L, uint32_t key) {
  return ((uint64_t)v << 40) | ((uint64_t)L << 32) | key;
}
__host__ __device__ inline void qdecode(uint64_t e, uint32_t& v, uint32_t& L, uint32_t& key) {
  key = (uint32_t)e;
  L = (uint32_t)(e >> 32) & 0xffu;
  v = (uint32_t)(e >> 40);
}

// ------------------------------------------------------------- launches
// kernels are defined in march.hip and tree.hip; the host API calls these
struct MarchArgs {
  Geo g;
  Fld f;
  Img img;
  Work w;
  const DevView* views;
};

hipError_t launch_init(const MarchArgs& a, hipStream_t s);
hipError_t launch_pack(const Geo& g, const Fld& f, void* packed, hipStream_t s);
hipError_t launch_pack_amr(const Geo& g, const Fld& f, void* packed, hipStream_t s);
hipError_t launch_leaf_map(const Geo& g, const Fld& f, void* packed, hipStream_t s);
// bytes of one packed cell record: (rho, j, kappa, 1/kappa) for RHO_J_KAPPA and
// for one-band RHO_T (j, kappa evaluated once when packing), (rho, T) otherwise
inline int packed_cell_bytes(int field_kind, int n_bands) {
  return (field_kind == AIR_FIELD_RHO_J_KAPPA || n_bands == 1) ? 16 : 8;
}

// packed index of cell (x, y, z): 2x2x2 bricks, x fastest
__host__ __device__ inline int brick_index(int x, int y, int z, int bnx, int bny) {
  return ((((z >> 1) * bny + (y >> 1)) * bnx + (x >> 1)) << 3) | (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
}
hipError_t launch_march_queue(const MarchArgs& a, int L, int grid_blocks, hipStream_t s);
// whether launch_march_queue runs level L as split tiles, and the tiles a
// queue launch of level L can hold; whether its rays lie a cell or more apart
bool split_level(const MarchArgs& a, int L);
int64_t queue_tile_bound(const MarchArgs& a, int L);
bool coarse_level(const MarchArgs& a, int L);
// speculative march of the learned proposal: the n = *count entries of spec
hipError_t launch_march_spec(const MarchArgs& a, const uint64_t* spec, const unsigned long long* count,
                             int grid_blocks, hipStream_t s);
struct LearnW {
  float w[MAXB];
};
// launch shapes that do not change results: waves per CU of the march grids,
// blocks per CU of the refinement test
struct Tune {
  int march_waves_per_cu = 16;
  int refine_blocks_per_cu = 4;
};
hipError_t launch_features(const MarchArgs& a, const LearnW& w, float* feat, hipStream_t s);
// the same maps standardised ((x - mean) * inv_std) and rounded to bf16
// straight into the network's input rows [V*N0*N0][8]
struct FeatNorm {
  float mean[4], inv_std[4];
};
hipError_t launch_features_bf16(const MarchArgs& a, const LearnW& w, const FeatNorm& nm, uint16_t* x0, hipStream_t s);
hipError_t launch_spec_emit(const uint8_t* depth, const unsigned long long* offsets, int64_t total, int64_t n0sq,
                            uint64_t* spec, hipStream_t s);
// a given speculation depth per coarse pixel instead of the network's choice:
// depth bytes, per-pixel work-list offsets and the list length (*spec_total
// must hold 0 before the launch)
hipError_t launch_spec_reserve(const uint8_t* given, int dmax, int64_t total, uint8_t* depth,
                               unsigned long long* off, unsigned long long* spec_total, hipStream_t s);
hipError_t launch_tree_depth(const int8_t* level, const int32_t* ix, const int32_t* iy, int64_t n, int N0,
                             int* depth, hipStream_t s);
hipError_t launch_refine(const MarchArgs& a, int L, float xcI, float xcN, const float* w, int grid_blocks,
                         hipStream_t s);
hipError_t launch_march_fixed(const MarchArgs& a, int level, float* images, int grid_blocks, hipStream_t s);
hipError_t launch_trace_pixels(const MarchArgs& a, int64_t n, const int32_t* level, const int32_t* ix,
                               const int32_t* iy, float* I, float* N, int32_t* visits, hipStream_t s);
// per chunk: existing nodes (chunk_counts), the other counters
// (chunk_stats[VS_N][n_chunks]) and, if flux_partial is not null, the leaf
// flux per band (flux_partial[n_chunks][nb]); in the same launch, if images
// is not null, the raster [V][nb + 1][R][R] painted from the leaves
hipError_t launch_count(const MarchArgs& a, unsigned long long* chunk_counts, unsigned* chunk_stats,
                        int64_t n_chunks, double* flux_partial, float* images, hipStream_t s);
// The result block of a render, copied to the host in one piece:
// [0, CTR_COUNT) the device counters, then the per (view, level) counters
// [V][MAXL][VS_N], then the flux [V][nb] (float64).  res_words gives its
// size in 8-byte words.
__host__ __device__ inline int64_t res_vstat_off() { return CTR_COUNT; }
__host__ __device__ inline int64_t res_flux_off(int V) { return CTR_COUNT + (int64_t)V * MAXL * VS_N; }
__host__ __device__ inline int64_t res_words(int V, int nb) { return res_flux_off(V) + (int64_t)V * nb; }
// after the count, in one launch: the exclusive scan of chunk_counts (if
// scan), the counter copy, the (view, level) sums and (if flux_partial) the
// flux of each (view, band), all into res
hipError_t launch_finish(const MarchArgs& a, unsigned long long* chunk_counts, int64_t n_chunks, bool scan,
                         const unsigned* chunk_stats, const double* flux_partial, unsigned long long* res,
                         hipStream_t s);
hipError_t launch_emit(const MarchArgs& a, const unsigned long long* chunk_offsets, int64_t n_chunks,
                       int32_t* id_map, uint64_t* node_pos, hipStream_t s);
struct TreeOut {
  int8_t* level;
  int32_t* ix;
  int32_t* iy;
  int32_t* parent;
  int32_t* first_child;
  uint8_t* state;
  float* I;
  float* N;
  float* xi_I;
  float* xi_N;
  int32_t* visits;
  int64_t capacity;
};
hipError_t launch_write_tree(const MarchArgs& a, const unsigned long long* chunk_offsets, const int32_t* id_map,
                             const uint64_t* node_pos, const TreeOut* outs, int grid_blocks, hipStream_t s);
// per-pixel spectra (spectra.hip): the bin table on the device, the store of
// traced spectra by work-queue position and the map from level-map position
// to queue position
struct SpecArgs {
  int nbins, stride;     // bins; row stride of the table (floats)
  const float* tab;      // [6][stride]: k0, -s, q, -E log2(e), e0, broadband weight
  float* store;          // [cap][nbins]
  unsigned long long cap;
  uint32_t* qpos;        // [V*S]
  unsigned* overflow;    // set when a ray's queue position lies past the store
};
// spectra in canonical node order: view v's rows start at row0[v], at most
// cap[v] of them (device arrays [V])
struct SpecOut {
  float* spectra;
  const int64_t* row0;
  const int64_t* cap;
};
constexpr int SPEC_CHUNK = 256;  // canonical nodes per partial sum of the image's spectrum
hipError_t launch_march_spectra(const MarchArgs& a, const SpecArgs& s, int L, int grid_blocks, hipStream_t st);
hipError_t launch_spectra_out(const MarchArgs& a, const SpecArgs& s, const unsigned long long* chunk_off,
                              int64_t n_chunks, const uint64_t* node_pos, const SpecOut& o, int64_t chunks_per_view,
                              double* partial, double* flux_dev, int grid_blocks, hipStream_t st);
// the interpolated raster of the finished tree (step vi super-resolution)
// into images [V][nb + 1][R][R]
hipError_t launch_superres(const MarchArgs& a, float* images, hipStream_t s);
hipError_t launch_fixed_flux(const float* images, int V, int nb, int64_t R, double pix_area, double* partial,
                             double* flux_dev, hipStream_t s);

constexpr int64_t CHUNK = 4096;  // positions per block in counting passes; levels start on a chunk

// allocation-free fixed render: layout of its static device workspace
// (counters, then the view table, then the flux partial sums)
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)AIR_NOALLOC_SCRATCH_BYTES;
constexpr size_t NOALLOC_CTR_OFF = 0;
constexpr size_t NOALLOC_VIEWS_OFF = 2048;
constexpr size_t NOALLOC_PARTIAL_OFF = 4096;
static_assert(sizeof(unsigned long long) * CTR_COUNT <= NOALLOC_VIEWS_OFF, "counters overlap the view table");
static_assert(NOALLOC_VIEWS_OFF + sizeof(DevView) * AIR_NOALLOC_MAX_VIEWS <= NOALLOC_PARTIAL_OFF,
              "view table overlaps the partial sums");
// the per-device address of the workspace (hipGetSymbolAddress once per
// device, with that device current), and the launch that clears its counters
// and writes the view table
hipError_t noalloc_init(int device, void** out);
hipError_t launch_noalloc_setup(const DevView* views, int n, void* scratch_ptr, hipStream_t s);

}  // namespace air
