// Host side of the AIR C ABI: argument validation, device workspace, and the
// level-synchronous launch sequence (section 2 steps i-vi).  All device work
// of one call is enqueued on the caller's stream; the host waits once, at
// the end, to return counts and fluxes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cstring>
#include <string>
#include <map>
#include <vector>

#include "air_common.h"
#include "cnn.h"

using namespace air;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct air_cnn {
  int device = 0;
  air::cnn::Net net;
};

// block tables checked when a field was packed on this context, with the
// packed buffer they went into: later calls that pass that packed field and
// the same tables skip the read-back
struct BlockSig {
  const void* packed;
  const void* lev;
  const void* crd;
  const void* chd;
  int n_blocks, n0, n1, n2, bs, max_level;
  bool operator==(const BlockSig& o) const {
    return packed == o.packed && lev == o.lev && crd == o.crd && chd == o.chd && n_blocks == o.n_blocks &&
           n0 == o.n0 && n1 == o.n1 && n2 == o.n2 && bs == o.bs && max_level == o.max_level;
  }
};

struct air_ctx {
  int device = 0;
  std::vector<BlockSig> checked;
  void* noalloc = nullptr;  // this device's static workspace of air_render_fixed_noalloc
  int num_cus = 256;
  int seg_shift_override = -1;  // AIR_SEG_SHIFT: tuning knob for the lanes per ray
  int64_t split_tiles = 4096;   // AIR_SPLIT_TILES: queue launches (levels >= 1) of at most this many tiles run split
  Tune eager;                   // launch shapes of air_render (AIR_MARCH_WAVES: march waves per CU)
  std::string err;
  DevBuf state, valI, valN, xiI, xiN, visits, rmin, rmax, queue, ctr, chunk, cstat, idmap, partial, flux, parts,
      views, touts, pack;
  // learned proposal: coarse maps, network activations and gradients, depth
  // choice and speculative work list
  // per-pixel spectra: bin table, spectra by queue position, queue position
  // per map position, per-view output rows, overflow flag, partial sums and
  // the image spectra
  DevBuf spec_tab, spec_store, spec_qpos, spec_rows, spec_flag, spec_part, spec_flux;
  void* host_spec = nullptr;  // pinned: overflow flag, then the image spectra
  size_t host_spec_n = 0;
  DevBuf nodepos, lmax0, feat, cx0, ca1, ca2, ca3, cz, cdz, cda, cdb, cdc, cwpart, closs_part, closs, depth8, scount,
      spec;
  // pixels of the last air_cnn_forward / air_cnn_loss_grad call whose
  // intermediates the network buffers hold (-1: none), and whether that call
  // computed gradients (air_cnn_tensor)
  int64_t cnn_pixels = -1;
  bool cnn_grads = false;
  unsigned long long* host_ctr = nullptr;  // pinned
  double* host_flux = nullptr;             // pinned
  unsigned long long* host_vstat = nullptr;
  size_t host_vstat_n = 0;
  size_t host_flux_n = 0;
  void* stage = nullptr;  // pinned staging of the view table (holds the last upload)
  size_t stage_n = 0;
  void* stage2 = nullptr;  // pinned staging of the tree output table (likewise)
  size_t stage2_n = 0;
  // what the device copies of the two tables hold (an identical table is
  // not sent again; every render ends with a stream sync, so no copy from
  // the staging buffers is in flight when they are compared or rewritten)
  const void* views_at = nullptr;  // device buffer (address and capacity) and bytes sent
  size_t views_cap = 0, views_bytes = 0;
  const void* touts_at = nullptr;
  size_t touts_cap = 0, touts_bytes = 0;
  // air_render_batch: the captured launch sequence of the last call and the
  // launch shapes chosen per workload shape
  std::string graph_key;
  // bumped whenever a context buffer is (re)allocated: captured launches hold
  // the buffers' addresses, so a graph is replayed only while it is unchanged
  uint64_t buf_gen = 0;
  hipStream_t cap_stream = nullptr;  // the graph is captured and replayed here
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  std::map<std::string, air::Tune> tuned;
  // timing events: [0] start, [1] end, then a pair around every march and
  // every test launch
  static constexpr int EV_FEAT0 = 2 + 4 * AIR_MAX_LEVELS, EV_SPEC0 = EV_FEAT0 + 1, EV_SPEC1 = EV_FEAT0 + 2;
  static constexpr int NEV = EV_FEAT0 + 3;
  hipEvent_t ev[NEV] = {};
};

namespace {

air_status fail(air_ctx* c, air_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(ctx, expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, AIR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// a render's final wait: poll the stream for up to 2 ms (a blocking
// synchronize may put the thread to sleep and wake it late, which shows on
// sub-millisecond calls), then block for longer ones
hipError_t spin_stream(hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e;
  while ((e = hipStreamQuery(s)) == hipErrorNotReady)
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) return hipStreamSynchronize(s);
  return e;
}

air_status ensure(air_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return AIR_OK;
  if (c) ++c->buf_gen;
  if (b.p) {
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 8;  // slack so slightly larger calls do not reallocate
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(c, AIR_ENOMEM, "device allocation of %zu bytes failed", want);
  }
  b.bytes = want;
  return AIR_OK;
}

air_status ensure_host(air_ctx* c, void** p, size_t* have, size_t bytes) {
  if (*have >= bytes && *p) return AIR_OK;
  if (c) ++c->buf_gen;
  // kernels and copies read and write these buffers asynchronously (a call
  // that failed after enqueueing did not wait for them): drain the device
  // before the old buffer goes
  if (*p) {
    (void)hipDeviceSynchronize();
    (void)hipHostFree(*p);
  }
  *p = nullptr;
  if (hipHostMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(c, AIR_ENOMEM, "pinned host allocation of %zu bytes failed", bytes);
  }
  *have = bytes;
  return AIR_OK;
}

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

air_status check_grid(air_ctx* c, const air_grid* g) {
  if (!g) return fail(c, AIR_EINVAL, "grid is NULL");
  if (g->kind != AIR_GRID_UNIFORM && g->kind != AIR_GRID_BLOCK_AMR)
    return fail(c, AIR_EINVAL, "grid kind %d unknown", g->kind);
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] < 1 || g->n[a] > (1 << 20)) return fail(c, AIR_EINVAL, "grid n[%d] = %d out of range", a, g->n[a]);
    if (!std::isfinite(g->lo[a]) || !std::isfinite(g->hi[a]) || !(g->hi[a] > g->lo[a]))
      return fail(c, AIR_EINVAL, "grid box on axis %d is empty or not finite", a);
  }
  if (g->kind == AIR_GRID_UNIFORM) {
    if ((int64_t)g->n[0] * g->n[1] * g->n[2] >= ((int64_t)1 << 30))
      return fail(c, AIR_EINVAL, "grid has 2^30 cells or more (field arrays must stay below 4 GiB)");
    return AIR_OK;
  }
  if (g->bs < 2 || g->bs > 32 || (g->bs & (g->bs - 1)))
    return fail(c, AIR_EINVAL, "block size %d is not a power of two in 2..32", g->bs);
  if (g->max_level < 0 || g->max_level > 20) return fail(c, AIR_EINVAL, "max_level %d out of range 0..20", g->max_level);
  for (int a = 0; a < 3; ++a)
    if (((int64_t)g->n[a] * g->bs << g->max_level) >= ((int64_t)1 << 30))
      return fail(c, AIR_EINVAL, "finest cells on axis %d reach 2^30", a);
  const int64_t base = (int64_t)g->n[0] * g->n[1] * g->n[2];
  if (g->n_blocks < base) return fail(c, AIR_EINVAL, "n_blocks %d below the %lld base blocks", g->n_blocks, (long long)base);
  if ((int64_t)g->n_blocks * g->bs * g->bs * g->bs >= ((int64_t)1 << 30))
    return fail(c, AIR_EINVAL, "grid has 2^30 cells or more (field arrays must stay below 4 GiB)");
  if (!g->block_level || !g->block_coord || !g->block_child) return fail(c, AIR_EINVAL, "block tables are NULL");
  return AIR_OK;
}

BlockSig sig_of(const air_grid* g, const void* packed) {
  return BlockSig{packed, g->block_level, g->block_coord, g->block_child, g->n_blocks, g->n[0], g->n[1], g->n[2],
                  g->bs, g->max_level};
}

// tables checked for this packed field by air_field_pack on this context
bool blocks_known(const air_ctx* c, const air_grid* g, const void* packed) {
  if (!packed) return false;
  const BlockSig k = sig_of(g, packed);
  for (const BlockSig& b : c->checked)
    if (b == k) return true;
  return false;
}

// The block tables are device data: read them back (on the caller's stream,
// so pending writes land first) and check that they describe one hierarchy,
// so the march's descent stays inside the tables.  Tables checked when the
// field passed in `packed` was packed on this context are not read again.
air_status check_blocks(air_ctx* c, const air_grid* g, hipStream_t s, const void* packed = nullptr) {
  if (g->kind != AIR_GRID_BLOCK_AMR) return AIR_OK;
  if (blocks_known(c, g, packed)) return AIR_OK;
  const int nb = g->n_blocks;
  std::vector<int32_t> lev(nb), crd(3 * (size_t)nb), chd(nb);
  HIPCHK(c, hipMemcpyAsync(lev.data(), g->block_level, 4 * (size_t)nb, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(crd.data(), g->block_coord, 12 * (size_t)nb, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(chd.data(), g->block_child, 4 * (size_t)nb, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const int64_t base = (int64_t)g->n[0] * g->n[1] * g->n[2];
  std::vector<uint8_t> owned(nb, 0);
  for (int64_t b = 0; b < nb; ++b) {
    if (b < base) {
      const int64_t want[3] = {b % g->n[0], (b / g->n[0]) % g->n[1], b / ((int64_t)g->n[0] * g->n[1])};
      if (lev[b] != 0 || crd[3 * b] != want[0] || crd[3 * b + 1] != want[1] || crd[3 * b + 2] != want[2])
        return fail(c, AIR_EINVAL, "base block %lld must have level 0 and coordinate (%lld, %lld, %lld)",
                    (long long)b, (long long)want[0], (long long)want[1], (long long)want[2]);
    } else if (!owned[b]) {
      return fail(c, AIR_EINVAL, "block %lld is nobody's child (children follow their parent)", (long long)b);
    }
    const int ch = chd[b];
    if (ch < 0) continue;
    if (lev[b] >= g->max_level) return fail(c, AIR_EINVAL, "block %lld at level %d has children", (long long)b, lev[b]);
    if (ch <= b || (int64_t)ch + 8 > nb)
      return fail(c, AIR_EINVAL, "block %lld: children %d..%d not after it inside the table", (long long)b, ch, ch + 7);
    for (int k = 0; k < 8; ++k) {
      const int64_t q = ch + k;
      if (owned[q]) return fail(c, AIR_EINVAL, "block %lld has two parents", (long long)q);
      owned[q] = 1;
      if (lev[q] != lev[b] + 1) return fail(c, AIR_EINVAL, "block %lld: level is not its parent's + 1", (long long)q);
      for (int a = 0; a < 3; ++a)
        if (crd[3 * q + a] != 2 * crd[3 * b + a] + ((k >> a) & 1))
          return fail(c, AIR_EINVAL, "block %lld: coordinate does not follow child offset %d", (long long)q, k);
    }
  }
  return AIR_OK;
}

air_status check_field(air_ctx* c, const air_field* f) {
  if (!f) return fail(c, AIR_EINVAL, "field is NULL");
  if (!f->rho) return fail(c, AIR_EINVAL, "field rho is NULL");
  if (f->kind == AIR_FIELD_RHO_J_KAPPA) {
    if (f->n_bands != 1) return fail(c, AIR_EINVAL, "a rho/j/kappa field has exactly one band");
    if (!f->emis || !f->kappa) return fail(c, AIR_EINVAL, "field emis/kappa is NULL");
  } else if (f->kind == AIR_FIELD_RHO_T) {
    if (f->n_bands < 1 || f->n_bands > AIR_MAX_BANDS)
      return fail(c, AIR_EINVAL, "n_bands %d out of range 1..%d", f->n_bands, AIR_MAX_BANDS);
    if (!f->temp) return fail(c, AIR_EINVAL, "field temp is NULL");
    for (int b = 0; b < f->n_bands; ++b)
      if (!finite3(f->band[b])) return fail(c, AIR_EINVAL, "band %d parameters not finite", b);
  } else {
    return fail(c, AIR_EINVAL, "field kind %d unknown", f->kind);
  }
  return AIR_OK;
}

air_status make_view(air_ctx* c, const air_view* v, DevView& out) {
  if (!finite3(v->dir) || !finite3(v->up) || !finite3(v->center) || !std::isfinite(v->width) || !(v->width > 0))
    return fail(c, AIR_EINVAL, "view has a non-finite value or width <= 0");
  double nd = std::sqrt(v->dir[0] * v->dir[0] + v->dir[1] * v->dir[1] + v->dir[2] * v->dir[2]);
  if (!(nd > 0)) return fail(c, AIR_EINVAL, "view direction is zero");
  for (int a = 0; a < 3; ++a) out.d[a] = v->dir[a] / nd;
  const double* u = v->up;
  const double* d = out.d;
  double x[3] = {u[1] * d[2] - u[2] * d[1], u[2] * d[0] - u[0] * d[2], u[0] * d[1] - u[1] * d[0]};
  double nx = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  double nu = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  if (!(nx > 1e-12 * nu)) return fail(c, AIR_EINVAL, "view up vector is zero or parallel to dir");
  for (int a = 0; a < 3; ++a) out.eu[a] = x[a] / nx;
  out.ev[0] = d[1] * out.eu[2] - d[2] * out.eu[1];
  out.ev[1] = d[2] * out.eu[0] - d[0] * out.eu[2];
  out.ev[2] = d[0] * out.eu[1] - d[1] * out.eu[0];
  for (int a = 0; a < 3; ++a) {
    out.c[a] = v->center[a];
    out.inv_d[a] = out.d[a] != 0.0 ? 1.0 / out.d[a] : 0.0;
  }
  out.width = v->width;
  return AIR_OK;
}

void fill_geo(const air_grid* g, Geo& G) {
  std::memset(&G, 0, sizeof G);
  G.kind = g->kind;
  const bool amr = g->kind == AIR_GRID_BLOCK_AMR;
  const int cells_per_n = amr ? g->bs : 1;
  for (int a = 0; a < 3; ++a) {
    G.n[a] = g->n[a];
    G.lo[a] = g->lo[a];
    G.hi[a] = g->hi[a];
    G.h[a] = (g->hi[a] - g->lo[a]) / ((double)g->n[a] * cells_per_n);
    G.inv_h[a] = ((double)g->n[a] * cells_per_n) / (g->hi[a] - g->lo[a]);
  }
  // lanes per ray: about 32 cells of the longest axis per lane, up to
  // MAX_SEG; fixed by the grid alone so every path traces a ray identically.
  // A block-AMR grid counts a quarter of its finest-level cells along the
  // axis (at least its base cells): deeply refined hierarchies get more
  // lanes per ray, whose cell chains are otherwise long at the fine levels
  // (measured on the section-3 ring, 4 levels, and the 2-level two-wind
  // hierarchy with 64 views x 8 bands, both faster than with twice the base
  // cells).
  int nmax = std::max(g->n[0], std::max(g->n[1], g->n[2])) * cells_per_n;
  if (amr && g->max_level > 0) nmax = std::max(nmax, (int)(((int64_t)nmax << g->max_level) / 4));
  int sh = 0;
  while ((1 << sh) < MAX_SEG && (32 << sh) < nmax) ++sh;
  G.seg_shift = sh;
  if (!amr) return;
  G.bs = g->bs;
  while ((1 << G.bs_shift) < g->bs) ++G.bs_shift;
  G.max_level = g->max_level;
  G.n_blocks = g->n_blocks;
  int64_t blocks_fine = 0;
  for (int a = 0; a < 3; ++a) {
    G.nf[a] = (g->n[a] * g->bs) << g->max_level;
    G.hf[a] = (g->hi[a] - g->lo[a]) / (double)G.nf[a];
    G.inv_hf[a] = (double)G.nf[a] / (g->hi[a] - g->lo[a]);
    blocks_fine += (int64_t)g->n[a] << g->max_level;
  }
  // a ray meets at most one block per finest block plane crossed, plus the
  // steps over block corners
  G.max_blocks = (int)std::min<int64_t>(2 * blocks_fine + 64, 1 << 30);
  G.bchild = g->block_child;
  G.bcoord = g->block_coord;
  G.blevel = g->block_level;
}

int64_t cells_of(const air_grid* g) {
  if (g->kind == AIR_GRID_BLOCK_AMR) return (int64_t)g->n_blocks * g->bs * g->bs * g->bs;
  return (int64_t)g->n[0] * g->n[1] * g->n[2];
}

// both layouts are whole 2x2x2 bricks: the uniform grid rounds each axis up
// to even, a block of bs^3 cells (bs even) is bs^3/8 bricks
int64_t packed_main_bytes(const air_grid* g, const air_field* f) {
  if (g->kind == AIR_GRID_BLOCK_AMR) return cells_of(g) * packed_cell_bytes(f->kind, f->n_bands);
  const int64_t bricks = (int64_t)((g->n[0] + 1) / 2) * ((g->n[1] + 1) / 2) * ((g->n[2] + 1) / 2);
  return 8 * bricks * packed_cell_bytes(f->kind, f->n_bands);
}

// A one-band (rho, T) field on a uniform grid also keeps its (rho, T) as
// 8-byte records after the 16-byte ones (256-byte aligned): the marches of
// the levels whose rays lie at least half a cell apart read those, since a
// 128-byte line then holds 4x2x2 cells instead of 2x2x2 and scattered rays
// fetch fewer lines.  The optics they evaluate are the packing's own, so a
// ray's values are the same bits from either copy.
int64_t packed_rt_bytes(const air_grid* g, const air_field* f) {
  if (g->kind != AIR_GRID_UNIFORM || f->kind != AIR_FIELD_RHO_T || f->n_bands != 1) return 0;
  const int64_t bricks = (int64_t)((g->n[0] + 1) / 2) * ((g->n[1] + 1) / 2) * ((g->n[2] + 1) / 2);
  return 8 * bricks * 8;
}

// A block-AMR field is followed by the leaf block of every position of the
// finest block lattice (4 bytes each), so the march locates a leaf with one
// load instead of a chain of child-table loads; lattices of more than 2^26
// positions have no map (the march descends the table).
int64_t packed_leaf_entries(const air_grid* g) {
  // an entry holds the leaf id in 28 bits and its level in 4
  if (g->kind != AIR_GRID_BLOCK_AMR || g->max_level < 0 || g->max_level > 15 || g->n_blocks >= (1 << 28)) return 0;
  int64_t e = 1;
  for (int a = 0; a < 3; ++a) {
    e *= (int64_t)g->n[a] << g->max_level;
    if (e > ((int64_t)1 << 26)) return 0;
  }
  return e;
}

// the copy or the map starts at the next multiple of 256 bytes
int64_t packed_rt_off(const air_grid* g, const air_field* f) { return (packed_main_bytes(g, f) + 255) / 256 * 256; }

int64_t packed_bytes_of(const air_grid* g, const air_field* f) {
  const int64_t rt = packed_rt_bytes(g, f), lm = 4 * packed_leaf_entries(g);
  if (rt) return packed_rt_off(g, f) + rt;
  if (lm) return packed_rt_off(g, f) + lm;
  return packed_main_bytes(g, f);
}

// each copy is read through a buffer resource with a 32-bit size
bool packed_too_large(const air_grid* g, const air_field* f) {
  return packed_main_bytes(g, f) >= ((int64_t)1 << 32) || packed_rt_bytes(g, f) >= ((int64_t)1 << 32);
}

void fill_fld(const air_field* f, const air_grid* g, Fld& F) {
  std::memset(&F, 0, sizeof F);
  F.kind = f->kind;
  F.nb = f->kind == AIR_FIELD_RHO_J_KAPPA ? 1 : f->n_bands;
  F.rho = f->rho;
  F.emis = f->emis;
  F.kappa = f->kappa;
  F.temp = f->temp;
  F.packed = f->packed;
  if (g->kind == AIR_GRID_UNIFORM) {
    F.bnx = (g->n[0] + 1) / 2;
    F.bny = (g->n[1] + 1) / 2;
    F.bnz = (g->n[2] + 1) / 2;
  }
  F.packed_bytes = (uint32_t)packed_main_bytes(g, f);
  F.rt_bytes = (uint32_t)packed_rt_bytes(g, f);
  F.rt_off = F.rt_bytes ? packed_rt_off(g, f) : 0;
  F.leaf_map = packed_leaf_entries(g) > 0 ? 1 : 0;
  F.leaf_off = F.leaf_map ? packed_rt_off(g, f) : 0;
  for (int b = 0; b < F.nb && f->kind == AIR_FIELD_RHO_T; ++b) {
    F.k0[b] = (float)f->band[b][0];
    F.s[b] = (float)f->band[b][1];
    F.q[b] = (float)f->band[b][2];
    F.rk0[b] = (float)(1.0 / f->band[b][0]);
  }
  // the ladder form for two or more bands whose s step evenly and whose q agree
  if (f->kind == AIR_FIELD_RHO_T && F.nb >= 2) {
    const double s0 = f->band[0][1], ds = f->band[1][1] - f->band[0][1];
    bool lad = true;
    for (int b = 0; b < F.nb; ++b) {
      lad = lad && f->band[b][2] == f->band[0][2] && f->band[b][0] > 0.0;
      lad = lad && std::fabs(f->band[b][1] - (s0 + b * ds)) <= 1e-12 * (1.0 + std::fabs(s0) + std::fabs(b * ds));
    }
    F.ladder = lad ? 1 : 0;
    F.s0 = (float)s0;
    F.ds = (float)ds;
    F.q0 = (float)f->band[0][2];
  }
}

hipError_t pack_any(const Geo& g, const Fld& f, void* packed, hipStream_t s) {
  if (g.kind != AIR_GRID_BLOCK_AMR) return launch_pack(g, f, packed, s);
  const hipError_t e = launch_pack_amr(g, f, packed, s);
  return e == hipSuccess && f.leaf_map ? launch_leaf_map(g, f, packed, s) : e;
}

// point the march at a packed layout: the caller's, or one written now
air_status ensure_packed(air_ctx* c, const air_grid* g, const air_field* f, MarchArgs& A, hipStream_t s) {
  const int64_t need = packed_bytes_of(g, f);
  if (packed_too_large(g, f)) return fail(c, AIR_ENOTSUP, "packed field of %lld bytes: a copy exceeds 4 GiB", (long long)need);
  if (f->packed) {
    // the leaf map is trusted only for a buffer packed on this context with
    // these tables and this shape; otherwise the march descends the table
    if (A.f.leaf_map && !blocks_known(c, g, f->packed)) A.f.leaf_map = 0;
    return AIR_OK;
  }
  air_status st = ensure(c, c->pack, (size_t)need);
  if (st) return st;
  A.f.packed = c->pack.p;
  HIPCHK(c, pack_any(A.g, A.f, c->pack.p, s));
  return AIR_OK;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

air_status upload_views(air_ctx* c, const air_view* views, int V, hipStream_t s, const DevView** out) {
  std::vector<DevView> hv(V);
  for (int k = 0; k < V; ++k) {
    air_status st = make_view(c, &views[k], hv[k]);
    if (st) return st;
  }
  air_status st = ensure(c, c->views, sizeof(DevView) * V);
  if (st) return st;
  const size_t bytes = sizeof(DevView) * V;
  const bool same = c->views_at == c->views.p && c->views_cap == c->views.bytes && c->views_bytes == bytes &&
                    c->stage && std::memcmp(c->stage, hv.data(), bytes) == 0;
  if (!same) {
    if ((st = ensure_host(c, &c->stage, &c->stage_n, bytes))) return st;
    std::memcpy(c->stage, hv.data(), bytes);
    c->views_at = nullptr;  // until the copy is queued
    HIPCHK(c, hipMemcpyAsync(c->views.p, c->stage, bytes, hipMemcpyHostToDevice, s));
    c->views_at = c->views.p;
    c->views_cap = c->views.bytes;
    c->views_bytes = bytes;
  }
  *out = (const DevView*)c->views.p;
  return AIR_OK;
}

// a multiple of 8 blocks (one share per XCD), about 16 waves per CU
int march_blocks(const air_ctx* c, int seg_shift, int waves_per_cu = 16) {
  const int per_cu = std::max(1, waves_per_cu >> seg_shift);
  return std::max(8, (c->num_cus * per_cu + 7) / 8 * 8);
}


// network workspace for P pixels (the training buffers too when asked)
air_status ensure_cnn_work(air_ctx* c, int64_t P, bool training) {
  air_status st;
  if ((st = ensure(c, c->cx0, 2 * cnn::XC * P))) return st;
  if ((st = ensure(c, c->ca1, 2 * cnn::HID * P))) return st;
  if ((st = ensure(c, c->ca2, 2 * cnn::HID * P))) return st;
  if ((st = ensure(c, c->ca3, 2 * cnn::HID * P))) return st;
  if ((st = ensure(c, c->cz, 4 * cnn::ZC * P))) return st;
  if (!training) return AIR_OK;
  if ((st = ensure(c, c->cdz, 2 * cnn::ZC * P))) return st;
  if ((st = ensure(c, c->cda, 2 * cnn::HID * P))) return st;
  if ((st = ensure(c, c->cdb, 2 * cnn::HID * P))) return st;
  if ((st = ensure(c, c->cdc, 2 * cnn::HID * P))) return st;
  if ((st = ensure(c, c->cwpart, 4 * cnn::wgrad_partial_floats()))) return st;
  if ((st = ensure(c, c->closs_part, 8 * cnn::loss_partial_doubles()))) return st;
  return ensure(c, c->closs, 16);
}

// device buffers and march arguments of one render of V views to Lm levels
air_status setup_render(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views, int V,
                        int N0, int Lm, bool range, hipStream_t s, MarchArgs& A, int64_t& n_chunks,
                        bool pack = true) {
  std::memset(&A, 0, sizeof A);
  fill_geo(grid, A.g);
  if (c->seg_shift_override >= 0) A.g.seg_shift = c->seg_shift_override;
  fill_fld(field, grid, A.f);
  const int nb = A.f.nb;
  A.img.N0 = N0;
  A.img.Lmax = Lm;
  A.img.V = V;
  // every level starts on a counting chunk, so a chunk belongs to one
  // (view, level)
  int64_t off = 0;
  for (int L = 0; L <= Lm; ++L) {
    A.img.off[L] = off;
    off = round_up(off + ((int64_t)N0 * N0 << (2 * L)), CHUNK);
  }
  for (int L = Lm + 1; L <= MAXL; ++L) A.img.off[L] = off;
  const int64_t S = off;
  A.img.S = S;
  const int64_t VS = (int64_t)V * S;
  n_chunks = VS / CHUNK;
  air_status st;
  if ((st = ensure(c, c->state, VS))) return st;
  if ((st = ensure(c, c->valI, 4 * VS * nb))) return st;
  if ((st = ensure(c, c->valN, 4 * VS))) return st;
  if ((st = ensure(c, c->xiI, 4 * VS))) return st;
  if ((st = ensure(c, c->xiN, 4 * VS))) return st;
  if ((st = ensure(c, c->visits, 4 * VS))) return st;
  if ((st = ensure(c, c->queue, 8 * VS))) return st;
  if ((st = ensure(c, c->ctr, 8 * CTR_COUNT))) return st;
  if ((st = ensure(c, c->chunk, 8 * (n_chunks + 1)))) return st;
  if ((st = ensure(c, c->cstat, 4 * VS_N * n_chunks))) return st;
  if ((st = ensure(c, c->partial, 8 * n_chunks * nb))) return st;
  A.w.state = (uint8_t*)c->state.p;
  A.w.valI = (float*)c->valI.p;
  A.w.valN = (float*)c->valN.p;
  A.w.xiI = (float*)c->xiI.p;
  A.w.xiN = (float*)c->xiN.p;
  A.w.visits = (int*)c->visits.p;
  A.w.queue = (uint64_t*)c->queue.p;
  A.w.qcap = (uint64_t)VS;
  A.w.ctr = (unsigned long long*)c->ctr.p;
  // split tiles for the coarse levels whose launches are small enough
  // (level 1 has the smallest bound of them); the partial buffer is sized
  // for the largest such launch
  A.w.split_tiles = c->split_tiles;
  if (Lm >= 1 && split_level(A, 1)) {
    int64_t tiles = 0;
    for (int L = 1; L <= Lm && split_level(A, L); ++L) tiles = queue_tile_bound(A, L);
    const size_t pb = 4 * (size_t)tiles * ((size_t)1 << A.g.seg_shift) * split_fields(march_nb(A.f.kind, nb)) * WAVE;
    if ((st = ensure(c, c->parts, pb))) return st;
    A.w.parts = (float*)c->parts.p;
    A.w.split_tiles = tiles;
  } else {
    A.w.split_tiles = 0;
  }
  if (range) {
    const int64_t n0 = (int64_t)V * N0 * N0;
    if ((st = ensure(c, c->rmin, 4 * n0))) return st;
    if ((st = ensure(c, c->rmax, 4 * n0))) return st;
    if ((st = ensure(c, c->lmax0, 4 * n0))) return st;
    A.w.rmin = (float*)c->rmin.p;
    A.w.rmax = (float*)c->rmax.p;
    A.w.lmax0 = (int*)c->lmax0.p;
  }
  if ((st = upload_views(c, views, V, s, &A.views))) return st;
  A.img.min_width = views[0].width;
  for (int k = 1; k < V; ++k) A.img.min_width = std::min(A.img.min_width, views[k].width);
  return pack ? ensure_packed(c, grid, field, A, s) : AIR_OK;
}

air_status check_render_args(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                             int n_views, const air_params* prm) {
  air_status st;
  if ((st = check_grid(c, grid))) return st;
  if ((st = check_field(c, field))) return st;
  if (!views || n_views < 1 || n_views > AIR_MAX_VIEWS)
    return fail(c, AIR_EINVAL, "n_views %d out of range 1..%d", n_views, AIR_MAX_VIEWS);
  if (!prm) return fail(c, AIR_EINVAL, "params is NULL");
  const int N0 = prm->coarse_n, Lm = prm->max_level;
  if (N0 < 1 || N0 > 65536) return fail(c, AIR_EINVAL, "coarse_n %d out of range", N0);
  if (Lm < 0 || Lm >= AIR_MAX_LEVELS) return fail(c, AIR_EINVAL, "max_level %d out of range 0..%d", Lm, AIR_MAX_LEVELS - 1);
  if ((double)N0 * N0 * std::pow(4.0, Lm) > 4294967295.0)
    return fail(c, AIR_EINVAL, "coarse_n^2 * 4^max_level exceeds 2^32 pixels per view");
  if (!std::isfinite(prm->xi_crit_I) || !std::isfinite(prm->xi_crit_N) || prm->xi_crit_I < 0 || prm->xi_crit_N < 0)
    return fail(c, AIR_EINVAL, "xi_crit must be finite and >= 0");
  if (prm->flags & ~(AIR_FLAG_TIMING | AIR_FLAG_SUPERRES)) return fail(c, AIR_EINVAL, "params.flags has unknown bits");
  return AIR_OK;
}

// device buffers of the learned steps
air_status ensure_learned(air_ctx* c, const MarchArgs& A) {
  const int64_t total = (int64_t)A.img.V * A.img.N0 * A.img.N0, VS = (int64_t)A.img.V * A.img.S;
  air_status st;
  if ((st = ensure(c, c->feat, 16 * total))) return st;
  if ((st = ensure_cnn_work(c, total, false))) return st;
  if ((st = ensure(c, c->depth8, total))) return st;
  if ((st = ensure(c, c->scount, 8 * (total + 1)))) return st;
  return ensure(c, c->spec, 8 * VS);
}

// the learned steps after the coarse march: feature maps, network, depth
// choice, work list, speculative march
air_status learned_steps(air_ctx* c, const MarchArgs& A, const air_cnn* net, const air_learn_params* lp,
                         const uint8_t* given_depth, const float* w, bool timing, const Tune& tune, hipStream_t s) {
  const int V = A.img.V, N0 = A.img.N0;
  const int64_t total = (int64_t)V * N0 * N0;
  if (timing) HIPCHK(c, hipEventRecord(c->ev[air_ctx::EV_FEAT0], s));
  const int dmax = std::min(lp->max_depth, std::min(A.img.Lmax, DEPTH_CLASSES - 1));
  unsigned long long* cnt = (unsigned long long*)c->scount.p;
  // the work list's length is counted in a device counter (cleared by the
  // render's init launch)
  unsigned long long* spec_n = A.w.ctr + CTR_SPEC;
  if (given_depth) {
    // the caller's depths instead of the network's choice
    HIPCHK(c, launch_spec_reserve(given_depth, dmax, total, (uint8_t*)c->depth8.p, cnt, spec_n, s));
  } else {
    LearnW W;
    for (int b = 0; b < MAXB; ++b) W.w[b] = w[b];
    FeatNorm nm;
    for (int k = 0; k < 4; ++k) {
      nm.mean[k] = net->net.mean[k];
      nm.inv_std[k] = 1.0f / net->net.stdv[k];
    }
    HIPCHK(c, launch_features_bf16(A, W, nm, (uint16_t*)c->cx0.p, s));
    // the four layers and the depth choice in one launch
    HIPCHK(c, cnn::infer_depth(net->net, (const uint16_t*)c->cx0.p, V, N0, N0, dmax, lp->c_ray, lp->c_sweep,
                               (uint8_t*)c->depth8.p, cnt, spec_n, s));
  }
  HIPCHK(c, launch_spec_emit((const uint8_t*)c->depth8.p, cnt, total, (int64_t)N0 * N0, (uint64_t*)c->spec.p, s));
  if (timing) HIPCHK(c, hipEventRecord(c->ev[air_ctx::EV_SPEC0], s));
  HIPCHK(c, launch_march_spec(A, (const uint64_t*)c->spec.p, spec_n,
                              march_blocks(c, A.g.seg_shift, tune.march_waves_per_cu), s));
  if (timing) HIPCHK(c, hipEventRecord(c->ev[air_ctx::EV_SPEC1], s));
  return AIR_OK;
}

// everything a render puts on the stream between its setup and its result
// copies: no allocation and no host wait, so it can be captured in a graph
struct Plan {
  MarchArgs A;
  int64_t n_chunks = 0;
  float xcI = 0, xcN = 0, w[MAXB] = {};
  const air_cnn* net = nullptr;
  const uint8_t* depth_in = nullptr;  // given speculation depths (air_render_proposal)
  air_learn_params lp{};
  bool trees = false, flux = false, timing = false, superres = false;
  float* images = nullptr;
  // where k_finish writes the result block: the context's pinned host buffer
  // (no copy back; a captured sequence is keyed on its address)
  unsigned long long* res = nullptr;
  // per-pixel spectra (air_render_spectra): the spectral march replaces the
  // band march, and the spectra are gathered and integrated after the tree
  bool spectral = false;
  SpecArgs spec{};
  SpecOut spec_out{};
  int64_t spec_cpv = 0;
  double* spec_partial = nullptr;
  double* spec_flux = nullptr;
};

air_status enqueue_render(air_ctx* c, const Plan& P, const Tune& tune, hipStream_t s) {
  const MarchArgs& A = P.A;
  const int Lm = A.img.Lmax;
  hipEvent_t* ev = c->ev;
  air_status st;
  // the level loop: trace the queue of new nodes, then test, close and
  // compact; the queue bounds live in device counters, so no host round trip
  HIPCHK(c, launch_init(A, s));
  for (int L = 0; L <= Lm; ++L) {
    if (P.timing) HIPCHK(c, hipEventRecord(ev[2 + 4 * L], s));
    if (P.spectral)
      HIPCHK(c, launch_march_spectra(A, P.spec, L, c->num_cus * 8, s));
    else
      HIPCHK(c, launch_march_queue(A, L, march_blocks(c, A.g.seg_shift, tune.march_waves_per_cu), s));
    if (P.timing) HIPCHK(c, hipEventRecord(ev[3 + 4 * L], s));
    if ((P.net || P.depth_in) && L == 0) {
      if ((st = learned_steps(c, A, P.net, &P.lp, P.depth_in, P.w, P.timing, tune, s))) return st;
      if (P.timing) HIPCHK(c, hipEventRecord(ev[3 + 4 * L], s));  // the test timing starts after the learned steps
    }
    if (L < Lm) HIPCHK(c, launch_refine(A, L, P.xcI, P.xcN, P.w, c->num_cus * tune.refine_blocks_per_cu, s));
    if (P.timing) HIPCHK(c, hipEventRecord(ev[4 + 4 * L], s));
  }
  unsigned long long* chunk = (unsigned long long*)c->chunk.p;
  double* fpart = P.flux ? (double*)c->partial.p : nullptr;
  HIPCHK(c, launch_count(A, chunk, (unsigned*)c->cstat.p, P.n_chunks, fpart, P.superres ? nullptr : P.images, s));
  if (P.superres && P.images) HIPCHK(c, launch_superres(A, P.images, s));
  HIPCHK(c, launch_finish(A, chunk, P.n_chunks, P.trees, (const unsigned*)c->cstat.p, fpart, P.res, s));
  if (P.trees) {
    HIPCHK(c, launch_emit(A, chunk, P.n_chunks, (int32_t*)c->idmap.p, (uint64_t*)c->nodepos.p, s));
    HIPCHK(c, launch_write_tree(A, chunk, (const int32_t*)c->idmap.p, (const uint64_t*)c->nodepos.p,
                                (const TreeOut*)c->touts.p, c->num_cus * 8, s));
    if (P.spectral)
      HIPCHK(c, launch_spectra_out(A, P.spec, chunk, P.n_chunks, (const uint64_t*)c->nodepos.p, P.spec_out,
                                   P.spec_cpv, P.spec_partial, P.spec_flux, c->num_cus * 8, s));
  }
  return AIR_OK;
}

// the graph key: every argument of every launch (pointers, sizes, scalars);
// the context's buffer generation stands for the addresses of its own
// buffers (queue maps, chunk counters, partial sums, tree index maps, ...)
std::string plan_key(const air_ctx* c, const Plan& P, const Tune& t) {
  std::string k(reinterpret_cast<const char*>(&P.A), sizeof P.A);
  k.append(reinterpret_cast<const char*>(&c->buf_gen), sizeof c->buf_gen);
  k.append(reinterpret_cast<const char*>(&P.n_chunks), sizeof P.n_chunks);
  k.append(reinterpret_cast<const char*>(&P.xcI), sizeof(float) * (2 + MAXB));
  k.append(reinterpret_cast<const char*>(&P.net), sizeof P.net);
  k.append(reinterpret_cast<const char*>(&P.depth_in), sizeof P.depth_in);
  if (P.net) {  // the standardisation is a kernel argument of the captured sequence
    k.append(reinterpret_cast<const char*>(P.net->net.mean), sizeof P.net->net.mean);
    k.append(reinterpret_cast<const char*>(P.net->net.stdv), sizeof P.net->net.stdv);
  }
  k.append(reinterpret_cast<const char*>(&P.lp), sizeof P.lp);
  const char flags[4] = {(char)P.trees, (char)P.flux, (char)P.timing, (char)P.superres};
  k.append(flags, 4);
  k.append(reinterpret_cast<const char*>(&P.images), sizeof P.images);
  k.append(reinterpret_cast<const char*>(&P.res), sizeof P.res);
  k.append(reinterpret_cast<const char*>(&t), sizeof t);
  return k;
}

// the workload shape the launch shapes are tuned for
std::string shape_key(const Plan& P) {
  char b[256];
  snprintf(b, sizeof b, "%d/%d,%d,%d/%d,%d/%d/%d/%d/%d", P.A.g.kind, P.A.g.n[0], P.A.g.n[1], P.A.g.n[2],
           P.A.g.bs, P.A.g.max_level, P.A.img.V, P.A.img.N0, P.A.img.Lmax, P.A.f.nb);
  return std::string(b) + (P.net ? "/learned" : P.depth_in ? "/proposal" : "/plain");
}

// pick the launch shapes by timing the whole render once per candidate
// (results do not depend on them), then keep the fastest for the shape
air_status autotune(air_ctx* c, const Plan& P, hipStream_t s, Tune& best) {
  const std::string key = shape_key(P);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    best = it->second;
    return AIR_OK;
  }
  float best_ms = 1e30f;
  for (int mw : {8, 16, 32})
    for (int rb : {2, 4, 8}) {
      Tune t;
      t.march_waves_per_cu = mw;
      t.refine_blocks_per_cu = rb;
      float ms = 0.0f;
      for (int rep = 0; rep < 2; ++rep) {  // the second run is timed
        HIPCHK(c, hipEventRecord(c->ev[0], s));
        air_status st = enqueue_render(c, P, t, s);
        if (st) return st;
        HIPCHK(c, hipEventRecord(c->ev[1], s));
        HIPCHK(c, hipEventSynchronize(c->ev[1]));
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  c->tuned[key] = best;
  return AIR_OK;
}

air_status render_core(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                       int32_t n_views, const air_params* prm, const air_cnn* net, const air_learn_params* lp,
                       air_tree* trees, float* images, double* flux, air_stats* stats, air_learn_stats* ls,
                       void* stream, bool batch, const air_spectrum* spectrum = nullptr, float* spectra = nullptr,
                       const uint8_t* given_depth = nullptr) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  air_status st;
  // the spectral render traces (rho, T) with its bin table; the level loop
  // refines on the broadband, carried as the one band of the maps
  air_field fone;
  if (spectrum) {
    fone = *field;
    fone.n_bands = 1;
    fone.packed = nullptr;
    field = &fone;
  }
  if ((st = check_render_args(c, grid, field, views, n_views, prm))) return st;
  for (int k = 0; trees && k < n_views; ++k)
    if (trees[k].capacity < 0) return fail(c, AIR_EINVAL, "tree %d capacity < 0", k);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_blocks(c, grid, s, field->packed))) return st;
  const bool learned = net != nullptr || given_depth != nullptr;
  const int N0 = prm->coarse_n, Lm = prm->max_level, V = n_views;
  Plan P;
  if ((st = setup_render(c, grid, field, views, V, N0, Lm, net != nullptr, s, P.A, P.n_chunks, !spectrum))) return st;
  const MarchArgs& A = P.A;
  const int nb = A.f.nb;
  P.A.w.skip_spec = learned ? 1 : 0;
  P.xcI = prm->xi_crit_I;
  P.xcN = prm->xi_crit_N;
  for (int b = 0; b < MAXB; ++b) P.w[b] = b < nb ? prm->band_weight[b] : 0.0f;
  const int nbins = spectrum ? spectrum->n_bins : 0;
  double* const spectrum_flux = spectrum ? flux : nullptr;  // the caller's [V][n_bins]
  if (spectrum) {
    P.w[0] = 1.0f;  // the broadband is already weighted
    P.spectral = true;
    // bin table [6][stride]: k0, -s, q, -E log2(e), e0, broadband weight
    const int stride = (nbins + 63) / 64 * 64;
    std::vector<float> tab(6 * (size_t)stride, 0.0f);
    for (int b = 0; b < nbins; ++b) {
      const double* r = spectrum->bins + 5 * (size_t)b;
      tab[0 * stride + b] = (float)r[0];
      tab[1 * stride + b] = (float)(-r[1]);
      tab[2 * stride + b] = (float)r[3];
      tab[3 * stride + b] = (float)(-r[4] * 1.4426950408889634);
      tab[4 * stride + b] = (float)r[2];
      tab[5 * stride + b] = spectrum->weight[b];
    }
    int64_t cap_total = 0, cap_max = 0;
    std::vector<int64_t> rows(2 * (size_t)V);
    for (int k = 0; k < V; ++k) {
      rows[k] = cap_total;
      rows[V + k] = trees[k].capacity;
      cap_total += trees[k].capacity;
      cap_max = std::max<int64_t>(cap_max, trees[k].capacity);
    }
    if (cap_total >= ((int64_t)1 << 32)) return fail(c, AIR_EINVAL, "total tree capacity reaches 2^32");
    if ((st = ensure(c, c->spec_tab, 4 * tab.size()))) return st;
    if ((st = ensure(c, c->spec_store, 4 * (size_t)std::max<int64_t>(cap_total, 1) * nbins))) return st;
    if ((st = ensure(c, c->spec_qpos, 4 * (size_t)V * A.img.S))) return st;
    if ((st = ensure(c, c->spec_rows, 8 * rows.size()))) return st;
    if ((st = ensure(c, c->spec_flag, 16))) return st;
    P.spec_cpv = (cap_max + SPEC_CHUNK - 1) / SPEC_CHUNK;
    if ((st = ensure(c, c->spec_part, 8 * (size_t)V * std::max<int64_t>(P.spec_cpv, 1) * nbins))) return st;
    if ((st = ensure(c, c->spec_flux, 8 * (size_t)V * nbins))) return st;
    if ((st = ensure_host(c, &c->host_spec, &c->host_spec_n, 16 + 8 * (size_t)V * nbins))) return st;
    HIPCHK(c, hipMemcpyAsync(c->spec_tab.p, tab.data(), 4 * tab.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->spec_rows.p, rows.data(), 8 * rows.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemsetAsync(c->spec_flag.p, 0, 16, s));
    P.spec = SpecArgs{nbins, stride, (const float*)c->spec_tab.p, (float*)c->spec_store.p,
                      (unsigned long long)cap_total, (uint32_t*)c->spec_qpos.p, (unsigned*)c->spec_flag.p};
    P.spec_out = SpecOut{spectra, (const int64_t*)c->spec_rows.p, (const int64_t*)c->spec_rows.p + V};
    P.spec_partial = (double*)c->spec_part.p;
    P.spec_flux = flux ? (double*)c->spec_flux.p : nullptr;
    flux = nullptr;  // the broadband flux of the result block is not asked for
  }
  P.net = net;
  P.depth_in = given_depth;
  if (lp) P.lp = *lp;
  P.trees = trees != nullptr;
  P.flux = flux != nullptr;
  P.images = images;
  P.timing = !batch && (prm->flags & AIR_FLAG_TIMING) != 0;
  P.superres = (prm->flags & AIR_FLAG_SUPERRES) != 0;
  const size_t res_bytes = 8 * (size_t)res_words(V, nb);
  if ((st = ensure_host(c, (void**)&c->host_vstat, &c->host_vstat_n, res_bytes))) return st;
  P.res = c->host_vstat;
  if (learned && (st = ensure_learned(c, A))) return st;
  if (learned) c->cnn_pixels = -1;  // the learned steps overwrite the network buffers
  if (trees) {
    if ((st = ensure(c, c->idmap, 4 * (size_t)V * A.img.S))) return st;
    if ((st = ensure(c, c->nodepos, 8 * (size_t)V * A.img.S))) return st;
    if ((st = ensure(c, c->touts, sizeof(TreeOut) * V))) return st;
    std::vector<TreeOut> to(V);
    for (int k = 0; k < V; ++k) {
      const air_tree& t = trees[k];
      to[k] = TreeOut{t.level, t.ix, t.iy, t.parent, t.first_child, t.state, t.I, t.N, t.xi_I, t.xi_N,
                      t.visits, t.capacity};
    }
    const size_t bytes = sizeof(TreeOut) * V;
    const bool same = c->touts_at == c->touts.p && c->touts_cap == c->touts.bytes && c->touts_bytes == bytes &&
                      c->stage2 && std::memcmp(c->stage2, to.data(), bytes) == 0;
    if (!same) {
      if ((st = ensure_host(c, &c->stage2, &c->stage2_n, bytes))) return st;
      std::memcpy(c->stage2, to.data(), bytes);
      c->touts_at = nullptr;
      HIPCHK(c, hipMemcpyAsync(c->touts.p, c->stage2, bytes, hipMemcpyHostToDevice, s));
      c->touts_at = c->touts.p;
      c->touts_cap = c->touts.bytes;
      c->touts_bytes = bytes;
    }
  }
  hipEvent_t* ev = c->ev;
  if (batch) {
    Tune tune;
    if ((st = autotune(c, P, s, tune))) return st;
    const std::string key = plan_key(c, P, tune);
    // capture on the context's own stream (the caller's may be the null
    // stream, which cannot be captured), after the uploads above
    hipStream_t cs = c->cap_stream;
    if (key != c->graph_key || !c->graph_exec) {
      if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
      if (c->graph) (void)hipGraphDestroy(c->graph);
      c->graph_exec = nullptr;
      c->graph = nullptr;
      c->graph_key.clear();
      HIPCHK(c, hipStreamSynchronize(s));  // the tuning runs are done before the sequence is captured
      HIPCHK(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      st = enqueue_render(c, P, tune, cs);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &g);
      if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(c, AIR_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
      HIPCHK(c, hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
      c->graph = g;
      c->graph_key = key;
    }
    // replayed on the caller's stream, after the uploads above
    HIPCHK(c, hipEventRecord(ev[0], s));
    HIPCHK(c, hipGraphLaunch(c->graph_exec, s));
  } else {
    HIPCHK(c, hipEventRecord(ev[0], s));
    if ((st = enqueue_render(c, P, c->eager, s))) return st;
  }
  HIPCHK(c, hipEventRecord(ev[1], s));
  const bool timing = P.timing;
  // one wait for the result block (counters, per-view counts, fluxes),
  // which k_finish wrote to the pinned host buffer
  if (spectrum) {
    unsigned char* hs = static_cast<unsigned char*>(c->host_spec);
    HIPCHK(c, hipMemcpyAsync(hs, c->spec_flag.p, 4, hipMemcpyDeviceToHost, s));
    if (P.spec_flux) HIPCHK(c, hipMemcpyAsync(hs + 16, P.spec_flux, 8 * (size_t)V * nbins, hipMemcpyDeviceToHost, s));
  }
  std::vector<uint8_t> depth_h;
  if (learned && ls) {
    depth_h.resize((size_t)V * N0 * N0);
    HIPCHK(c, hipMemcpyAsync(depth_h.data(), c->depth8.p, depth_h.size(), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, spin_stream(s));
  const unsigned long long* hc = c->host_vstat;  // the counters lead the result block
  const unsigned long long* hv = c->host_vstat + res_vstat_off();
  if (hc[CTR_OVERFLOW]) return fail(c, AIR_EDEVICE, "internal work queue overflow");
  bool spec_overflow = false;
  if (spectrum) {
    const unsigned char* hs = static_cast<const unsigned char*>(c->host_spec);
    spec_overflow = *reinterpret_cast<const unsigned*>(hs) != 0;
    if (spectrum_flux) std::memcpy(spectrum_flux, hs + 16, 8 * (size_t)V * nbins);
  }
  if (flux) std::memcpy(flux, c->host_vstat + res_flux_off(V), 8 * V * nb);
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    for (int k = 0; k < CTR_SLOTS; ++k) {
      stats->hits += (int64_t)hc[CTR_HITS + k];
      stats->visits += (int64_t)hc[CTR_VISITS + k];
    }
    for (int v = 0; v < V; ++v)
      for (int L = 0; L <= Lm; ++L) {
        const unsigned long long* r = hv + ((size_t)v * MAXL + L) * VS_N;
        stats->rays_per_level[L] += (int64_t)r[VS_NODES];
        stats->leaves += (int64_t)r[VS_LEAVES];
        stats->tested += (int64_t)r[VS_TESTED];
        stats->flagged += (int64_t)r[VS_FLAGGED];
        stats->balance += (int64_t)r[VS_BALANCE];
      }
    for (int L = 0; L <= Lm; ++L) {
      stats->rays += stats->rays_per_level[L];
      if (stats->rays_per_level[L]) stats->depth = L;
    }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) stats->ms_total = ms;
    for (int L = 0; timing && L <= Lm; ++L) {
      if (hipEventElapsedTime(&ms, ev[2 + 4 * L], ev[3 + 4 * L]) == hipSuccess) stats->ms_march += ms;
      if (hipEventElapsedTime(&ms, ev[3 + 4 * L], ev[4 + 4 * L]) == hipSuccess) stats->ms_test += ms;
    }
    stats->march_launches = Lm + 1;
    if (learned) {
      if (timing && hipEventElapsedTime(&ms, ev[air_ctx::EV_SPEC0], ev[air_ctx::EV_SPEC1]) == hipSuccess)
        stats->ms_march += ms;
      stats->march_launches += 1;
    }
  }
  if (learned && ls) {
    std::memset(ls, 0, sizeof *ls);
    for (int v = 0; v < V; ++v)
      for (int L = 0; L <= Lm; ++L) {
        const unsigned long long* r = hv + ((size_t)v * MAXL + L) * VS_N;
        ls->spec_rays += (int64_t)r[VS_SPEC];
        ls->wasted += (int64_t)r[VS_WASTED];
        ls->missing += (int64_t)r[VS_MISSING];
      }
    for (uint8_t d : depth_h) ls->depth_hist[d] += 1;
    float ms = 0.0f;
    if (timing && hipEventElapsedTime(&ms, ev[air_ctx::EV_FEAT0], ev[air_ctx::EV_SPEC0]) == hipSuccess)
      ls->ms_features = ms;
    if (timing && hipEventElapsedTime(&ms, ev[air_ctx::EV_SPEC0], ev[air_ctx::EV_SPEC1]) == hipSuccess)
      ls->ms_spec = ms;
  }
  air_status res = AIR_OK;
  for (int k = 0; trees && k < V; ++k) {
    int64_t n = 0, leaves = 0;
    for (int L = 0; L < MAXL; ++L) {
      const unsigned long long* r = hv + ((size_t)k * MAXL + L) * VS_N;
      trees[k].n_per_level[L] = L <= Lm ? (int64_t)r[VS_NODES] : 0;
      if (L <= Lm) {
        n += (int64_t)r[VS_NODES];
        leaves += (int64_t)r[VS_LEAVES];
      }
    }
    trees[k].n_nodes = n;
    trees[k].n_leaves = leaves;
    if (n > trees[k].capacity)
      res = fail(c, AIR_ECAPACITY, "tree %d needs %lld nodes, capacity %lld", k, (long long)n,
                 (long long)trees[k].capacity);
  }
  if (res == AIR_OK && spec_overflow)
    res = fail(c, AIR_ECAPACITY, "traced rays exceed the trees' total capacity (spectra store)");
  return res;
}

}  // namespace

extern "C" {

air_status air_create(air_ctx** out, int32_t device) {
  if (!out) return AIR_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return AIR_EINVAL;
  }
  air_ctx* c = new air_ctx();
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return AIR_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cus = prop.multiProcessorCount;
  if (const char* e = std::getenv("AIR_MARCH_WAVES")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 64) c->eager.march_waves_per_cu = v;
  }
  if (const char* e = std::getenv("AIR_SEG_SHIFT")) {
    const int v = std::atoi(e);
    if (v >= 0 && (1 << v) <= MAX_SEG) c->seg_shift_override = v;
  }
  if (const char* e = std::getenv("AIR_SPLIT_TILES")) {
    const long long v = std::atoll(e);
    if (v >= 0 && v <= (1 << 20)) c->split_tiles = v;
  }
  size_t have = 0;
  if (ensure_host(c, (void**)&c->host_ctr, &have, sizeof(unsigned long long) * CTR_COUNT)) {
    delete c;
    return AIR_ENOMEM;
  }
  for (int k = 0; k < air_ctx::NEV; ++k)
    if (hipEventCreate(&c->ev[k]) != hipSuccess) {
      air_destroy(c);
      return AIR_EDEVICE;
    }
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    air_destroy(c);
    return AIR_EDEVICE;
  }
  // the device is current: the static workspace's address on this device
  if (noalloc_init(device, &c->noalloc) != hipSuccess) {
    (void)hipGetLastError();
    air_destroy(c);
    return AIR_EDEVICE;
  }
  *out = c;
  return AIR_OK;
}

void air_destroy(air_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (DevBuf* b : {&c->state, &c->valI, &c->valN, &c->xiI, &c->xiN, &c->visits, &c->rmin, &c->rmax, &c->queue,
                    &c->ctr, &c->chunk, &c->cstat, &c->idmap, &c->partial, &c->flux, &c->views,
                    &c->touts, &c->pack, &c->nodepos, &c->lmax0, &c->feat, &c->cx0, &c->ca1, &c->ca2, &c->ca3, &c->cz,
                    &c->cdz, &c->cda, &c->cdb, &c->cdc, &c->cwpart, &c->closs_part, &c->closs, &c->depth8, &c->scount,
                    &c->spec, &c->parts, &c->spec_tab, &c->spec_store, &c->spec_qpos, &c->spec_rows,
                    &c->spec_flag, &c->spec_part, &c->spec_flux})
    if (b->p) (void)hipFree(b->p);
  if (c->host_spec) (void)hipHostFree(c->host_spec);
  if (c->host_ctr) (void)hipHostFree(c->host_ctr);
  if (c->host_flux) (void)hipHostFree(c->host_flux);
  if (c->host_vstat) (void)hipHostFree(c->host_vstat);
  if (c->stage) (void)hipHostFree(c->stage);
  if (c->stage2) (void)hipHostFree(c->stage2);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int k = 0; k < air_ctx::NEV; ++k)
    if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
  delete c;
}

const char* air_last_error(const air_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

air_status air_render(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                      int32_t n_views, const air_params* prm, air_tree* trees, float* images, double* flux,
                      air_stats* stats, void* stream) {
  return render_core(c, grid, field, views, n_views, prm, nullptr, nullptr, trees, images, flux, stats, nullptr,
                     stream, false);
}

air_status air_render_batch(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                            int32_t n_views, const air_params* prm, air_tree* trees, float* images, double* flux,
                            air_stats* stats, void* stream) {
  return render_core(c, grid, field, views, n_views, prm, nullptr, nullptr, trees, images, flux, stats, nullptr,
                     stream, true);
}

air_status air_render_learned(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                              int32_t n_views, const air_params* prm, const air_cnn* net,
                              const air_learn_params* learn, air_tree* trees, float* images, double* flux,
                              air_stats* stats, air_learn_stats* learn_stats, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!net || !learn) return fail(c, AIR_EINVAL, "network or learn parameters NULL");
  if (net->device != c->device) return fail(c, AIR_EINVAL, "network and context are on different devices");
  if (!std::isfinite(learn->c_ray) || !std::isfinite(learn->c_sweep) || learn->c_ray < 0 || learn->c_sweep < 0)
    return fail(c, AIR_EINVAL, "c_ray and c_sweep must be finite and >= 0");
  if (learn->max_depth < 0 || learn->flags != 0) return fail(c, AIR_EINVAL, "max_depth < 0 or flags != 0");
  return render_core(c, grid, field, views, n_views, prm, net, learn, trees, images, flux, stats, learn_stats,
                     stream, false);
}

air_status air_render_spectra(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                              int32_t n_views, const air_params* prm, const air_spectrum* spectrum, air_tree* trees,
                              float* spectra, float* images, double* flux, air_stats* stats, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!spectrum || spectrum->n_bins < 1 || spectrum->n_bins > AIR_MAX_BINS || !spectrum->bins || !spectrum->weight)
    return fail(c, AIR_EINVAL, "spectrum: 1..%d bins with their table and weights", AIR_MAX_BINS);
  for (int b = 0; b < spectrum->n_bins; ++b) {
    const double* r = spectrum->bins + 5 * (size_t)b;
    if (!std::isfinite(r[0]) || !std::isfinite(r[1]) || !std::isfinite(r[2]) || !std::isfinite(r[3]) ||
        !std::isfinite(r[4]) || r[0] < 0 || r[2] < 0 || !std::isfinite(spectrum->weight[b]) || spectrum->weight[b] < 0)
      return fail(c, AIR_EINVAL, "bin %d: parameters must be finite, k0, e0 and the weight >= 0", b);
  }
  if (!grid || grid->kind != AIR_GRID_UNIFORM)
    return fail(c, grid ? AIR_ENOTSUP : AIR_EINVAL, "spectra are traced on uniform grids");
  if (!field || field->kind != AIR_FIELD_RHO_T || !field->rho || !field->temp)
    return fail(c, AIR_EINVAL, "spectra need a (rho, T) field");
  if (!trees) return fail(c, AIR_EINVAL, "spectra need the trees");
  if (prm && (prm->flags & AIR_FLAG_SUPERRES)) return fail(c, AIR_ENOTSUP, "no super-resolution with spectra");
  return render_core(c, grid, field, views, n_views, prm, nullptr, nullptr, trees, images, flux, stats, nullptr,
                     stream, false, spectrum, spectra);
}

air_status air_render_proposal(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                               int32_t n_views, const air_params* prm, const uint8_t* depth, int32_t max_depth,
                               air_tree* trees, float* images, double* flux, air_stats* stats,
                               air_learn_stats* learn_stats, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!depth) return fail(c, AIR_EINVAL, "depth is NULL");
  if (max_depth < 0) return fail(c, AIR_EINVAL, "max_depth < 0");
  air_learn_params lp{};
  lp.max_depth = max_depth;
  return render_core(c, grid, field, views, n_views, prm, nullptr, &lp, trees, images, flux, stats, learn_stats,
                     stream, false, nullptr, nullptr, depth);
}

air_status air_render_fixed(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                            int32_t n_views, int32_t coarse_n, int32_t level, float* images, double* flux,
                            air_stats* stats, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  air_status st;
  if ((st = check_grid(c, grid))) return st;
  if ((st = check_field(c, field))) return st;
  if (!views || n_views < 1 || n_views > AIR_MAX_VIEWS)
    return fail(c, AIR_EINVAL, "n_views %d out of range 1..%d", n_views, AIR_MAX_VIEWS);
  if (coarse_n < 1 || level < 0 || level >= AIR_MAX_LEVELS)
    return fail(c, AIR_EINVAL, "coarse_n %d / level %d out of range", coarse_n, level);
  const int64_t R = (int64_t)coarse_n << level;
  if ((double)R * R > 4294967295.0) return fail(c, AIR_EINVAL, "raster exceeds 2^32 pixels per view");
  if (flux && !images) return fail(c, AIR_EINVAL, "flux needs the image buffer");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_blocks(c, grid, s, field->packed))) return st;
  MarchArgs A;
  std::memset(&A, 0, sizeof A);
  fill_geo(grid, A.g);
  if (c->seg_shift_override >= 0) A.g.seg_shift = c->seg_shift_override;
  fill_fld(field, grid, A.f);
  const int nb = A.f.nb;
  A.img.N0 = coarse_n;
  A.img.Lmax = level;
  A.img.V = n_views;
  if ((st = ensure(c, c->ctr, 8 * CTR_COUNT))) return st;
  A.w.ctr = (unsigned long long*)c->ctr.p;
  if ((st = upload_views(c, views, n_views, s, &A.views))) return st;
  if ((st = ensure_packed(c, grid, field, A, s))) return st;
  HIPCHK(c, hipMemsetAsync(A.w.ctr, 0, 8 * CTR_COUNT, s));
  HIPCHK(c, hipEventRecord(c->ev[0], s));
  HIPCHK(c, hipEventRecord(c->ev[2], s));
  HIPCHK(c, launch_march_fixed(A, level, images, march_blocks(c, A.g.seg_shift), s));
  HIPCHK(c, hipEventRecord(c->ev[3], s));
  const int64_t cpp = (R * R + CHUNK - 1) / CHUNK;
  if (flux) {
    if ((st = ensure(c, c->partial, 8 * (size_t)n_views * nb * cpp))) return st;
    if ((st = ensure(c, c->flux, 8 * (size_t)n_views * nb))) return st;
    // every view has the same pixel size only if widths agree: reduce per view
    std::vector<double> area(n_views);
    for (int k = 0; k < n_views; ++k) {
      double px = views[k].width / (double)R;
      area[k] = px * px;
    }
    for (int k = 0; k < n_views; ++k)
      HIPCHK(c, launch_fixed_flux(images + (size_t)k * (nb + 1) * R * R, 1, nb, R, area[k],
                                  (double*)c->partial.p + (size_t)k * nb * cpp, (double*)c->flux.p + k * nb, s));
  }
  HIPCHK(c, hipEventRecord(c->ev[1], s));
  HIPCHK(c, hipMemcpyAsync(c->host_ctr, A.w.ctr, 8 * CTR_COUNT, hipMemcpyDeviceToHost, s));
  if (flux) {
    if ((st = ensure_host(c, (void**)&c->host_flux, &c->host_flux_n, 8 * n_views * nb))) return st;
    HIPCHK(c, hipMemcpyAsync(c->host_flux, c->flux.p, 8 * n_views * nb, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  if (flux) std::memcpy(flux, c->host_flux, 8 * n_views * nb);
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->rays = (int64_t)n_views * R * R;
    stats->rays_per_level[level] = stats->rays;
    for (int k = 0; k < CTR_SLOTS; ++k) {
      stats->hits += (int64_t)c->host_ctr[CTR_HITS + k];
      stats->visits += (int64_t)c->host_ctr[CTR_VISITS + k];
    }
    stats->leaves = stats->rays;
    stats->depth = level;
    stats->march_launches = 1;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) stats->ms_total = ms;
    if (hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess) stats->ms_march = ms;
  }
  return AIR_OK;
}

air_status air_render_fixed_noalloc(air_ctx* c, const air_grid* grid, const air_field* field,
                                    const air_view* views, int32_t n_views, int32_t coarse_n, int32_t level,
                                    float* images, double* flux, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  air_status st;
  if ((st = check_grid(c, grid))) return st;
  if ((st = check_field(c, field))) return st;
  if (!views || n_views < 1 || n_views > AIR_NOALLOC_MAX_VIEWS)
    return fail(c, AIR_EINVAL, "n_views %d out of range 1..%d (allocation-free limit)", n_views,
                AIR_NOALLOC_MAX_VIEWS);
  if (coarse_n < 1 || level < 0 || level >= AIR_MAX_LEVELS)
    return fail(c, AIR_EINVAL, "coarse_n %d / level %d out of range", coarse_n, level);
  const int64_t R = (int64_t)coarse_n << level;
  if ((double)R * R > 4294967295.0) return fail(c, AIR_EINVAL, "raster exceeds 2^32 pixels per view");
  if (flux && !images) return fail(c, AIR_EINVAL, "flux needs the image buffer");
  if (!field->packed) return fail(c, AIR_EINVAL, "the allocation-free render needs a packed field (air_field_pack)");
  if (packed_too_large(grid, field)) return fail(c, AIR_ENOTSUP, "packed field: a copy exceeds 4 GiB");
  if (grid->kind == AIR_GRID_BLOCK_AMR && !blocks_known(c, grid, field->packed))
    return fail(c, AIR_EINVAL, "block tables not checked for this packed field: pack it with air_field_pack on "
                               "this context first");
  const int nb = field->kind == AIR_FIELD_RHO_J_KAPPA ? 1 : field->n_bands;
  const int64_t cpp = (R * R + CHUNK - 1) / CHUNK;
  const int64_t partial_bytes = 8 * (int64_t)n_views * nb * cpp;
  if (flux && partial_bytes > (int64_t)(NOALLOC_SCRATCH_BYTES - NOALLOC_PARTIAL_OFF))
    return fail(c, AIR_EINVAL, "flux partial sums of %lld bytes exceed the allocation-free workspace (%lld bytes)",
                (long long)partial_bytes, (long long)(NOALLOC_SCRATCH_BYTES - NOALLOC_PARTIAL_OFF));
  DevView hv[AIR_NOALLOC_MAX_VIEWS];
  for (int k = 0; k < n_views; ++k)
    if ((st = make_view(c, &views[k], hv[k]))) return st;
  if (!c->noalloc) return fail(c, AIR_EDEVICE, "allocation-free workspace unavailable on this device");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  unsigned char* ws = static_cast<unsigned char*>(c->noalloc);
  MarchArgs A;
  std::memset(&A, 0, sizeof A);
  fill_geo(grid, A.g);
  if (c->seg_shift_override >= 0) A.g.seg_shift = c->seg_shift_override;
  fill_fld(field, grid, A.f);
  A.img.N0 = coarse_n;
  A.img.Lmax = level;
  A.img.V = n_views;
  A.w.ctr = reinterpret_cast<unsigned long long*>(ws + NOALLOC_CTR_OFF);
  A.views = reinterpret_cast<const DevView*>(ws + NOALLOC_VIEWS_OFF);
  HIPCHK(c, launch_noalloc_setup(hv, n_views, ws, s));
  HIPCHK(c, launch_march_fixed(A, level, images, march_blocks(c, A.g.seg_shift), s));
  if (flux) {
    double* partial = reinterpret_cast<double*>(ws + NOALLOC_PARTIAL_OFF);
    for (int k = 0; k < n_views; ++k) {
      const double px = views[k].width / (double)R;
      HIPCHK(c, launch_fixed_flux(images + (size_t)k * (nb + 1) * R * R, 1, nb, R, px * px,
                                  partial + (size_t)k * nb * cpp, flux + (size_t)k * nb, s));
    }
  }
  return AIR_OK;
}

air_status air_trace_pixels(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* view,
                            int32_t coarse_n, int64_t n, const int32_t* level, const int32_t* ix,
                            const int32_t* iy, float* I, float* N, int32_t* visits, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  air_status st;
  if ((st = check_grid(c, grid))) return st;
  if ((st = check_field(c, field))) return st;
  if (!view) return fail(c, AIR_EINVAL, "view is NULL");
  if (coarse_n < 1 || n < 0) return fail(c, AIR_EINVAL, "coarse_n or n out of range");
  if (n > 0 && (!level || !ix || !iy || !I)) return fail(c, AIR_EINVAL, "level/ix/iy/I must not be NULL");
  if (n == 0) return AIR_OK;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_blocks(c, grid, s, field->packed))) return st;
  MarchArgs A;
  std::memset(&A, 0, sizeof A);
  fill_geo(grid, A.g);
  if (c->seg_shift_override >= 0) A.g.seg_shift = c->seg_shift_override;
  fill_fld(field, grid, A.f);
  A.img.N0 = coarse_n;
  A.img.V = 1;
  if ((st = upload_views(c, view, 1, s, &A.views))) return st;
  if ((st = ensure_packed(c, grid, field, A, s))) return st;
  HIPCHK(c, launch_trace_pixels(A, n, level, ix, iy, I, N, visits, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return AIR_OK;
}

int64_t air_field_packed_bytes(const air_grid* grid, const air_field* field) {
  air_status st;
  if ((st = check_grid(nullptr, grid))) return st;
  if ((st = check_field(nullptr, field))) return st;
  return packed_bytes_of(grid, field);
}

air_status air_field_pack(air_ctx* c, const air_grid* grid, const air_field* field, void* packed, int64_t bytes,
                          void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  air_status st;
  if ((st = check_grid(c, grid))) return st;
  if ((st = check_field(c, field))) return st;
  const int64_t need = packed_bytes_of(grid, field);
  if (!packed || bytes < need) return fail(c, AIR_EINVAL, "packed buffer of %lld bytes, %lld needed", (long long)bytes, (long long)need);
  if (packed_too_large(grid, field))
    return fail(c, AIR_ENOTSUP, "packed field of %lld bytes: a copy exceeds 4 GiB", (long long)need);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  if ((st = check_blocks(c, grid, (hipStream_t)stream))) return st;
  MarchArgs A;
  std::memset(&A, 0, sizeof A);
  fill_geo(grid, A.g);
  fill_fld(field, grid, A.f);
  HIPCHK(c, pack_any(A.g, A.f, packed, (hipStream_t)stream));
  if (grid->kind == AIR_GRID_BLOCK_AMR && !blocks_known(c, grid, packed)) {
    // this packed field and these tables: later calls skip the read-back
    auto& v = c->checked;
    v.erase(std::remove_if(v.begin(), v.end(), [&](const BlockSig& b) { return b.packed == packed; }), v.end());
    if (v.size() >= 64) v.erase(v.begin());
    v.push_back(sig_of(grid, packed));
  }
  return AIR_OK;
}

// ------------------------------------------------------------ learned proposal
air_status air_cnn_create(air_ctx* c, air_cnn** out) {
  if (!c || !out) return AIR_EINVAL;
  c->err.clear();
  *out = nullptr;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  air_cnn* n = new air_cnn;
  n->device = c->device;
  cnn::Net& N = n->net;
  const size_t P = AIR_CNN_PARAMS;
  bool ok = hipMalloc(&N.theta, 4 * P) == hipSuccess && hipMalloc(&N.m, 4 * P) == hipSuccess &&
            hipMalloc(&N.v, 4 * P) == hipSuccess && hipMalloc(&N.grad, 4 * P) == hipSuccess;
  const int csi[cnn::LAYERS] = {cnn::XC, cnn::HID, cnn::HID, cnn::HID};
  const int cso[cnn::LAYERS] = {cnn::HID, cnn::HID, cnn::HID, cnn::ZC};
  const int rows[cnn::LAYERS] = {cnn::HID, cnn::HID, cnn::HID, 16};
  for (int l = 0; ok && l < cnn::LAYERS; ++l) {
    ok = hipMalloc(&N.wf[l], 2 * (size_t)rows[l] * cnn::KPAD(csi[l])) == hipSuccess;
    if (ok && l > 0) ok = hipMalloc(&N.wt[l], 2 * (size_t)cnn::HID * cnn::KPAD(cso[l])) == hipSuccess;
  }
  if (ok)
    ok = hipMemset(N.theta, 0, 4 * P) == hipSuccess && hipMemset(N.m, 0, 4 * P) == hipSuccess &&
         hipMemset(N.v, 0, 4 * P) == hipSuccess && hipMemset(N.grad, 0, 4 * P) == hipSuccess &&
         cnn::prep_weights(N, nullptr) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    air_cnn_destroy(n);
    return fail(c, AIR_ENOMEM, "network allocation failed");
  }
  *out = n;
  return AIR_OK;
}

void air_cnn_destroy(air_cnn* n) {
  if (!n) return;
  (void)hipSetDevice(n->device);
  cnn::Net& N = n->net;
  for (float* p : {N.theta, N.m, N.v, N.grad})
    if (p) (void)hipFree(p);
  for (int l = 0; l < cnn::LAYERS; ++l) {
    if (N.wf[l]) (void)hipFree(N.wf[l]);
    if (N.wt[l]) (void)hipFree(N.wt[l]);
  }
  delete n;
}

air_status air_cnn_set(air_ctx* c, air_cnn* n, const float* params, const float* mean, const float* scale) {
  if (!c || !n) return AIR_EINVAL;
  c->err.clear();
  if (n->device != c->device) return fail(c, AIR_EINVAL, "network and context are on different devices");
  if (!params || !mean || !scale) return fail(c, AIR_EINVAL, "params, mean or scale is NULL");
  for (int k = 0; k < cnn::FEAT; ++k)
    if (!std::isfinite(mean[k]) || !std::isfinite(scale[k]) || !(scale[k] > 0))
      return fail(c, AIR_EINVAL, "feature mean must be finite and scale > 0");
  for (int k = 0; k < AIR_CNN_PARAMS; ++k)
    if (!std::isfinite(params[k])) return fail(c, AIR_EINVAL, "parameter %d not finite", k);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  cnn::Net& N = n->net;
  const size_t P = AIR_CNN_PARAMS;
  HIPCHK(c, hipMemcpy(N.theta, params, 4 * P, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemset(N.m, 0, 4 * P));
  HIPCHK(c, hipMemset(N.v, 0, 4 * P));
  HIPCHK(c, hipMemset(N.grad, 0, 4 * P));
  for (int k = 0; k < cnn::FEAT; ++k) {
    N.mean[k] = mean[k];
    N.stdv[k] = scale[k];
  }
  N.step = 0;
  HIPCHK(c, cnn::prep_weights(N, nullptr));
  HIPCHK(c, hipDeviceSynchronize());
  return AIR_OK;
}

air_status air_cnn_get(air_ctx* c, const air_cnn* n, float* params, float* mean, float* scale) {
  if (!c || !n) return AIR_EINVAL;
  c->err.clear();
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  if (params) {
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(params, n->net.theta, 4 * (size_t)AIR_CNN_PARAMS, hipMemcpyDeviceToHost));
  }
  for (int k = 0; k < cnn::FEAT; ++k) {
    if (mean) mean[k] = n->net.mean[k];
    if (scale) scale[k] = n->net.stdv[k];
  }
  return AIR_OK;
}

namespace {
air_status check_maps(air_ctx* c, const air_cnn* n, const float* feat, int32_t n_maps, int32_t h, int32_t w) {
  if (!n) return fail(c, AIR_EINVAL, "network is NULL");
  if (n->device != c->device) return fail(c, AIR_EINVAL, "network and context are on different devices");
  if (!feat) return fail(c, AIR_EINVAL, "features NULL");
  if (n_maps < 1 || h < 1 || w < 1 || (int64_t)n_maps * h * w >= ((int64_t)1 << 31) / 64)
    return fail(c, AIR_EINVAL, "map count or size out of range");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  return AIR_OK;
}

air_status cnn_forward_all(air_ctx* c, const air_cnn* n, const float* feat, int n_maps, int h, int w, float* z,
                           hipStream_t s) {
  const int64_t P = (int64_t)n_maps * h * w;
  const cnn::Net& N = n->net;
  HIPCHK(c, cnn::input_maps(feat, P, N.mean, N.stdv, (uint16_t*)c->cx0.p, s));
  HIPCHK(c, cnn::conv_forward(0, N, (const uint16_t*)c->cx0.p, n_maps, h, w, c->ca1.p, s));
  HIPCHK(c, cnn::conv_forward(1, N, (const uint16_t*)c->ca1.p, n_maps, h, w, c->ca2.p, s));
  HIPCHK(c, cnn::conv_forward(2, N, (const uint16_t*)c->ca2.p, n_maps, h, w, c->ca3.p, s));
  HIPCHK(c, cnn::conv_forward(3, N, (const uint16_t*)c->ca3.p, n_maps, h, w, z, s));
  return AIR_OK;
}
}  // namespace

air_status air_cnn_forward(air_ctx* c, air_cnn* n, const float* feat, int32_t n_maps, int32_t h, int32_t w,
                           float* logits, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  air_status st;
  if ((st = check_maps(c, n, feat, n_maps, h, w))) return st;
  if (!logits) return fail(c, AIR_EINVAL, "logits NULL");
  if ((st = ensure_cnn_work(c, (int64_t)n_maps * h * w, false))) return st;
  if ((st = cnn_forward_all(c, n, feat, n_maps, h, w, logits, (hipStream_t)stream))) return st;
  // the logits went to the caller's buffer: keep a copy beside the other
  // intermediates
  HIPCHK(c, hipMemcpyAsync(c->cz.p, logits, 4 * (size_t)cnn::ZC * n_maps * h * w, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
  c->cnn_pixels = (int64_t)n_maps * h * w;
  c->cnn_grads = false;
  return AIR_OK;
}

air_status air_cnn_tensor(air_ctx* c, int32_t which, void* out, int64_t bytes, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (c->cnn_pixels < 0) return fail(c, AIR_EINVAL, "no network call to inspect on this context");
  const int64_t P = c->cnn_pixels;
  const DevBuf* src = nullptr;
  int64_t need = 0;
  switch (which) {
    case AIR_CNN_T_X0: src = &c->cx0; need = 2 * cnn::XC * P; break;
    case AIR_CNN_T_A1: src = &c->ca1; need = 2 * cnn::HID * P; break;
    case AIR_CNN_T_A2: src = &c->ca2; need = 2 * cnn::HID * P; break;
    case AIR_CNN_T_A3: src = &c->ca3; need = 2 * cnn::HID * P; break;
    case AIR_CNN_T_Z: src = &c->cz; need = 4 * cnn::ZC * P; break;
    case AIR_CNN_T_DZ: src = &c->cdz; need = 2 * cnn::ZC * P; break;
    case AIR_CNN_T_D3: src = &c->cda; need = 2 * cnn::HID * P; break;
    case AIR_CNN_T_D2: src = &c->cdb; need = 2 * cnn::HID * P; break;
    case AIR_CNN_T_D1: src = &c->cdc; need = 2 * cnn::HID * P; break;
    default: return fail(c, AIR_EINVAL, "tensor %d unknown", which);
  }
  if (which >= AIR_CNN_T_DZ && !c->cnn_grads)
    return fail(c, AIR_EINVAL, "the last network call computed no gradients");
  if (!out || bytes < need) return fail(c, AIR_EINVAL, "output of %lld bytes, %lld needed", (long long)bytes, (long long)need);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  HIPCHK(c, hipMemcpyAsync(out, src->p, (size_t)need, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return AIR_OK;
}

air_status air_cnn_loss_grad(air_ctx* c, air_cnn* n, const float* feat, const int32_t* labels, int32_t n_maps,
                             int32_t h, int32_t w, const float* class_weight, double* loss, float* grad,
                             void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  air_status st;
  if ((st = check_maps(c, n, feat, n_maps, h, w))) return st;
  if (!labels || !class_weight) return fail(c, AIR_EINVAL, "labels or class weights NULL");
  for (int k = 0; k < cnn::CLASSES; ++k)
    if (!std::isfinite(class_weight[k]) || class_weight[k] < 0) return fail(c, AIR_EINVAL, "class weight %d invalid", k);
  const int64_t P = (int64_t)n_maps * h * w;
  if ((st = ensure_cnn_work(c, P, true))) return st;
  hipStream_t s = (hipStream_t)stream;
  cnn::Net& N = n->net;
  if ((st = cnn_forward_all(c, n, feat, n_maps, h, w, (float*)c->cz.p, s))) return st;
  HIPCHK(c, cnn::loss_and_dz((const float*)c->cz.p, labels, P, class_weight, (double*)c->closs_part.p,
                             (double*)c->closs.p, (uint16_t*)c->cdz.p, s));
  float* wp = (float*)c->cwpart.p;
  const uint16_t* cdz = (const uint16_t*)c->cdz.p;
  uint16_t* d3 = (uint16_t*)c->cda.p;  // gradient at the input of layer 3 (= at a3), and so on
  uint16_t* d2 = (uint16_t*)c->cdb.p;
  uint16_t* d1 = (uint16_t*)c->cdc.p;
  // back through layers 3..0: weight gradient from (dy, input), then the
  // input gradient masked by the input's ReLU
  HIPCHK(c, cnn::conv_weight_grad(3, N, cdz, (const uint16_t*)c->ca3.p, n_maps, h, w, wp, s));
  HIPCHK(c, cnn::conv_input_grad(3, N, cdz, (const uint16_t*)c->ca3.p, n_maps, h, w, d3, s));
  HIPCHK(c, cnn::conv_weight_grad(2, N, d3, (const uint16_t*)c->ca2.p, n_maps, h, w, wp, s));
  HIPCHK(c, cnn::conv_input_grad(2, N, d3, (const uint16_t*)c->ca2.p, n_maps, h, w, d2, s));
  HIPCHK(c, cnn::conv_weight_grad(1, N, d2, (const uint16_t*)c->ca1.p, n_maps, h, w, wp, s));
  HIPCHK(c, cnn::conv_input_grad(1, N, d2, (const uint16_t*)c->ca1.p, n_maps, h, w, d1, s));
  HIPCHK(c, cnn::conv_weight_grad(0, N, d1, (const uint16_t*)c->cx0.p, n_maps, h, w, wp, s));
  c->cnn_pixels = P;
  c->cnn_grads = true;
  if (grad) HIPCHK(c, hipMemcpyAsync(grad, N.grad, 4 * (size_t)AIR_CNN_PARAMS, hipMemcpyDeviceToDevice, s));
  if (loss) {
    double host[2];
    HIPCHK(c, hipMemcpyAsync(host, c->closs.p, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    *loss = host[1];
  }
  return AIR_OK;
}

air_status air_cnn_adam(air_ctx* c, air_cnn* n, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!n) return fail(c, AIR_EINVAL, "network is NULL");
  if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(c, AIR_EINVAL, "Adam hyper-parameters out of range");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(c, cnn::adam(n->net, AIR_CNN_PARAMS, lr, beta1, beta2, eps, s));
  HIPCHK(c, cnn::prep_weights(n->net, s));
  return AIR_OK;
}

air_status air_features(air_ctx* c, const air_grid* grid, const air_field* field, const air_view* views,
                        int32_t n_views, int32_t coarse_n, const float* band_weight, float* features, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  air_params prm;
  std::memset(&prm, 0, sizeof prm);
  prm.coarse_n = coarse_n;
  air_status st;
  if ((st = check_render_args(c, grid, field, views, n_views, &prm))) return st;
  if (!band_weight || !features) return fail(c, AIR_EINVAL, "band weights or features NULL");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_blocks(c, grid, s, field->packed))) return st;
  MarchArgs A;
  int64_t n_chunks = 0;
  if ((st = setup_render(c, grid, field, views, n_views, coarse_n, 0, true, s, A, n_chunks))) return st;
  LearnW W;
  for (int b = 0; b < MAXB; ++b) W.w[b] = b < A.f.nb ? band_weight[b] : 0.0f;
  HIPCHK(c, launch_init(A, s));
  HIPCHK(c, launch_march_queue(A, 0, march_blocks(c, A.g.seg_shift), s));
  HIPCHK(c, launch_features(A, W, features, s));
  return AIR_OK;
}

air_status air_tree_depth(air_ctx* c, const air_tree* tree, int32_t coarse_n, int32_t* depth, void* stream) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!tree || !depth || coarse_n < 1) return fail(c, AIR_EINVAL, "tree, depth or coarse_n invalid");
  if (tree->n_nodes < 0 || tree->n_nodes > tree->capacity) return fail(c, AIR_EINVAL, "tree n_nodes out of range");
  if (tree->n_nodes > 0 && (!tree->level || !tree->ix || !tree->iy))
    return fail(c, AIR_EINVAL, "tree level/ix/iy NULL");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(c, hipMemsetAsync(depth, 0, 4 * (size_t)coarse_n * coarse_n, s));
  if (tree->n_nodes > 0)
    HIPCHK(c, launch_tree_depth(tree->level, tree->ix, tree->iy, tree->n_nodes, coarse_n, depth, s));
  return AIR_OK;
}


// ---------------------------------------------------------------- checkpoints, tune cache, trees

namespace {
// network checkpoint: header, feature standardisation, parameters and the
// optimiser state, in native byte order
struct CnnFileHeader {
  char magic[8];
  int32_t n_params;
  int32_t n_features;
  int64_t step;
};
constexpr char CNN_MAGIC[8] = {'A', 'I', 'R', 'C', 'N', 'N', '0', '1'};
constexpr char TUNE_MAGIC[] = "libair-tune 1";

bool all_finite(const std::vector<float>& v, size_t b, size_t e) {
  for (size_t k = b; k < e; ++k)
    if (!std::isfinite(v[k])) return false;
  return true;
}
}  // namespace

air_status air_cnn_save(air_ctx* c, const air_cnn* n, const char* path) {
  if (!c || !n) return AIR_EINVAL;
  c->err.clear();
  if (!path) return fail(c, AIR_EINVAL, "path is NULL");
  if (n->device != c->device) return fail(c, AIR_EINVAL, "network and context are on different devices");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  const cnn::Net& N = n->net;
  const size_t P = AIR_CNN_PARAMS;
  std::vector<float> buf(3 * P);
  HIPCHK(c, hipDeviceSynchronize());
  HIPCHK(c, hipMemcpy(buf.data(), N.theta, 4 * P, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(buf.data() + P, N.m, 4 * P, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(buf.data() + 2 * P, N.v, 4 * P, hipMemcpyDeviceToHost));
  CnnFileHeader h;
  std::memcpy(h.magic, CNN_MAGIC, sizeof h.magic);
  h.n_params = AIR_CNN_PARAMS;
  h.n_features = cnn::FEAT;
  h.step = N.step;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(c, AIR_EINVAL, "cannot open %s for writing", path);
  bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 && std::fwrite(N.mean, 4, cnn::FEAT, f) == (size_t)cnn::FEAT &&
            std::fwrite(N.stdv, 4, cnn::FEAT, f) == (size_t)cnn::FEAT &&
            std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, AIR_EINVAL, "writing %s failed", path);
  return AIR_OK;
}

air_status air_cnn_load(air_ctx* c, air_cnn* n, const char* path) {
  if (!c || !n) return AIR_EINVAL;
  c->err.clear();
  if (!path) return fail(c, AIR_EINVAL, "path is NULL");
  if (n->device != c->device) return fail(c, AIR_EINVAL, "network and context are on different devices");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(c, AIR_EINVAL, "cannot open %s", path);
  const size_t P = AIR_CNN_PARAMS;
  CnnFileHeader h;
  float mean[cnn::FEAT], scale[cnn::FEAT];
  std::vector<float> buf(3 * P);
  bool ok = std::fread(&h, sizeof h, 1, f) == 1 && std::memcmp(h.magic, CNN_MAGIC, sizeof h.magic) == 0 &&
            h.n_params == AIR_CNN_PARAMS && h.n_features == cnn::FEAT && h.step >= 0 &&
            std::fread(mean, 4, cnn::FEAT, f) == (size_t)cnn::FEAT &&
            std::fread(scale, 4, cnn::FEAT, f) == (size_t)cnn::FEAT &&
            std::fread(buf.data(), 4, buf.size(), f) == buf.size();
  char extra;
  ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the optimiser state
  std::fclose(f);
  if (!ok) return fail(c, AIR_EINVAL, "%s is not a checkpoint of this network", path);
  for (int k = 0; k < cnn::FEAT; ++k)
    if (!std::isfinite(mean[k]) || !std::isfinite(scale[k]) || !(scale[k] > 0))
      return fail(c, AIR_EINVAL, "%s: feature mean must be finite and scale > 0", path);
  if (!all_finite(buf, 0, 3 * P)) return fail(c, AIR_EINVAL, "%s: parameters or moments not finite", path);
  for (size_t k = 2 * P; k < 3 * P; ++k)
    if (buf[k] < 0.0f) return fail(c, AIR_EINVAL, "%s: negative second moment", path);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  cnn::Net& N = n->net;
  HIPCHK(c, hipDeviceSynchronize());
  HIPCHK(c, hipMemcpy(N.theta, buf.data(), 4 * P, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(N.m, buf.data() + P, 4 * P, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(N.v, buf.data() + 2 * P, 4 * P, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemset(N.grad, 0, 4 * P));
  for (int k = 0; k < cnn::FEAT; ++k) {
    N.mean[k] = mean[k];
    N.stdv[k] = scale[k];
  }
  N.step = h.step;
  HIPCHK(c, cnn::prep_weights(N, nullptr));
  HIPCHK(c, hipDeviceSynchronize());
  return AIR_OK;
}

air_status air_tune_save(air_ctx* c, const char* path) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!path) return fail(c, AIR_EINVAL, "path is NULL");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "device query failed");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(c, AIR_EINVAL, "cannot open %s for writing", path);
  bool ok = std::fprintf(f, "%s %s %d\n", TUNE_MAGIC, prop.gcnArchName, c->num_cus) > 0;
  for (const auto& kv : c->tuned)
    ok = ok && std::fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.march_waves_per_cu,
                            kv.second.refine_blocks_per_cu) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, AIR_EINVAL, "writing %s failed", path);
  return AIR_OK;
}

air_status air_tune_load(air_ctx* c, const char* path) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!path) return fail(c, AIR_EINVAL, "path is NULL");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "device query failed");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(c, AIR_EINVAL, "cannot open %s", path);
  char line[512], arch[256];
  int cus = 0;
  const size_t ml = sizeof TUNE_MAGIC - 1;
  if (!std::fgets(line, sizeof line, f) || std::strncmp(line, TUNE_MAGIC, ml) != 0 ||
      std::sscanf(line + ml, " %255s %d", arch, &cus) != 2) {
    std::fclose(f);
    return fail(c, AIR_EINVAL, "%s is not a launch-shape cache", path);
  }
  if (std::strcmp(arch, prop.gcnArchName) != 0 || cus != c->num_cus) {
    std::fclose(f);
    return fail(c, AIR_EINVAL, "%s was tuned on %s with %d CUs, this device is %s with %d", path, arch, cus,
                prop.gcnArchName, c->num_cus);
  }
  // every entry is checked before any is taken
  std::map<std::string, Tune> got;
  char key[256];
  int mw = 0, rb = 0, lno = 1;
  while (std::fgets(line, sizeof line, f)) {
    ++lno;
    if (std::sscanf(line, "%255s %d %d", key, &mw, &rb) != 3 || !(mw == 8 || mw == 16 || mw == 32) ||
        !(rb == 2 || rb == 4 || rb == 8)) {
      std::fclose(f);
      return fail(c, AIR_EINVAL, "%s line %d: not an entry of launch shapes", path, lno);
    }
    Tune t;
    t.march_waves_per_cu = mw;
    t.refine_blocks_per_cu = rb;
    got[key] = t;
  }
  std::fclose(f);
  for (const auto& kv : got) c->tuned[kv.first] = kv.second;
  return AIR_OK;
}

air_status air_tree_free(air_ctx* c, air_tree* t) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!t) return fail(c, AIR_EINVAL, "tree is NULL");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  void* ptrs[] = {t->level, t->ix, t->iy, t->parent, t->first_child, t->state, t->I, t->N, t->xi_I, t->xi_N,
                  t->visits};
  hipError_t e = hipSuccess;
  for (void* q : ptrs)
    if (q) {
      const hipError_t r = hipFree(q);
      if (e == hipSuccess) e = r;
    }
  std::memset(t, 0, sizeof *t);
  if (e != hipSuccess) return fail(c, AIR_EDEVICE, "hipFree failed: %s", hipGetErrorString(e));
  return AIR_OK;
}

air_status air_tree_alloc(air_ctx* c, int32_t n_bands, int64_t capacity, air_tree* t) {
  if (!c) return AIR_EINVAL;
  c->err.clear();
  if (!t) return fail(c, AIR_EINVAL, "tree is NULL");
  if (n_bands < 1 || n_bands > AIR_MAX_BANDS) return fail(c, AIR_EINVAL, "n_bands %d out of range", n_bands);
  if (capacity < 1 || capacity >= ((int64_t)1 << 31)) return fail(c, AIR_EINVAL, "capacity out of range");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AIR_EDEVICE, "hipSetDevice failed");
  std::memset(t, 0, sizeof *t);
  const size_t n = (size_t)capacity;
  struct {
    void** p;
    size_t bytes;
  } arrays[] = {{(void**)&t->level, n},         {(void**)&t->ix, 4 * n},     {(void**)&t->iy, 4 * n},
                {(void**)&t->parent, 4 * n},    {(void**)&t->first_child, 4 * n},
                {(void**)&t->state, n},         {(void**)&t->I, 4 * n * n_bands},
                {(void**)&t->N, 4 * n},         {(void**)&t->xi_I, 4 * n},   {(void**)&t->xi_N, 4 * n},
                {(void**)&t->visits, 4 * n}};
  for (auto& a : arrays)
    if (hipMalloc(a.p, a.bytes) != hipSuccess) {
      (void)hipGetLastError();
      *a.p = nullptr;
      (void)air_tree_free(c, t);
      return fail(c, AIR_ENOMEM, "tree of %lld nodes does not fit", (long long)capacity);
    }
  t->capacity = capacity;
  return AIR_OK;
}

}  // extern "C"
