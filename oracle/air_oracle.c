/*
 * FP64 CPU oracle for adaptive image ray-tracing (AIR), after Parkin 2010,
 * "Adaptive image ray-tracing for astrophysical simulations" (MNRAS Letter).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no source, header or table with the HIP path.
 *
 * What it computes, step by step, in double precision:
 *   - view geometry and one ray through each pixel centre (paper section 2,
 *     step ii: "a ray for each respective pixel");
 *   - the exact formal solution of dI/ds = j - kappa*I and dN/ds = rho along
 *     that ray for cell-constant fields, found WITHOUT a DDA: every plane
 *     crossing of the finest grid spacing is collected, the three sorted
 *     per-axis lists are merged, and the cell holding each segment midpoint
 *     is located from scratch (uniform grid or block AMR, section 3 grid);
 *   - the truncation-error estimate of Eq. 2 / Eq. 3 (section 3), in the
 *     reading with bounded cross terms documented in the design notes;
 *   - the level-synchronous image refinement of section 2 steps ii-v: scan
 *     the tested pixels of one level, apply the 2:1 level rule between
 *     adjacent pixels (step iii) through a recursive closure, refine, trace
 *     the new pixels, repeat until nothing refines or the level cap;
 *   - output (step vi): a raster painted from the leaves, and the broadband
 *     flux sum over leaves of pixel area times intensity (Table 1 caption).
 *
 * Sums use Neumaier compensation.  Per-level node maps are dense row-major
 * (index j*R + i), levels concatenated in order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXB 1024
#define ORC_MAXL 16

/* node state bits */
#define ORC_EXIST 1u
#define ORC_TESTED 2u   /* created by the criterion (or level 0): eligible for the test */
#define ORC_FLAGGED 4u  /* the test asked for refinement */
#define ORC_BALANCE 8u  /* created only to keep the 2:1 rule */
#define ORC_REFINED 16u /* has four children */

typedef struct {
  int32_t kind; /* 0 uniform, 1 block AMR */
  int32_t n[3]; /* uniform: cells per axis.  AMR: base blocks per axis */
  double lo[3], hi[3];
  int32_t bs;        /* AMR: cells per block edge */
  int32_t max_level; /* AMR: deepest block level */
  int32_t n_blocks;
  const int32_t* blevel; /* [n_blocks] */
  const int32_t* bcoord; /* [n_blocks][3] block coordinate at its own level */
  const int32_t* bchild; /* [n_blocks] first of 8 children (x fastest) or -1 */
} orc_grid;

typedef struct {
  int32_t kind; /* 0: rho, emissivity, opacity (one band).  1: rho, T, power-law bands.
                   2: rho, T, spectral bins */
  int32_t n_bands;
  const float* rho;
  const float* emis;
  const float* kappa;
  const float* temp;
  /* kind 1: [n_bands][3] = kappa0, s, q : kappa = kappa0 rho T^-s, j = rho^2 T^q.
     kind 2: [n_bands][5] = kappa0, s, e0, q, E : kappa = kappa0 rho T^-s,
             j = e0 rho^2 T^q exp(-E / T) */
  const double* band;
} orc_field;

typedef struct {
  double dir[3], up[3], center[3], width;
} orc_view;

typedef struct {
  double I[ORC_MAXB];
  double N;
  double rho_min, rho_max;
  int32_t lmax; /* finest grid level crossed, -1 for a miss */
  int32_t nvis; /* number of distinct consecutive cells visited */
} orc_ray;

/* ---------------------------------------------------------------- sums */
typedef struct {
  double s, c;
} nsum;

static void nadd(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------ geometry */
/* Image basis: e_u = normalise(up x d), e_v = d x e_u; d is the looking
 * direction, so rays run front to back from the observer along +d. */
static void view_basis(const orc_view* v, double d[3], double eu[3], double ev[3]) {
  double nd = sqrt(v->dir[0] * v->dir[0] + v->dir[1] * v->dir[1] + v->dir[2] * v->dir[2]);
  for (int a = 0; a < 3; ++a) d[a] = v->dir[a] / nd;
  double u[3] = {v->up[1] * d[2] - v->up[2] * d[1], v->up[2] * d[0] - v->up[0] * d[2],
                 v->up[0] * d[1] - v->up[1] * d[0]};
  double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (int a = 0; a < 3; ++a) eu[a] = u[a] / nu;
  ev[0] = d[1] * eu[2] - d[2] * eu[1];
  ev[1] = d[2] * eu[0] - d[0] * eu[2];
  ev[2] = d[0] * eu[1] - d[1] * eu[0];
}

/* centre of pixel (L, i, j): i counts along e_u, j along e_v */
static void pixel_center(const orc_view* v, const double eu[3], const double ev[3], int N0, int L,
                         int i, int j, double c[3]) {
  double s = v->width / (double)((int64_t)N0 << L);
  double au = -0.5 * v->width + ((double)i + 0.5) * s;
  double av = -0.5 * v->width + ((double)j + 0.5) * s;
  for (int a = 0; a < 3; ++a) c[a] = v->center[a] + au * eu[a] + av * ev[a];
}

/* ------------------------------------------------------ point location */
static int64_t fine_cells(const orc_grid* g, int a) {
  if (g->kind == 0) return g->n[a];
  return (int64_t)g->n[a] * g->bs << g->max_level;
}

/* Cell holding point x: data index and grid level.  Half-open cells:
 * floor rule, clamped against the exit rounding only. */
static int64_t locate(const orc_grid* g, const double x[3], int* level) {
  int64_t F[3];
  for (int a = 0; a < 3; ++a) {
    int64_t nf = fine_cells(g, a);
    double h = (g->hi[a] - g->lo[a]) / (double)nf;
    int64_t k = (int64_t)floor((x[a] - g->lo[a]) / h);
    if (k < 0) k = 0;
    if (k > nf - 1) k = nf - 1;
    F[a] = k;
  }
  if (g->kind == 0) {
    *level = 0;
    return F[0] + (int64_t)g->n[0] * (F[1] + (int64_t)g->n[1] * F[2]);
  }
  const int mL = g->max_level, bs = g->bs;
  int64_t bc[3];
  for (int a = 0; a < 3; ++a) bc[a] = (F[a] >> mL) / bs;
  int64_t b = bc[0] + (int64_t)g->n[0] * (bc[1] + (int64_t)g->n[1] * bc[2]);
  int l = 0;
  while (g->bchild[b] >= 0) {
    ++l;
    int off = 0;
    for (int a = 0; a < 3; ++a) {
      int64_t cb = (F[a] >> (mL - l)) / bs; /* block coordinate at level l */
      int64_t c = cb - 2 * (int64_t)g->bcoord[3 * b + a];
      off |= (int)c << a;
    }
    b = g->bchild[b] + off;
  }
  int64_t cc[3];
  for (int a = 0; a < 3; ++a) cc[a] = (F[a] >> (mL - l)) - (int64_t)bs * g->bcoord[3 * b + a];
  *level = l;
  return b * (int64_t)bs * bs * bs + cc[0] + bs * (cc[1] + (int64_t)bs * cc[2]);
}

/* ------------------------------------------------------------- the ray */
/* f(x) = (1 - e^-x)/x, the exact weight of a constant-source segment */
static double seg_weight(double x) { return x == 0.0 ? 1.0 : -expm1(-x) / x; }

static void cell_optics(const orc_field* f, int64_t idx, double* rho, double* jb, double* kb) {
  double r = (double)f->rho[idx];
  *rho = r;
  if (f->kind == 0) {
    jb[0] = (double)f->emis[idx];
    kb[0] = (double)f->kappa[idx];
  } else if (f->kind == 1) {
    double T = (double)f->temp[idx];
    for (int b = 0; b < f->n_bands; ++b) {
      kb[b] = f->band[3 * b + 0] * r * pow(T, -f->band[3 * b + 1]);
      jb[b] = r * r * pow(T, f->band[3 * b + 2]);
    }
  } else {
    double T = (double)f->temp[idx];
    for (int b = 0; b < f->n_bands; ++b) {
      const double* q = f->band + 5 * b;
      kb[b] = q[0] * r * pow(T, -q[1]);
      jb[b] = q[2] * r * r * pow(T, q[3]) * exp(-q[4] / T);
    }
  }
}

/* work must hold 3 * (max fine cells + 1) doubles */
static void trace_ray(const orc_grid* g, const orc_field* f, const double o[3], const double d[3],
                      double* work, orc_ray* r) {
  memset(r, 0, sizeof *r);
  r->lmax = -1;
  const int nb = f->kind == 0 ? 1 : f->n_bands;
  double t0 = -INFINITY, t1 = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0) {
      double ta = (g->lo[a] - o[a]) / d[a], tb = (g->hi[a] - o[a]) / d[a];
      t0 = fmax(t0, fmin(ta, tb));
      t1 = fmin(t1, fmax(ta, tb));
    } else if (!(o[a] >= g->lo[a] && o[a] < g->hi[a])) {
      return; /* parallel to this slab and outside it */
    }
  }
  if (!(t0 < t1)) return;

  /* every crossing of a finest-spacing plane strictly inside (t0, t1) */
  double* lst[3];
  int64_t cnt[3] = {0, 0, 0};
  int64_t maxn = 0;
  for (int a = 0; a < 3; ++a)
    if (fine_cells(g, a) + 1 > maxn) maxn = fine_cells(g, a) + 1;
  for (int a = 0; a < 3; ++a) {
    lst[a] = work + a * maxn;
    if (d[a] == 0.0) continue;
    int64_t nf = fine_cells(g, a);
    double h = (g->hi[a] - g->lo[a]) / (double)nf;
    for (int64_t m = 0; m <= nf; ++m) {
      int64_t mm = d[a] > 0 ? m : nf - m; /* ascending t */
      double t = (g->lo[a] + (double)mm * h - o[a]) / d[a];
      if (t > t0 && t < t1) lst[a][cnt[a]++] = t;
    }
  }

  nsum I[ORC_MAXB], tau[ORC_MAXB], N = {0, 0};
  memset(I, 0, sizeof I);
  memset(tau, 0, sizeof tau);
  double jb[ORC_MAXB], kb[ORC_MAXB];
  int64_t p[3] = {0, 0, 0};
  double ta = t0;
  int64_t prev = -1;
  int nvis = 0, lmax = -1;
  double rmin = INFINITY, rmax = -INFINITY;
  for (;;) {
    /* next event: the smallest remaining crossing, or the exit */
    double tb = t1;
    int ax = -1;
    for (int a = 0; a < 3; ++a)
      if (p[a] < cnt[a] && lst[a][p[a]] < tb) {
        tb = lst[a][p[a]];
        ax = a;
      }
    double ds = tb - ta;
    if (ds > 0.0) {
      double tm = 0.5 * (ta + tb), x[3];
      for (int a = 0; a < 3; ++a) x[a] = o[a] + tm * d[a];
      int lev;
      int64_t idx = locate(g, x, &lev);
      double rho;
      cell_optics(f, idx, &rho, jb, kb);
      for (int b = 0; b < nb; ++b) {
        double dt = kb[b] * ds;
        nadd(&I[b], exp(-nval(&tau[b])) * jb[b] * ds * seg_weight(dt));
        nadd(&tau[b], dt);
      }
      nadd(&N, rho * ds);
      if (idx != prev) ++nvis;
      prev = idx;
      if (lev > lmax) lmax = lev;
      if (rho < rmin) rmin = rho;
      if (rho > rmax) rmax = rho;
    }
    if (ax < 0) break;
    ++p[ax];
    ta = tb;
  }
  for (int b = 0; b < nb; ++b) r->I[b] = nval(&I[b]);
  r->N = nval(&N);
  r->nvis = nvis;
  r->lmax = lmax;
  r->rho_min = nvis ? rmin : 0.0;
  r->rho_max = nvis ? rmax : 0.0;
}

static int64_t work_len(const orc_grid* g) {
  int64_t m = 0;
  for (int a = 0; a < 3; ++a)
    if (fine_cells(g, a) + 1 > m) m = fine_cells(g, a) + 1;
  return 3 * m;
}

/* ------------------------------------------------------ public: rays */
/* Trace one ray with origin o and direction d (need not be unit). */
void orc_trace(const orc_grid* g, const orc_field* f, const double o[3], const double dir[3],
               orc_ray* out) {
  double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  double d[3] = {dir[0] / nd, dir[1] / nd, dir[2] / nd};
  double* work = (double*)malloc(sizeof(double) * work_len(g));
  trace_ray(g, f, o, d, work, out);
  free(work);
}

void orc_view_basis(const orc_view* v, double d[3], double eu[3], double ev[3]) {
  view_basis(v, d, eu, ev);
}

void orc_pixel_center(const orc_view* v, int N0, int L, int i, int j, double c[3]) {
  double d[3], eu[3], ev[3];
  view_basis(v, d, eu, ev);
  pixel_center(v, eu, ev, N0, L, i, j, c);
}

/* Trace n individual pixels (L[k], i[k], j[k]).  I is [n_bands][n]. */
void orc_trace_pixels(const orc_grid* g, const orc_field* f, const orc_view* v, int N0, int64_t n,
                      const int32_t* L, const int32_t* pi, const int32_t* pj, double* I, double* N,
                      int32_t* lmax, int32_t* nvis, double* rmin, double* rmax) {
  double d[3], eu[3], ev[3];
  view_basis(v, d, eu, ev);
  const int nb = f->kind == 0 ? 1 : f->n_bands;
  const int64_t wl = work_len(g);
#pragma omp parallel
  {
    double* work = (double*)malloc(sizeof(double) * wl);
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
      double c[3];
      orc_ray r;
      pixel_center(v, eu, ev, N0, L[k], pi[k], pj[k], c);
      trace_ray(g, f, c, d, work, &r);
      for (int b = 0; b < nb; ++b) I[(int64_t)b * n + k] = r.I[b];
      N[k] = r.N;
      if (lmax) lmax[k] = r.lmax;
      if (nvis) nvis[k] = r.nvis;
      if (rmin) rmin[k] = r.rho_min;
      if (rmax) rmax[k] = r.rho_max;
    }
    free(work);
  }
}

/* Fixed-resolution image at level L: R = N0 * 2^L, outputs row-major j*R+i,
 * I as [n_bands][R*R]. */
void orc_render_fixed(const orc_grid* g, const orc_field* f, const orc_view* v, int N0, int L,
                      double* I, double* N, int32_t* lmax, int32_t* nvis) {
  double d[3], eu[3], ev[3];
  view_basis(v, d, eu, ev);
  const int nb = f->kind == 0 ? 1 : f->n_bands;
  const int64_t R = (int64_t)N0 << L, n = R * R;
  const int64_t wl = work_len(g);
#pragma omp parallel
  {
    double* work = (double*)malloc(sizeof(double) * wl);
#pragma omp for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
      double c[3];
      orc_ray r;
      pixel_center(v, eu, ev, N0, L, (int)(k % R), (int)(k / R), c);
      trace_ray(g, f, c, d, work, &r);
      for (int b = 0; b < nb; ++b) I[(int64_t)b * n + k] = r.I[b];
      N[k] = r.N;
      if (lmax) lmax[k] = r.lmax;
      if (nvis) nvis[k] = r.nvis;
    }
    free(work);
  }
}

/* ------------------------------------------------------- the criterion */
/* Truncation-error estimate at a pixel from its 3x3 same-level stencil
 * p[(b+1)*3 + (a+1)] = value at offset (a, b), a along u, b along v.
 * hx / hy say whether both u / v neighbours lie inside the image; a
 * direction without them contributes no term and drops the cross terms.
 * Numerator: squared second differences, the mixed one counted for both
 * orderings (Eq. 3 sums over all u,v).  Denominator: squared sums of the
 * absolute forward and backward first differences (Eq. 2 in each
 * direction); for the mixed pair, the first differences along one
 * direction taken at the two offsets of the other, scaled like the mixed
 * numerator.  A flat stencil (zero denominator) gives 0. */
double orc_xi(const double* p, int hx, int hy) {
#define P(a, b) p[((b) + 1) * 3 + ((a) + 1)]
  double num = 0.0, den = 0.0;
  if (hx) {
    double n = P(1, 0) - 2.0 * P(0, 0) + P(-1, 0);
    double dd = fabs(P(1, 0) - P(0, 0)) + fabs(P(0, 0) - P(-1, 0));
    num += n * n;
    den += dd * dd;
  }
  if (hy) {
    double n = P(0, 1) - 2.0 * P(0, 0) + P(0, -1);
    double dd = fabs(P(0, 1) - P(0, 0)) + fabs(P(0, 0) - P(0, -1));
    num += n * n;
    den += dd * dd;
  }
  if (hx && hy) {
    double nxy = 0.25 * (P(1, 1) - P(-1, 1) - P(1, -1) + P(-1, -1));
    double dxy = 0.25 * (fabs(P(1, 1) - P(-1, 1)) + fabs(P(1, -1) - P(-1, -1)));
    double dyx = 0.25 * (fabs(P(1, 1) - P(1, -1)) + fabs(P(-1, 1) - P(-1, -1)));
    num += 2.0 * nxy * nxy;
    den += dxy * dxy + dyx * dyx;
  }
#undef P
  if (den == 0.0) return 0.0;
  return sqrt(num / den);
}

/* ------------------------------------------------------------ the tree */
typedef struct {
  int N0, Lmax, nb;
  int64_t off[ORC_MAXL + 2];
  uint8_t* state;
  double *xiI, *xiN, *I, *N, *rmin, *rmax;
  int32_t *lmax, *nvis;
  int64_t total;
  const uint8_t* force_flags; /* test hook: flags per position instead of the criterion */
  int8_t* born;               /* step that created each node (-1: base image), may be NULL */
  int step;
  int64_t *nl, *nl_i, *nl_j;  /* list of nodes created in the current step */
  int64_t n_new, cap_new;
  int err;
} tree_t;

static int64_t R_of(const tree_t* t, int L) { return (int64_t)t->N0 << L; }
static int64_t pos(const tree_t* t, int L, int64_t i, int64_t j) {
  return t->off[L] + j * R_of(t, L) + i;
}

static void push_new(tree_t* t, int L, int64_t i, int64_t j) {
  if (t->n_new == t->cap_new) {
    t->cap_new = t->cap_new ? 2 * t->cap_new : 1024;
    t->nl = (int64_t*)realloc(t->nl, sizeof(int64_t) * t->cap_new);
    t->nl_i = (int64_t*)realloc(t->nl_i, sizeof(int64_t) * t->cap_new);
    t->nl_j = (int64_t*)realloc(t->nl_j, sizeof(int64_t) * t->cap_new);
  }
  t->nl[t->n_new] = L;
  t->nl_i[t->n_new] = i;
  t->nl_j[t->n_new] = j;
  ++t->n_new;
}

static void refine(tree_t* t, int L, int64_t i, int64_t j, uint8_t kind) {
  t->state[pos(t, L, i, j)] |= ORC_REFINED;
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) {
      t->state[pos(t, L + 1, 2 * i + a, 2 * j + b)] |= (uint8_t)(ORC_EXIST | kind);
      if (t->born) t->born[pos(t, L + 1, 2 * i + a, 2 * j + b)] = (int8_t)t->step;
      push_new(t, L + 1, 2 * i + a, 2 * j + b);
    }
}

/* Make node (L, i, j) exist: its parent must be refined, and before that
 * the parent's own eight neighbours must exist, recursively (2:1 rule with
 * edge and corner adjacency). */
static void ensure(tree_t* t, int L, int64_t i, int64_t j) {
  if (t->state[pos(t, L, i, j)] & ORC_EXIST) return;
  if (L == 0) { /* every base pixel exists: unreachable in a valid tree */
    t->err = 1;
    return;
  }
  int64_t Pi = i >> 1, Pj = j >> 1, R1 = R_of(t, L - 1);
  if (!(t->state[pos(t, L - 1, Pi, Pj)] & ORC_EXIST)) {
    t->err = 2;
    return;
  }
  for (int db = -1; db <= 1; ++db)
    for (int da = -1; da <= 1; ++da) {
      if (!da && !db) continue;
      int64_t qi = Pi + da, qj = Pj + db;
      if (qi < 0 || qj < 0 || qi >= R1 || qj >= R1) continue;
      ensure(t, L - 1, qi, qj);
    }
  refine(t, L - 1, Pi, Pj, ORC_BALANCE);
}

static void trace_new(tree_t* t, const orc_grid* g, const orc_field* f, const orc_view* v) {
  if (!g) return; /* structure-only mode */
  double d[3], eu[3], ev[3];
  view_basis(v, d, eu, ev);
  const int64_t wl = work_len(g);
  const int nb = t->nb;
#pragma omp parallel
  {
    double* work = (double*)malloc(sizeof(double) * wl);
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < t->n_new; ++k) {
      int L = (int)t->nl[k];
      double c[3];
      orc_ray r;
      pixel_center(v, eu, ev, t->N0, L, (int)t->nl_i[k], (int)t->nl_j[k], c);
      trace_ray(g, f, c, d, work, &r);
      int64_t p = pos(t, L, t->nl_i[k], t->nl_j[k]);
      for (int b = 0; b < nb; ++b) t->I[(int64_t)b * t->total + p] = r.I[b];
      t->N[p] = r.N;
      if (t->lmax) t->lmax[p] = r.lmax;
      if (t->nvis) t->nvis[p] = r.nvis;
      if (t->rmin) t->rmin[p] = r.rho_min;
      if (t->rmax) t->rmax[p] = r.rho_max;
    }
    free(work);
  }
}

/* value used in a level-L stencil at (i, j): the level-L node if it
 * exists, else the covering level-(L-1) node */
static double stencil_value(const tree_t* t, int L, int64_t i, int64_t j, int which,
                            const double* w) {
  int64_t p = pos(t, L, i, j);
  if (!(t->state[p] & ORC_EXIST)) p = pos(t, L - 1, i >> 1, j >> 1);
  if (which == 1) return t->N[p];
  double s = 0.0;
  for (int b = 0; b < t->nb; ++b) s += (w ? w[b] : 1.0) * t->I[(int64_t)b * t->total + p];
  return s;
}

/*
 * Plain AIR for one view.  Arrays are dense per level (row-major j*R+i),
 * levels concatenated; total = sum_L (N0*2^L)^2.  I is [n_bands][total].
 * xiI / xiN are NaN where the criterion was not evaluated.  lmax, nvis,
 * rmin, rmax may be NULL.  force_flags (test hook, may be NULL): when
 * given, a tested node is flagged iff force_flags[pos] != 0 and no ray is
 * traced (grid and field may then be NULL).
 * Returns the number of nodes (rays traced), or a negative error.
 * counts[L] receives the node count per level; born (may be NULL) the step
 * that created each node (-1 for the base image).
 */
int64_t orc_air(const orc_grid* g, const orc_field* f, const orc_view* v, int N0, int Lmax,
                double xc_I, double xc_N, const double* band_w, const uint8_t* force_flags,
                uint8_t* state, double* xiI, double* xiN, double* I, double* N, int32_t* lmax,
                int32_t* nvis, double* rmin, double* rmax, int64_t* counts, int8_t* born) {
  if (N0 < 1 || Lmax < 0 || Lmax > ORC_MAXL - 1) return -1;
  tree_t t;
  memset(&t, 0, sizeof t);
  t.N0 = N0;
  t.Lmax = Lmax;
  t.nb = f ? (f->kind == 0 ? 1 : f->n_bands) : 1;
  t.off[0] = 0;
  for (int L = 0; L <= Lmax; ++L) t.off[L + 1] = t.off[L] + R_of(&t, L) * R_of(&t, L);
  t.total = t.off[Lmax + 1];
  t.state = state;
  t.xiI = xiI;
  t.xiN = xiN;
  t.I = I;
  t.N = N;
  t.lmax = lmax;
  t.nvis = nvis;
  t.rmin = rmin;
  t.rmax = rmax;
  t.force_flags = force_flags;
  t.born = born;
  memset(state, 0, (size_t)t.total);
  if (born) memset(born, -1, (size_t)t.total);
  for (int64_t k = 0; k < t.total; ++k) {
    xiI[k] = NAN;
    xiN[k] = NAN;
  }

  /* step i: base image, every pixel traced and tested */
  int64_t R0 = R_of(&t, 0);
  for (int64_t j = 0; j < R0; ++j)
    for (int64_t i = 0; i < R0; ++i) {
      state[pos(&t, 0, i, j)] = ORC_EXIST | ORC_TESTED;
      push_new(&t, 0, i, j);
    }
  trace_new(&t, force_flags ? NULL : g, f, v);
  int64_t nodes = t.n_new;

  uint8_t* flag = NULL;
  for (int L = 0; L < Lmax; ++L) {
    int64_t R = R_of(&t, L);
    flag = (uint8_t*)realloc(flag, (size_t)(R * R));
    int64_t nflag = 0;
    /* step iii: every xi of this level before any change to the tree */
#pragma omp parallel for schedule(static) reduction(+ : nflag)
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i) {
        int64_t p = pos(&t, L, i, j);
        flag[j * R + i] = 0;
        if (!(state[p] & ORC_TESTED)) continue;
        int hx = i > 0 && i < R - 1, hy = j > 0 && j < R - 1;
        double s[9], sN[9];
        for (int b = -1; b <= 1; ++b)
          for (int a = -1; a <= 1; ++a) {
            int64_t qi = i + a, qj = j + b;
            int k = (b + 1) * 3 + (a + 1);
            if (qi < 0 || qj < 0 || qi >= R || qj >= R) {
              s[k] = sN[k] = 0.0; /* never read: that direction is dropped */
              continue;
            }
            s[k] = stencil_value(&t, L, qi, qj, 0, band_w);
            sN[k] = stencil_value(&t, L, qi, qj, 1, band_w);
          }
        double x1 = orc_xi(s, hx, hy), x2 = orc_xi(sN, hx, hy);
        xiI[p] = x1;
        xiN[p] = x2;
        int fl = force_flags ? (force_flags[p] != 0) : (x1 >= xc_I || x2 >= xc_N);
        flag[j * R + i] = (uint8_t)fl;
        nflag += fl;
      }
    if (nflag == 0) break;
    t.n_new = 0;
    t.step = L;
    /* steps iii-iv: 2:1 closure around every flagged pixel, then refine */
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i) {
        if (!flag[j * R + i]) continue;
        for (int db = -1; db <= 1; ++db)
          for (int da = -1; da <= 1; ++da) {
            if (!da && !db) continue;
            int64_t qi = i + da, qj = j + db;
            if (qi < 0 || qj < 0 || qi >= R || qj >= R) continue;
            ensure(&t, L, qi, qj);
          }
      }
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i)
        if (flag[j * R + i]) {
          state[pos(&t, L, i, j)] |= ORC_FLAGGED;
          refine(&t, L, i, j, ORC_TESTED);
        }
    if (t.err) break;
    /* step ii again: trace everything new before the next level */
    trace_new(&t, force_flags ? NULL : g, f, v);
    nodes += t.n_new;
  }
  free(flag);
  free(t.nl);
  free(t.nl_i);
  free(t.nl_j);
  if (t.err) return -10 - t.err;
  if (counts)
    for (int L = 0; L <= Lmax; ++L) {
      int64_t c = 0;
      for (int64_t p = t.off[L]; p < t.off[L + 1]; ++p) c += (state[p] & ORC_EXIST) != 0;
      counts[L] = c;
    }
  return nodes;
}

/* ----------------------------------------------------------- output */
/* Paint every leaf over its square of the finest raster (R = N0*2^Lmax).
 * vals is one per-node array of length total; out is R*R row-major. */
void orc_paint_leaves(int N0, int Lmax, const uint8_t* state, const double* vals, double* out) {
  int64_t off = 0, Rf = (int64_t)N0 << Lmax;
  for (int L = 0; L <= Lmax; ++L) {
    int64_t R = (int64_t)N0 << L, sc = (int64_t)1 << (Lmax - L);
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i) {
        uint8_t s = state[off + j * R + i];
        if (!(s & ORC_EXIST) || (s & ORC_REFINED)) continue;
        double val = vals[off + j * R + i];
        for (int64_t y = j * sc; y < (j + 1) * sc; ++y)
          for (int64_t x = i * sc; x < (i + 1) * sc; ++x) out[y * Rf + x] = val;
      }
    off += R * R;
  }
}

/* Super-resolution output (section 2 step vi suggests interpolating between
 * neighbouring pixels whose levels differ; the cited method is not given, so
 * this is the reading stated in the design notes): every pixel of the finest
 * raster lying in a level-L leaf takes the bilinear interpolation, at its
 * centre, of the level-L point samples around it.  A level-L sample at
 * (i, j) is the value of the level-L node if it exists in the final tree,
 * otherwise of the level-(L-1) node covering that position (the 2:1 rule
 * makes it exist for the neighbours of a leaf); positions beyond the image
 * edge take the nearest edge position.  Level-L coordinates of a finest pixel
 * x: u = (x + 1/2) / 2^(Lmax-L) - 1/2 (sample i sits at u = i). */
static double sample_value(int N0, const int64_t* off, const uint8_t* state, const double* vals, int L,
                           int64_t i, int64_t j) {
  const int64_t R = (int64_t)N0 << L;
  if (i < 0) i = 0;
  if (j < 0) j = 0;
  if (i > R - 1) i = R - 1;
  if (j > R - 1) j = R - 1;
  const int64_t p = off[L] + j * R + i;
  if ((state[p] & ORC_EXIST) || L == 0) return vals[p];
  return vals[off[L - 1] + (j >> 1) * (R >> 1) + (i >> 1)];
}

void orc_superres(int N0, int Lmax, const uint8_t* state, const double* vals, double* out) {
  int64_t off[ORC_MAXL + 2];
  off[0] = 0;
  for (int L = 0; L <= Lmax; ++L) off[L + 1] = off[L] + ((int64_t)N0 << L) * ((int64_t)N0 << L);
  const int64_t Rf = (int64_t)N0 << Lmax;
  for (int L = 0; L <= Lmax; ++L) {
    const int64_t R = (int64_t)N0 << L, sc = (int64_t)1 << (Lmax - L);
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i) {
        const uint8_t s = state[off[L] + j * R + i];
        if (!(s & ORC_EXIST) || (s & ORC_REFINED)) continue;
        for (int64_t y = j * sc; y < (j + 1) * sc; ++y)
          for (int64_t x = i * sc; x < (i + 1) * sc; ++x) {
            const double u = ((double)x + 0.5) / (double)sc - 0.5, v = ((double)y + 0.5) / (double)sc - 0.5;
            const int64_t i0 = (int64_t)floor(u), j0 = (int64_t)floor(v);
            const double fu = u - (double)i0, fv = v - (double)j0;
            const double a = sample_value(N0, off, state, vals, L, i0, j0);
            const double b = sample_value(N0, off, state, vals, L, i0 + 1, j0);
            const double c = sample_value(N0, off, state, vals, L, i0, j0 + 1);
            const double d = sample_value(N0, off, state, vals, L, i0 + 1, j0 + 1);
            out[y * Rf + x] = (1.0 - fu) * (1.0 - fv) * a + fu * (1.0 - fv) * b + (1.0 - fu) * fv * c + fu * fv * d;
          }
      }
  }
}

/* Flux: sum over leaves of (pixel area) * value, Neumaier-compensated. */
double orc_leaf_flux(int N0, int Lmax, double width, const uint8_t* state, const double* vals) {
  nsum s = {0, 0};
  int64_t off = 0;
  for (int L = 0; L <= Lmax; ++L) {
    int64_t R = (int64_t)N0 << L;
    double px = width / (double)R, area = px * px;
    for (int64_t k = 0; k < R * R; ++k) {
      uint8_t st = state[off + k];
      if ((st & ORC_EXIST) && !(st & ORC_REFINED)) nadd(&s, area * vals[off + k]);
    }
    off += R * R;
  }
  return nval(&s);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of later parallel regions (n >= 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------- parity-test helper */
/* First-order bound on how far xi can move when each stencil value p_k
 * moves by a relative amount delta (the value tolerance of a float32
 * evaluation): sum over k of the larger change of xi under p_k -> p_k (1 +-
 * delta).  A flag decided by a float32 path can differ from this oracle's
 * only where |xi - xi_crit| is within this bound.  p is [n][9]; the result
 * is written to out[n]. */
void orc_xi_sens(int64_t n, const double* p, const int32_t* hx, const int32_t* hy, double delta, double* xi,
                 double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    double q[9];
    memcpy(q, p + 9 * k, sizeof q);
    double x0 = orc_xi(q, hx[k], hy[k]), s = 0.0;
    for (int m = 0; m < 9; ++m) {
      double v = q[m], h = fabs(v) * delta, worst = 0.0;
      q[m] = v + h;
      worst = fmax(worst, fabs(orc_xi(q, hx[k], hy[k]) - x0));
      q[m] = v - h;
      worst = fmax(worst, fabs(orc_xi(q, hx[k], hy[k]) - x0));
      q[m] = v;
      s += worst;
    }
    xi[k] = x0;
    out[k] = s;
  }
}
