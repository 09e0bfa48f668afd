"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host only): a driver that includes air_oracle.c runs its entry points on a
small uniform grid and a small block-AMR hierarchy, and must finish without a
report (any report aborts it: -fno-sanitize-recover)."""
import os
import shutil
import subprocess

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

DRIVER = r"""
#include <stdio.h>

#include "air_oracle.c"

static int64_t total_of(int N0, int Lm) {
  int64_t t = 0;
  for (int L = 0; L <= Lm; ++L) t += (int64_t)(N0 << L) * (N0 << L);
  return t;
}

/* plain AIR, painting, super-resolution and flux on one grid and view */
static int run(const orc_grid* g, const orc_field* f, const orc_view* v, int N0, int Lm, double xc) {
  const int64_t T = total_of(N0, Lm);
  const int nb = f->kind == 0 ? 1 : f->n_bands;
  uint8_t* state = malloc(T);
  double *xiI = malloc(8 * T), *xiN = malloc(8 * T), *I = malloc(8 * T * nb), *N = malloc(8 * T);
  double *rmin = malloc(8 * T), *rmax = malloc(8 * T);
  int32_t *lmax = malloc(4 * T), *nvis = malloc(4 * T);
  int8_t* born = malloc(T);
  int64_t counts[ORC_MAXL];
  const int64_t nn = orc_air(g, f, v, N0, Lm, xc, 2.0, NULL, NULL, state, xiI, xiN, I, N, lmax, nvis, rmin, rmax,
                             counts, born);
  if (nn <= 0) return 1;
  const int64_t R = (int64_t)N0 << Lm;
  double* img = malloc(8 * R * R);
  orc_paint_leaves(N0, Lm, state, I, img);
  orc_superres(N0, Lm, state, I, img);
  const double flux = orc_leaf_flux(N0, Lm, v->width, state, I);
  /* a few individual pixels and the fixed image one level down */
  int32_t Ls[3] = {0, Lm, Lm > 0 ? Lm - 1 : 0}, is[3] = {0, (int32_t)R - 1, 1}, js[3] = {N0 - 1, 0, 1};
  double pI[3 * ORC_MAXB], pN[3];
  orc_trace_pixels(g, f, v, N0, 3, Ls, is, js, pI, pN, NULL, NULL, NULL, NULL);
  const int Lf = Lm > 0 ? Lm - 1 : 0;
  const int64_t Rf = (int64_t)N0 << Lf;
  double *fI = malloc(8 * Rf * Rf * nb), *fN = malloc(8 * Rf * Rf);
  orc_render_fixed(g, f, v, N0, Lf, fI, fN, NULL, NULL);
  printf("nodes %lld flux %.6e\n", (long long)nn, flux);
  free(state), free(xiI), free(xiN), free(I), free(N), free(rmin), free(rmax), free(lmax), free(nvis), free(born);
  free(img), free(fI), free(fN);
  return 0;
}

int main(void) {
  orc_set_threads(2);
  /* uniform 16^3 Gaussian blob, (rho, j, kappa) */
  enum { n = 16 };
  float *rho = malloc(4 * n * n * n), *emis = malloc(4 * n * n * n), *kap = malloc(4 * n * n * n);
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const double dx = (x + 0.5) / n - 0.5, dy = (y + 0.5) / n - 0.5, dz = (z + 0.5) / n - 0.5;
        const double r = exp(-(dx * dx + dy * dy + dz * dz) / 0.02) + 1e-3;
        const int k = (z * n + y) * n + x;
        rho[k] = (float)r, emis[k] = (float)(r * r), kap[k] = (float)(0.5 * r);
      }
  orc_grid gu = {0, {n, n, n}, {0, 0, 0}, {1, 1, 1}, 0, 0, 0, NULL, NULL, NULL};
  orc_field fu = {0, 1, rho, emis, kap, NULL, NULL};
  orc_view v1 = {{0.3, 0.5, 0.8}, {0, 1, 0}, {0.5, 0.5, 0.5}, 1.3};
  if (run(&gu, &fu, &v1, 8, 3, 0.3)) return 1;
  orc_view v2 = {{0, 0, 1}, {0, 1, 0}, {0.5, 0.5, 0.5}, 1.0};
  if (run(&gu, &fu, &v2, 4, 2, 0.0)) return 1;
  /* block AMR: 2^3 base blocks of 4^3 cells, block 0 refined into 8 */
  enum { bs = 4, nblk = 16, cells = nblk * bs * bs * bs };
  int32_t blevel[nblk], bcoord[nblk * 3], bchild[nblk];
  for (int b = 0; b < 8; ++b) {
    blevel[b] = 0, bchild[b] = b == 0 ? 8 : -1;
    bcoord[3 * b] = b & 1, bcoord[3 * b + 1] = (b >> 1) & 1, bcoord[3 * b + 2] = b >> 2;
  }
  for (int c = 0; c < 8; ++c) {
    const int b = 8 + c;
    blevel[b] = 1, bchild[b] = -1;
    bcoord[3 * b] = c & 1, bcoord[3 * b + 1] = (c >> 1) & 1, bcoord[3 * b + 2] = c >> 2;
  }
  float *arho = malloc(4 * cells), *atemp = malloc(4 * cells);
  for (int k = 0; k < cells; ++k) arho[k] = 0.5f + 0.01f * (float)(k % 37), atemp[k] = 1.0f + 0.1f * (float)(k % 11);
  const double band[6] = {1.0, 1.5, 0.5, 0.3, 1.0, 0.5};
  orc_grid ga = {1, {2, 2, 2}, {0, 0, 0}, {1, 1, 1}, bs, 1, nblk, blevel, bcoord, bchild};
  orc_field fa = {1, 2, arho, NULL, NULL, atemp, band};
  orc_view v3 = {{-0.4, 0.7, 0.55}, {0, 0, 1}, {0.5, 0.5, 0.5}, 1.4};
  if (run(&ga, &fa, &v3, 8, 2, 0.2)) return 1;
  free(rho), free(emis), free(kap), free(arho), free(atemp);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", ORACLE, str(src), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.count("nodes") == 3
