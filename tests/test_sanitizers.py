"""Host sanitizers (no GPU): the oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc) and driven through every entry point -- the
four geometries and both lattices, friction, thermal noise of both forms,
electron sheets and phonons, open ends, masked walls, the plain and the screened
quadrature, population get/set --
must run without a single report.  The library's host-side planning
(geometry classification, wall tables, arena layout) is exercised the same
way through lbm_footprint, with the sanitizers on the host pass of the
library's build."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int lattice, precision, geometry, nx, ny, nz;
  double tube_radius, tube_cy, tube_cz, tau, rho0, force[3], wall_velocity_top;
  const unsigned char *solid;
} P;
typedef struct {
  double T, omega0, gamma_s, omega_l, gamma_l, a_l, d;
  int nq, nw;
  double q_max, w_max, lambda_target;
  int dispersion, coupling;
  double v_l;
} S;
typedef struct ora_ctx ora_ctx;
int ora_create(const P *, ora_ctx **);
void ora_destroy(ora_ctx *);
long ora_wall_count(const ora_ctx *);
long ora_fluid_count(const ora_ctx *);
void ora_wall_coords(const ora_ctx *, int32_t *);
void ora_wall_links(const ora_ctx *, double *);
int ora_set_friction(ora_ctx *, const double *);
int ora_set_thermal(ora_ctx *, double, int, uint64_t);
int ora_set_electrons(ora_ctx *, double, double, double, double);
int ora_set_open_ends(ora_ctx *, int, double, double);
int ora_set_noise_closure(ora_ctx *, const double *, int, int, const double *, const double *);
int ora_set_phonons(ora_ctx *, double, double, double, double);
void ora_get_phonons(const ora_ctx *, double *, double *);
void ora_get_electrons(const ora_ctx *, double *, double *);
void ora_step(ora_ctx *, long);
void ora_fields(const ora_ctx *, double *, double *, double *, double *);
void ora_invariants(const ora_ctx *, double *);
void ora_get_populations(const ora_ctx *, double *);
void ora_set_populations(ora_ctx *, const double *, long);
void ora_friction(const S *, const double *, long, double *, double *);

static int run(int q, int geom, int nx, int ny, int nz, double R, int mode, int elec) {
  P p = {q, 0, geom, nx, ny, nz, R, (ny - 1) / 2.0, (nz - 1) / 2.0, 0.8, 1.0, {1e-6, 0, 0}, 0, 0};
  unsigned char *mask = calloc((size_t)nx * ny, 1);
  if (geom == 3) { /* corrugated floor, a step in the ceiling, a post */
    for (int x = 0; x < nx; x++) {
      for (int y = 0; y < 1 + (x % 3); y++) mask[x + nx * y] = 1;
      if (x >= nx / 2) mask[x + nx * (ny - 1)] = 1;
    }
    mask[nx / 3 + nx * (ny / 2)] = 1;
    p.solid = mask;
  }
  ora_ctx *o;
  if (ora_create(&p, &o)) return 1;
  long nw = ora_wall_count(o), nc = (long)nx * ny * nz;
  double *lam = malloc(sizeof(double) * (nw + 1));
  int32_t *xyz = malloc(sizeof(int32_t) * 3 * (nw + 1));
  double *links = malloc(sizeof(double) * 19 * (nw + 1));
  double *f = malloc(sizeof(double) * 4 * nc), *g = malloc(sizeof(double) * q * nc);
  double *ue = malloc(sizeof(double) * 2 * nz * nx), *pe = malloc(sizeof(double) * 6 * nz * nx);
  double inv[3];
  for (long k = 0; k < nw; k++) lam[k] = 0.01 * (k % 7);
  ora_wall_coords(o, xyz);
  ora_wall_links(o, links);
  if (ora_set_friction(o, lam)) return 2;
  if (mode && ora_set_thermal(o, 1e-6, mode, 9)) return 3;
  if (mode == 1) {
    double gam[6 * 2 * 3], wx[2] = {0.3, 0.7}, wt[3] = {0.2, 0.5, 0.3};
    for (int k = 0; k < 36; k++) gam[k] = 0.5 + 0.1 * (k % 5);
    if (ora_set_noise_closure(o, gam, 2, 3, wx, wt)) return 7;
  }
  if (elec && ora_set_electrons(o, 0.9, 1.0, 0.05, 1e-6)) return 4;
  if (elec && ora_set_phonons(o, 0.8, 1.2, 0.02, 0.1)) return 8;
  if (!elec && geom <= 1 && ora_set_open_ends(o, 1, 1.0001, 0.9999)) return 6;
  ora_step(o, 7);
  ora_fields(o, f, f + nc, f + 2 * nc, f + 3 * nc);
  ora_invariants(o, inv);
  ora_get_populations(o, g);
  ora_set_populations(o, g, 7);
  ora_step(o, 3);
  if (elec) ora_get_electrons(o, ue, pe);
  if (elec) ora_get_phonons(o, ue, pe);
  if (!isfinite(inv[0]) || !isfinite(inv[1])) return 5;
  free(lam); free(xyz); free(links); free(f); free(g); free(ue); free(pe); free(mask);
  ora_destroy(o);
  return 0;
}

int main(void) {
  int rc = 0;
  rc |= run(9, 0, 12, 6, 1, 0, 0, 0);
  rc |= run(9, 0, 12, 6, 1, 0, 2, 1);
  rc |= run(19, 0, 7, 5, 4, 0, 1, 1);
  rc |= run(19, 1, 9, 5, 6, 0, 2, 0);
  rc |= run(19, 0, 6, 5, 3, 0, 0, 0);
  rc |= run(19, 2, 5, 14, 14, 5.0, 1, 0);
  rc |= run(9, 3, 13, 9, 1, 0, 1, 0);
  rc |= run(19, 3, 8, 10, 3, 0, 2, 0);
  for (int c = 0; c < 2; c++) {
    S s = {1.0, 2.0, 0.5, 3.0, 1.0, 0.5, 1.0, 9, 17, 10.0, 20.0, 0.05, 1, c, 0.4 * c};
    double om[3] = {1.5, 2.0, 2.5}, raw[3], lat[3];
    ora_friction(&s, om, 3, raw, lat);
    for (int k = 0; k < 3; k++)
      if (!(raw[k] > 0) || !(lat[k] > 0)) rc |= 8;
  }
  printf("driver rc %d\n", rc);
  return rc;
}
"""

HOST_DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include "lbm.h"
int main(void) {
  int bad = 0;
  for (int geom = 0; geom < 4; geom++)
    for (int q = 9; q <= 19; q += 10)
      for (int prec = 0; prec < 3; prec++)
        for (int nx = 1; nx <= 300; nx += 37)
          for (int ny = 1; ny <= 40; ny += 13) {
            if (q == 9 && geom != LBM_SLAB && geom != LBM_MASKED) continue;
            lbm_params p = {0};
            uint8_t *mask = (uint8_t *)calloc((size_t)nx * (ny + 9), 1);
            for (int x = 0; x < nx; x++) /* steps on the floor, a post */
              for (int y = 0; y < (x / 5) % 3 && y < ny; y++) mask[x + nx * y] = 1;
            if (ny > 4) mask[nx / 2 + nx * (ny / 2)] = 1;
            p.solid = mask;
            p.lattice = q; p.precision = prec; p.geometry = geom;
            p.nx = nx; p.ny = geom == LBM_TUBE ? 2 * (ny / 2) + 9 : ny;
            p.nz = q == 9 ? 1 : (geom == LBM_TUBE ? p.ny : ny / 2 + 1);
            p.tube_radius = (p.ny - 8) / 2.0; p.tube_cy = (p.ny - 1) / 2.0;
            p.tube_cz = (p.nz - 1) / 2.0; p.tau = 0.7; p.rho0 = 1.0;
            size_t b = 0;
            lbm_status s = lbm_footprint(&p, &b);
            if (s == LBM_OK && b == 0) bad++;
            free(mask);
          }
  lbm_params p = {0};
  p.lattice = 19; p.tau = 0.4;  /* rejected parameters */
  size_t b;
  if (lbm_footprint(&p, &b) == LBM_OK) bad++;
  printf("host driver bad %d\n", bad);
  return bad;
}
"""


def _gcc_has_sanitizers(tmp):
    src = os.path.join(tmp, "probe.c")
    with open(src, "w") as f:
        f.write("int main(void){return 0;}\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", src, "-o", os.path.join(tmp, "p")],
                       capture_output=True)
    return r.returncode == 0


def test_oracle_under_asan_and_ubsan(tmp_path):
    tmp = str(tmp_path)
    if not _gcc_has_sanitizers(tmp):
        pytest.skip("gcc without sanitizer runtimes")
    drv = os.path.join(tmp, "driver.c")
    with open(drv, "w") as f:
        f.write(DRIVER)
    exe = os.path.join(tmp, "oracle_asan")
    subprocess.run(["gcc", "-std=gnu99", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, drv, os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm"],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "driver rc 0" in r.stdout


def test_library_host_planning_under_asan_and_ubsan(tmp_path):
    # the sanitizers on the host pass only (device code unoptimised, to build
    # fast; no GPU call): make_plan for every geometry, lattice and storage
    # precision over a range of shapes
    tmp = str(tmp_path)
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not _gcc_has_sanitizers(tmp):
        pytest.skip("hipcc or sanitizer runtimes missing")
    drv = os.path.join(tmp, "host_driver.cpp")
    with open(drv, "w") as f:
        f.write(HOST_DRIVER)
    exe = os.path.join(tmp, "lbm_host_asan")
    csrc = os.path.join(ROOT, "paper_2403_15768_amd", "csrc")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-g0", "-std=c++17",
           "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-g", "-I", os.path.join(ROOT, "include"), "-I", csrc, "-o", exe, drv,
           os.path.join(csrc, "lbm_api.hip"), os.path.join(csrc, "lbm_batch.hip"),
           os.path.join(csrc, "lbm_kernels.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "host driver bad 0" in r.stdout
