"""The oracle's C under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): a small driver runs every entry point the tests use (tables,
forces, pressure, a switching run with and without the Verlet candidate
list, the adjoint) on a 128-atom crystal, and the run must end cleanly with
no sanitizer report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(os.path.dirname(HERE), "oracle", "eam_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_pot orc_pot;
typedef struct {
    int mode, fix_com;
    double T, gamma, dt, mass, k, k2;
    uint64_t seed;
    double skin;
    int nlist_cap;
} orc_params;

orc_pot* orc_pot_create(int, double, const double*, const double*, int, double, const double*);
void orc_pot_free(orc_pot*);
int orc_eam(const orc_pot*, int, const double*, const double*, double*, double*, double*, double*, double*);
int orc_pressure(const orc_pot*, int, const double*, const double*, double, const double*, double*);
int orc_schedule(int, int, double, int, int, int, int, double*);
void orc_init_velocities(const orc_params*, int, double*);
int orc_run(const orc_pot*, const orc_params*, int, const double*, const double*, double*, double*, int,
            const double*, int64_t, double, double*, double*, double*, const double*);
int orc_adjoint_theta(const orc_pot*, int, const double*, const double*, double*);

int main(void)
{
    enum { NK = 500, NC = 4, N = 2 * NC * NC * NC, S = 40 };
    const double rc = 5.3, rho_max = 200.0, a = 2.855;
    double phi[NK], rho[NK], F[NK];
    for (int k = 0; k < NK; ++k) {
        const double r = rc * k / (NK - 1), q = rho_max * k / (NK - 1);
        const double s = r < 4.8 ? 1.0 : 0.5 * (1.0 + cos(M_PI * (r - 4.8) / 0.5));
        phi[k] = (0.5 * exp(-7.0 * (r / 2.48 - 1.0)) - 0.9 * exp(-3.5 * (r / 2.48 - 1.0))) * s;
        rho[k] = exp(-6.0 * (r / 2.48 - 1.0)) * s;
        F[k] = -2.0 * sqrt(q);
    }
    orc_pot* p = orc_pot_create(NK, rc, phi, rho, NK, rho_max, F);
    if (!p) return 10;
    static double x0[3 * N], x[3 * N], v[3 * N], f[3 * N], e[N], rh[N], fp[N];
    const double L[3] = {NC * a, NC * a, NC * a};
    int i = 0;
    for (int ix = 0; ix < NC; ++ix)
        for (int iy = 0; iy < NC; ++iy)
            for (int iz = 0; iz < NC; ++iz)
                for (int b = 0; b < 2; ++b, ++i) {
                    x0[3 * i] = (ix + 0.5 * b) * a;
                    x0[3 * i + 1] = (iy + 0.5 * b) * a;
                    x0[3 * i + 2] = (iz + 0.5 * b) * a;
                }
    for (int q = 0; q < 3 * N; ++q) x[q] = x0[q] + 0.05 * sin(1.7 * q);
    double U = 0.0, P[3];
    if (orc_eam(p, N, x, L, f, &U, e, rh, fp) & ~4) return 11;
    if (orc_pressure(p, N, x, NULL, 55.845, L, P) & ~4) return 12;
    static double lam[S + 1], dH[S], W[S], en[S], g[3 * NK];
    if (orc_schedule(0, 2, 1.0, 10, 10, 5, 5, lam)) return 13;
    for (int skin10 = 0; skin10 <= 3; skin10 += 3) {
        orc_params P0 = {0, 1, 300.0, 10.0, 0.001, 55.845, 5.0, 0.0, 7, skin10 / 10.0, 256};
        orc_init_velocities(&P0, N, v);
        for (int q = 0; q < 3 * N; ++q) x[q] = x0[q];
        if (orc_run(p, &P0, N, x0, L, x, v, S, lam, 0, 0.0, dH, W, en, NULL) & ~4) return 14;
    }
    if (orc_pressure(p, N, x, v, 55.845, L, P) & ~4) return 15;
    if (orc_adjoint_theta(p, N, x, L, g) & ~4) return 16;
    orc_pot_free(p);
    printf("ok %.6f %.6f\n", U / N, W[S - 1]);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", ORACLE_C, str(src), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-2000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.startswith("ok ")
