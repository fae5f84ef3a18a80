"""The oracle (oracle/adref.c) under AddressSanitizer and
UndefinedBehaviorSanitizer: a C driver compiled together with it calls every
entry point on small systems (forces, energy, the matrix-free, row and dense
mobility with both tensors, multi-system RK4 and noisy Heun runs with
records, the stroke-averaged right-hand side and run) and exits 0 only if
each call succeeds with finite results and the three mobility forms agree.
Any out-of-bounds access, use after free, leak, signed overflow or other
undefined behaviour aborts the driver. The host logic of the runtime is run
under the same sanitizers in test_host_order.py."""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]

DRIVER = r"""
#include <stdio.h>
#include "adref.c"

static int finite_all(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}
#define CHECK(what, cond)                                    \
    do {                                                     \
        if (!(cond)) {                                       \
            fprintf(stderr, "failed: %s\n", what);           \
            return 1;                                        \
        }                                                    \
    } while (0)

int main(void) {
    enum { S = 12, N = 2 * S };
    double X[3 * N], phi[S], F[3 * N], u[3 * N], ud[3 * N], ur[3 * 4];
    for (int s = 0; s < S; ++s) {
        const double cx = 12.0 * (s % 3), cy = 12.0 * ((s / 3) % 2), cz = 12.0 * (s / 6);
        X[6 * s + 0] = cx; X[6 * s + 1] = cy; X[6 * s + 2] = cz;
        X[6 * s + 3] = cx + 4.0; X[6 * s + 4] = cy + 0.3 * s; X[6 * s + 5] = cz;
        phi[s] = 0.37 * s;
    }
    /* two spheres of neighbouring dumbbells inside the steric range */
    X[3 * 2 + 0] = X[3 * 1 + 0] + 1.5;
    X[3 * 2 + 1] = X[3 * 1 + 1];
    X[3 * 2 + 2] = X[3 * 1 + 2];
    adref_params p = {1.0, 1.0, 1.0, 4.0, 1.0, 100.0, 0.05, 10.0, 2.0, 0, 0, 0.0, 7};
    for (int tensor = 0; tensor < 2; ++tensor) {
        p.tensor = tensor;
        CHECK("forces", adref_forces(&p, N, X, phi, 0.3, F) == ADREF_OK && finite_all(F, 3 * N));
        CHECK("energy", isfinite(adref_energy(&p, N, X, phi, 0.3)));
        CHECK("mobility", adref_mobility(&p, N, X, F, u) == ADREF_OK && finite_all(u, 3 * N));
        CHECK("mobility_dense", adref_mobility_dense(&p, N, X, F, ud) == ADREF_OK);
        double mx = 0.0, dmax = 0.0;
        for (int i = 0; i < 3 * N; ++i) {
            mx = fmax(mx, fabs(u[i]));
            dmax = fmax(dmax, fabs(u[i] - ud[i]));
        }
        CHECK("dense equals matrix-free", dmax <= 1e-12 * mx);
        const int64_t rows[4] = {0, 5, 11, 23};
        CHECK("mobility_rows", adref_mobility_rows(&p, N, X, F, 4, rows, ur) == ADREF_OK);
        for (int r = 0; r < 4; ++r)
            for (int a = 0; a < 3; ++a) CHECK("rows equal full", ur[3 * r + a] == u[3 * rows[r] + a]);
    }
    /* two systems of 5 and 7 dumbbells, records every 5 steps */
    const int64_t off[3] = {0, 10, 24};
    double centres[4 * S * 3], com[4 * 2 * 3], Xr[3 * N];
    for (int integ = 0; integ < 2; ++integ) {
        memcpy(Xr, X, sizeof X);
        p.integrator = integ;
        p.kT = integ ? 0.01 : 0.0;
        CHECK("run", adref_run(&p, 2, off, Xr, phi, 0.0, 3, 20, 5, centres, com) == ADREF_OK);
        CHECK("run finite", finite_all(Xr, 3 * N) && finite_all(centres, 4 * S * 3) && finite_all(com, 4 * 2 * 3));
    }
    /* stroke-averaged equations of 3 swimmers */
    double R[9] = {0, 0, 0, 20, 0, 0, 0, 25, 5}, Nv[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, dR[9], dN[9];
    p.integrator = 0;
    p.kT = 0.0;
    CHECK("sa_rhs", adref_sa_rhs(&p, 3, R, Nv, phi, dR, dN) == ADREF_OK && finite_all(dR, 9) && finite_all(dN, 9));
    CHECK("sa_run", adref_sa_run(&p, 3, R, Nv, phi, 0.5, 40) == ADREF_OK && finite_all(R, 9) && finite_all(Nv, 9));
    /* refused arguments leave no trace */
    CHECK("odd N refused", adref_forces(&p, N - 1, X, phi, 0.3, F) == ADREF_EINVAL);
    const int64_t bad_rows[1] = {N};
    CHECK("row out of range refused", adref_mobility_rows(&p, N, X, F, 1, bad_rows, ur) == ADREF_EINVAL);
    puts("ok");
    return 0;
}
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    (tmp_path / "driver.c").write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.run([gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-builtin-sin", "-fno-builtin-cos", "-fno-builtin-sincos",
                    "-I", str(ROOT / "oracle"), str(tmp_path / "driver.c"), "-lm", "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120,
                         env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stderr[-3000:]
