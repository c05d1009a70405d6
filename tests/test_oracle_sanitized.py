"""The oracle's C chain built with AddressSanitizer and UndefinedBehaviour-
Sanitizer (host code only) and run through a full small cycle -- init,
thresholds, sweeps and attempt ranges cut inside sweeps, reweight, flatness,
KL, widths, ln g -- on lattices with one to four words per row.  Any invalid
memory access or undefined operation aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <math.h>
void oracle_init(int L, int W, uint32_t seed, int8_t *spins, int32_t *energies);
void oracle_thresholds(int N, const double *omega, uint64_t *table);
void oracle_attempts_ids(int L, int n, const uint32_t *ids, uint32_t seed, int8_t *spins,
                         int32_t *energies, const uint64_t *table, uint64_t pos0, uint64_t count,
                         int record, uint64_t *hist, int nthreads);
void oracle_reweight(int N, double *omega, const uint64_t *hist);
double oracle_flatness(int N, const uint64_t *hist);
double oracle_chebyshev(int N, const uint64_t *hist);
double oracle_kl_divergence(int N, const uint64_t *hist, int w_prev);
int oracle_width(int N, const uint64_t *hist);
int oracle_reachable_width(int N, const uint64_t *hist);
int oracle_log_dos(int N, const uint64_t *hist, const double *omega, int norm, double *out);
int32_t oracle_energy(int L, const int8_t *spins);
int main(void) {
    int Ls[] = {4, 6, 34, 66, 128};
    for (int t = 0; t < 5; ++t) {
        int L = Ls[t], N = L * L, W = 3;
        int8_t *s = malloc((size_t)W * N);
        int32_t *e = malloc(W * sizeof(int32_t));
        double *om = calloc(N + 1, sizeof(double));
        uint64_t *tab = malloc((size_t)(N + 1) * 5 * sizeof(uint64_t));
        uint64_t *h = calloc(N + 1, sizeof(uint64_t));
        double *lg = malloc((N + 1) * sizeof(double));
        oracle_init(L, W, 7, s, e);
        for (int k = 0; k <= N; ++k) om[k] = sin(0.37 * k) * 2.0;
        uint64_t pos = 0;
        for (int it = 0; it < 3; ++it) {
            oracle_thresholds(N, om, tab);
            uint64_t counts[3] = {(uint64_t)N + 3, 5, (uint64_t)2 * N - 1};
            for (int c = 0; c < 3; ++c) {
                for (int k = 0; k <= N; ++k) h[k] = 0;
                oracle_attempts_ids(L, W, NULL, 7, s, e, tab, pos, counts[c], c != 1, h, 2);
                pos += counts[c];
            }
            oracle_reweight(N, om, h);
            volatile double f = oracle_flatness(N, h) + oracle_chebyshev(N, h) +
                                oracle_kl_divergence(N, h, oracle_reachable_width(N, h)) + oracle_width(N, h);
            (void)f;
            oracle_log_dos(N, h, om, 1, lg);
        }
        for (int w = 0; w < W; ++w)
            if (oracle_energy(L, s + (size_t)w * N) != e[w]) { printf("energy mismatch\n"); return 1; }
        free(s); free(e); free(om); free(tab); free(h); free(lg);
    }
    printf("ok\n");
    return 0;
}
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "oracle_asan"
    cmd = [gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(ROOT, "oracle", "muca_oracle.c"), str(drv),
           "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip().endswith("ok")
