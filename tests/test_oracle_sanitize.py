"""The C oracle built with AddressSanitizer + UndefinedBehaviorSanitizer (and,
separately, ThreadSanitizer over its OpenMP loops) on the CPU: a driver runs
its trace, forward and back projections and DROP on a small scan (hand-made
rays, among them a non-finite record and a NaN b) and the run must end clean
with no sanitizer report.  Host code only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle", "orc.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "orc.c"   /* the oracle itself, in this translation unit */
int main(void)
{
    orc_grid g;
    memset(&g, 0, sizeof g);
    g.nx = 8; g.ny = 8; g.nz = 2;
    for (int a = 0; a < 3; ++a) g.pitch[a] = 1.0;
    g.origin[0] = -4.0; g.origin[1] = -4.0; g.origin[2] = -1.0;
    orc_mlp m;
    memset(&m, 0, sizeof m);
    m.u_in = -5.0; m.u_out = 5.0; m.step = 1.0;
    const double poly[6] = {7.457e-6, 4.548e-7, -5.777e-8, 1.301e-8, -9.228e-10, 2.687e-11};
    memcpy(m.poly, poly, sizeof poly);
    m.E0 = 13.6; m.X0 = 36.08; m.log_term = 1;
    enum { N = 300 };
    static float f[9][N];
    float b[N];
    for (int i = 0; i < N; ++i) {
        double t = -3.5 + 7.0 * (i % 37) / 37.0, v = -0.8 + 1.6 * (i % 11) / 11.0;
        f[0][i] = (float)t; f[1][i] = (float)v; f[2][i] = 0.01f * (float)((i % 5) - 2);
        f[3][i] = 0.005f * (float)((i % 3) - 1);
        f[4][i] = (float)(t + 0.3 * sin(i)); f[5][i] = (float)(v + 0.1 * cos(i));
        f[6][i] = f[2][i]; f[7][i] = f[3][i];
        f[8][i] = (float)(2.0 * M_PI * (i % 90) / 90.0);
        b[i] = (float)(5.0 + (i % 7));
    }
    f[0][13] = NAN;
    f[8][77] = INFINITY;
    b[101] = NAN;
    orc_protons p;
    memset(&p, 0, sizeof p);
    p.t_in = f[0]; p.v_in = f[1]; p.th_in = f[2]; p.ph_in = f[3];
    p.t_out = f[4]; p.v_out = f[5]; p.th_out = f[6]; p.ph_out = f[7]; p.gantry = f[8];
    p.n = N;
    const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    enum { CAP = 64 };
    int32_t *vox = malloc(sizeof(int32_t) * N * CAP);
    double *ch = malloc(sizeof(double) * N * CAP);
    int64_t *nnz = malloc(sizeof(int64_t) * N);
    orc_trace_batch(&g, &m, &p, 0, N, CAP, vox, ch, nnz);
    double *x = malloc(sizeof(double) * nvox), *y = malloc(sizeof(double) * N), *n2 = malloc(sizeof(double) * N);
    int64_t *nd = malloc(sizeof(int64_t) * N);
    for (int64_t j = 0; j < nvox; ++j) x[j] = 1.0;
    orc_forward(&g, &m, &p, 0, x, y, n2, nd);
    double *r = malloc(sizeof(double) * N), *gr = calloc(nvox, sizeof(double));
    for (int i = 0; i < N; ++i) r[i] = 0.01 * i;
    r[5] = NAN;
    orc_backproject(&g, &m, &p, 0, r, gr);
    orc_drop(&g, &m, &p, b, x, 40, 0.3, 2, 0, -1, 0);
    double s = 0.0;
    for (int64_t j = 0; j < nvox; ++j) s += x[j] + gr[j];
    for (int i = 0; i < N; ++i) s += y[i] + n2[i] + (double)nnz[i];
    if (!isfinite(s)) { fprintf(stderr, "non-finite result\n"); return 2; }
    printf("ok %.6f\n", s);
    free(vox); free(ch); free(nnz); free(x); free(y); free(n2); free(nd); free(r); free(gr);
    return 0;
}
"""


def _build_and_run(tmp, flags, env_extra):
    drv = os.path.join(tmp, "driver.c")
    open(drv, "w").write(DRIVER)
    exe = os.path.join(tmp, "driver")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off", *flags,
           "-I" + os.path.join(ROOT, "oracle"), drv, "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, OMP_NUM_THREADS="4", **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        r = _build_and_run(tmp, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                           {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
        assert r.stdout.startswith("ok ")


LLVM = "/opt/rocm/llvm"
ARCHER = os.path.join(LLVM, "lib", "libarcher.so")


def _tsan_run(tmp, source):
    drv = os.path.join(tmp, "driver.c")
    open(drv, "w").write(source)
    exe = os.path.join(tmp, "driver")
    cmd = [os.path.join(LLVM, "bin", "clang"), "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-ffp-contract=off", "-fsanitize=thread", "-I" + os.path.join(ROOT, "oracle"), drv, "-o", exe,
           "-L" + os.path.join(LLVM, "lib"), "-Wl,-rpath," + os.path.join(LLVM, "lib"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    # the OpenMP runtime's own bookkeeping (work sharing, thread start) is not
    # instrumented: accesses from modules built without the sanitizer are
    # ignored (Archer's own advice), the program's are all checked
    env = dict(os.environ, OMP_NUM_THREADS="4", OMP_TOOL_LIBRARIES=ARCHER,
               TSAN_OPTIONS="ignore_noninstrumented_modules=1 halt_on_error=0 report_signal_unsafe=0",
               LD_LIBRARY_PATH=os.path.join(LLVM, "lib") + ":" + os.environ.get("LD_LIBRARY_PATH", ""))
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)


@pytest.mark.skipif(not os.path.exists(ARCHER), reason="clang with the OpenMP ThreadSanitizer tool not available")
def test_oracle_openmp_loops_under_thread_sanitizer():
    # ThreadSanitizer over the oracle's OpenMP loops, built with clang and its
    # OpenMP runtime and run with the Archer tool, which tells the sanitizer
    # about OpenMP's barriers and task synchronisation (an OpenMP runtime the
    # tool cannot see makes every parallel region look racy)
    with tempfile.TemporaryDirectory() as tmp:
        r = _tsan_run(tmp, DRIVER)
        assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert r.stdout.startswith("ok ")


@pytest.mark.skipif(not os.path.exists(ARCHER), reason="clang with the OpenMP ThreadSanitizer tool not available")
def test_thread_sanitizer_setup_reports_a_planted_race():
    # the same build and suppressions still report a race between OpenMP
    # threads on program data (a shared sum without a reduction)
    racy = r"""
#include <stdio.h>
int main(void)
{
    double s = 0.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < 4000; ++i) s += 1e-3 * i;
    printf("ok %f\n", s);
    return 0;
}
"""
    with tempfile.TemporaryDirectory() as tmp:
        r = _tsan_run(tmp, racy)
        assert "WARNING: ThreadSanitizer: data race" in r.stderr, r.stderr[-2000:]
