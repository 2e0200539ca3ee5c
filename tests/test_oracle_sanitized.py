"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code): a small C driver, compiled together with oracle/pget_oracle.c with
gcc -fsanitize=address,undefined, runs forward, J v and J^T w (with and
without the depth factor and the depth-dependent response), the blur and
its transpose, and the regulariser on small geometries (odd and even sizes,
one bin, one angle, no blur) and checks the adjoint identity.  Any invalid
access or undefined operation aborts the driver."""
import os
import shutil
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pget_oracle.c")

DRIVER = textwrap.dedent(r"""
    #include <math.h>
    #include <stdio.h>
    #include <stdlib.h>

    typedef struct {
        int n, n_angles, n_bins, psf_radius;
        double angle0, arc, bin_size, step, psf_sigma, atten_scale;
        const double* depth;
        const double* resp;
        const double* far_taps;
    } og_geometry;
    int og_n_samples(const og_geometry*);
    int og_psf_half_width(const og_geometry*);
    void og_psf_taps(const og_geometry*, double*);
    void og_forward(const og_geometry*, const double*, const double*, double*);
    void og_forward_raw(const og_geometry*, const double*, const double*, double*);
    void og_psf(const og_geometry*, const double*, double*);
    void og_psf_transpose(const og_geometry*, const double*, double*);
    void og_jvp(const og_geometry*, const double*, const double*, const double*, const double*, double*);
    void og_vjp(const og_geometry*, const double*, const double*, const double*, double*, double*);
    double og_reg_energy(int, double, const double*);
    void og_reg_gradient(int, double, const double*, double*);

    static unsigned long long s = 12345;
    static double rnd(void) { s = s * 6364136223846793005ULL + 1442695040888963407ULL; return (double)(s >> 11) / 9007199254740992.0; }
    static double* arr(size_t n, double lo, double hi) {
        double* a = (double*)malloc(sizeof(double) * n);
        for (size_t i = 0; i < n; ++i) a[i] = lo + (hi - lo) * rnd();
        return a;
    }

    static int run(int n, int na, int nb, double sigma, double step, double bin, double arc, int with_depth, int with_resp) {
        og_geometry g = {n, na, nb, -1, 0.3, arc, bin, step, sigma, 0.8, NULL, NULL, NULL};
        int nt = og_n_samples(&g), K = og_psf_half_width(&g);
        double* depth = arr(nt, 1.0, 1.5);
        double* resp = arr(nt, 0.0, 1.0);
        double* far = (double*)malloc(sizeof(double) * (2 * K + 1));
        for (int k = -K; k <= K; ++k) far[k + K] = exp(-(double)(k * k) / 8.0);
        if (with_depth) g.depth = depth;
        if (with_resp) { g.resp = resp; g.far_taps = far; }
        size_t n2 = (size_t)n * n, ns = (size_t)na * nb;
        double *f = arr(n2, 0.1, 1.0), *mu = arr(n2, 0.0, 0.2), *vf = arr(n2, -1, 1), *vm = arr(n2, -1, 1);
        double *w = arr(ns, -1, 1), *y = arr(ns, 0, 0), *p = arr(ns, 0, 0), *jv = arr(ns, 0, 0), *v = arr(ns, 0, 0);
        double *gf = arr(n2, 0, 0), *gm = arr(n2, 0, 0), *rg = arr(n2, 0, 0);
        double* taps = (double*)malloc(sizeof(double) * (2 * K + 1));
        og_psf_taps(&g, taps);
        og_forward(&g, f, mu, y);
        og_forward_raw(&g, f, mu, p);
        og_psf(&g, p, v);
        og_psf_transpose(&g, w, v);
        og_jvp(&g, f, mu, vf, vm, jv);
        og_vjp(&g, f, mu, w, gf, gm);
        double e = og_reg_energy(n, 0.5, f);
        og_reg_gradient(n, 0.5, f, rg);
        double lhs = 0, rhs = 0;
        for (size_t i = 0; i < ns; ++i) lhs += jv[i] * w[i];
        for (size_t i = 0; i < n2; ++i) rhs += vf[i] * gf[i] + vm[i] * gm[i];
        int ok = fabs(lhs - rhs) <= 1e-10 * (fabs(lhs) + 1e-300) && isfinite(e);
        printf("n=%d na=%d nb=%d sigma=%g depth=%d resp=%d adjoint %.3e %s\n", n, na, nb, sigma, with_depth,
               with_resp, fabs(lhs - rhs) / (fabs(lhs) + 1e-300), ok ? "ok" : "FAIL");
        free(depth); free(resp); free(far); free(f); free(mu); free(vf); free(vm); free(w); free(y); free(p);
        free(jv); free(v); free(gf); free(gm); free(rg); free(taps);
        return ok;
    }

    int main(void) {
        int ok = 1;
        const double pi = 3.14159265358979323846;
        for (int d = 0; d < 2; ++d)
            for (int r = 0; r < 2; ++r) {
                ok &= run(9, 7, 13, 1.5, 1.0, 1.0, 2 * pi, d, r);
                ok &= run(8, 6, 12, 1.0, 1.5, 2.0, pi, d, r);
            }
        ok &= run(2, 1, 1, 0.0, 1.0, 1.0, 2 * pi, 1, 0);
        ok &= run(3, 5, 1, 1.0, 1.0, 1.0, 2 * pi, 0, 1);
        ok &= run(16, 1, 24, 2.0, 1.0, 1.0, 2 * pi, 1, 1);
        return ok ? 0 : 1;
    }
""")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    flags = ["-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer"]
    subprocess.run(["gcc"] + flags + ["-o", str(exe), str(drv), SRC, "-lm"], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout and r.stdout.count(" ok") == 11
