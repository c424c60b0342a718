// Native driver of lib_llgdisk's C ABI, built together with the library's
// sources under the host address and undefined-behaviour sanitizers
// (tests/native/build_sanitized.py).  It calls every entry point of
// include/llgdisk.h with valid arguments and the error paths with invalid
// ones, frees everything it creates, and checks results that need no
// reference beyond the library itself: graph replays and the entry point
// without allocation equal eager calls bit for bit, the on-chip plan equals
// the global one, |m| stays 1 under renormalisation, energies and spectra are
// finite, errors come back as the documented codes.  Exit status 0 when every
// check passes.
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/lsan_interface.h>
#define LLG_LEAK_CHECK() __lsan_do_leak_check()
#endif
#endif
#ifndef LLG_LEAK_CHECK
#define LLG_LEAK_CHECK() ((void)0)
#endif

#include "../../include/llgdisk.h"

namespace {

int g_checks = 0, g_failed = 0;

void check(bool ok, const char* what) {
    ++g_checks;
    if (!ok) {
        ++g_failed;
        std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, llg_last_error());
    }
}

#define HIP_OK(x)                                                                     \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            std::fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            return 2;                                                                 \
        }                                                                             \
    } while (0)

// In-plane vortex with a Gaussian out-of-plane core at (x0, y0) (cells), packed [3][D][D].
void vortex(int D, double x0, double y0, float* out) {
    const double c = 0.5 * (D - 1), w = 2.5;
    for (int j = 0; j < D; ++j)
        for (int i = 0; i < D; ++i) {
            const double x = i - c - x0, y = j - c - y0, r2 = x * x + y * y;
            const double mz = std::exp(-r2 / (w * w)), s = std::sqrt(1.0 - mz * mz), r = std::sqrt(r2) + 1e-12;
            out[0 * D * D + j * D + i] = (float)(-y / r * s);
            out[1 * D * D + j * D + i] = (float)(x / r * s);
            out[2 * D * D + j * D + i] = (float)mz;
        }
}

struct Dev {
    void* p = nullptr;
    explicit Dev(size_t bytes) { (void)hipMalloc(&p, bytes); }
    ~Dev() { (void)hipFree(p); }
    float* f() const { return static_cast<float*>(p); }
    double* d() const { return static_cast<double*>(p); }
};

std::vector<float> to_host(const float* d, size_t n) {
    std::vector<float> h(n);
    (void)hipMemcpy(h.data(), d, n * sizeof(float), hipMemcpyDeviceToHost);
    return h;
}

}  // namespace

int main() {
    hipStream_t st = nullptr;
    HIP_OK(hipStreamCreate(&st));
    llg_params p{};
    double lam = 0.0;
    check(llg_params_from_si(13e-12, 8.6e5, 1.76e11, 2.0, 10.0, 0.03, 0.0, 0.02, &p, &lam) == 0, "params_from_si");
    check(lam > 5.0 && lam < 5.6, "lambda_ex of permalloy");
    p.dtau = 0.04;

    // ---- a ragged batch: P = 64, 128, 256
    const double R[3] = {30.0, 44.0, 100.0}, L[3] = {10.0, 6.0, 20.0};
    llg_disk h = nullptr;
    check(llg_batch_create(3, R, L, 2.0, nullptr, &h) == 0 && h, "batch_create");
    if (!h) return 1;
    check(llg_disk_count(h) == 3, "disk_count");
    const long long n = llg_state_size(h);
    std::vector<float> m0(n);
    for (int k = 0; k < 3; ++k) {
        int D = 0, P = 0, nc = 0;
        check(llg_disk_info(h, k, &D, &P, &nc) == 0 && D == (int)(R[k]) && nc > 0, "disk_info");
        check(llg_disk_workgroups(h, k) >= 1, "disk_workgroups");
        // core between cell centres: a cell exactly at the core would have no in-plane angle
        vortex(D, 1.3, -0.6, m0.data() + llg_disk_offset(h, k));
    }
    std::vector<llg_params> ps(3, p);
    Dev m(n * 4), m2(n * 4), H(n * 4), out(64 * 8), work(n * 4);
    HIP_OK(hipMemcpy(m.p, m0.data(), n * 4, hipMemcpyHostToDevice));

    check(llg_demag_field(h, m.f(), H.f(), st) == 0, "demag_field");
    check(llg_rhs(h, m.f(), H.f(), ps.data(), st) == 0, "rhs");
    check(llg_energy(h, m.f(), ps.data(), out.d(), st) == 0, "energy");
    {
        std::vector<double> e(12);
        HIP_OK(hipMemcpy(e.data(), out.p, 12 * 8, hipMemcpyDeviceToHost));
        bool fin = true;
        for (double v : e) fin = fin && std::isfinite(v);
        check(fin && e[0] < 0.0, "energy finite, vortex below zero");
    }
    check(llg_mean_m(h, m.f(), out.d(), st) == 0, "mean_m");
    check(llg_vortex_core_position(h, m.f(), lam, nullptr, out.d(), st) == 0, "core position");
    {
        std::vector<double> c(15);
        HIP_OK(hipMemcpy(c.data(), out.p, 15 * 8, hipMemcpyDeviceToHost));
        check(c[4] >= 1 && c[9] >= 1 && c[14] >= 1, "a +1 vortex in every disk");
    }

    // ---- integrators, graph and the entry point without allocation
    HIP_OK(hipMemcpy(m2.p, m.p, n * 4, hipMemcpyDeviceToDevice));
    check(llg_rk4_step(h, m.f(), 12, ps.data(), st) == 0, "rk4_step");
    llg_graph g = nullptr;
    check(llg_graph_create(h, 0, m2.f(), 12, ps.data(), 0, 0, &g) == 0 && g, "graph_create");
    check(llg_graph_launch(g, st) == 0, "graph_launch");
    HIP_OK(hipStreamSynchronize(st));
    check(to_host(m.f(), n) == to_host(m2.f(), n), "graph replay equals eager steps");
    llg_graph_destroy(g);
    HIP_OK(hipMemcpy(m2.p, m.p, n * 4, hipMemcpyDeviceToDevice));
    check(llg_rk4_step(h, m.f(), 7, ps.data(), st) == 0, "rk4_step again");
    check(llg_noalloc_bytes(h) > 0, "noalloc_bytes");
    check(llg_rk4_step_noalloc(h, m2.f(), 7, ps.data(), st) == 0, "rk4_step_noalloc");
    HIP_OK(hipStreamSynchronize(st));
    check(to_host(m.f(), n) == to_host(m2.f(), n), "no-allocation steps equal rk4_step");
    check(llg_check(h, st) == 0, "check after integrators");

    // on-chip plan equals the global one
    HIP_OK(hipMemcpy(m2.p, m.p, n * 4, hipMemcpyDeviceToDevice));
    check(llg_rk4_step(h, m.f(), 5, ps.data(), st) == 0, "rk4_step global");
    check(llg_set_on_chip(h, 128) == 0 && llg_get_on_chip(h) == 128, "set_on_chip");
    check(llg_rk4_step(h, m2.f(), 5, ps.data(), st) == 0, "rk4_step on chip");
    HIP_OK(hipStreamSynchronize(st));
    check(to_host(m.f(), n) == to_host(m2.f(), n), "on-chip steps equal global ones");
    check(llg_set_on_chip(h, 0) == 0, "set_on_chip off");

    // Heun with renormalisation: |m| = 1 inside the disks
    llg_params ph = p;
    ph.temp = 0.02;
    ph.renorm = 1;
    std::vector<llg_params> phs(3, ph);
    check(llg_heun_step(h, m.f(), 6, 11, 0, 0, phs.data(), st) == 0, "heun_step");
    check(llg_step_counter_set(h, 100, st) == 0, "step_counter_set");
    check(llg_heun_step(h, m.f(), 4, 11, LLG_STEP_COUNTER, 0, phs.data(), st) == 0, "heun_step on counter");
    unsigned long long step = 0;
    check(llg_step_counter_get(h, &step, st) == 0 && step == 104, "step counter advanced");
    {
        std::vector<float> hm = to_host(m.f(), n);
        double worst = 0.0;
        for (int k = 0; k < 3; ++k) {
            int D = 0, P = 0, nc = 0;
            llg_disk_info(h, k, &D, &P, &nc);
            const float* q = hm.data() + llg_disk_offset(h, k);
            for (int c = 0; c < D * D; ++c) {
                const double s = (double)q[c] * q[c] + (double)q[D * D + c] * q[D * D + c] +
                                 (double)q[2 * D * D + c] * q[2 * D * D + c];
                if (s > 0.0) worst = std::fmax(worst, std::fabs(std::sqrt(s) - 1.0));
            }
        }
        check(worst < 1e-6, "|m| = 1 after renormalised Heun steps");
    }
    check(llg_noise(h, 11, 3, 0, H.f(), st) == 0, "noise");

    // series and spectra
    const long long ns = 64, every = 2;
    Dev series(ns / every * 3 * 4 * 8);
    check(llg_rk4_series(h, m.f(), ns, ps.data(), every, series.d(), st) == 0, "rk4_series");
    check(llg_heun_series(h, m.f(), ns, 11, 500, 0, phs.data(), every, series.d(), st) == 0, "heun_series");
    Dev spec(3 * (32 / 2 + 1) * 8), pwork(4 * 32 * 3 * 8);
    check(llg_power_spectrum(series.d(), 3, 4, 32, 3 * 4, 1, 1, pwork.d(), spec.d(), st) == 0, "power_spectrum");
    {
        std::vector<double> s(3 * 17);
        HIP_OK(hipMemcpy(s.data(), spec.p, s.size() * 8, hipMemcpyDeviceToHost));
        bool ok = true;
        for (double v : s) ok = ok && std::isfinite(v) && v >= 0.0;
        check(ok, "power spectra finite and non-negative");
    }

    // relaxation, adjoints, core-position cotangent
    const double X[6] = {2.0, 0.0, 4.0, 0.0, 6.0, 0.0};
    std::vector<llg_params> pr(3, p);
    for (auto& q : pr) q.alpha = 0.0;
    check(llg_relax(h, m.f(), X, 4.0 * lam, 2.0, 1e-4, 200, pr.data(), out.d(), st) == 0, "relax");
    const long long nst = 2;
    Dev rec(8 * nst * n * 4), ybar(n * 4), pgrad(6 * 8), core(15 * 8), rbar(6 * 8);
    HIP_OK(hipMemset(pgrad.p, 0, 6 * 8));
    HIP_OK(hipMemcpy(ybar.p, m.p, n * 4, hipMemcpyDeviceToDevice));
    check(llg_rk4_record(h, m.f(), nst, ps.data(), rec.f(), st) == 0, "rk4_record");
    check(llg_rk4_vjp(h, rec.f(), nst, ybar.f(), pgrad.d(), ps.data(), st) == 0, "rk4_vjp");
    check(llg_heun_record(h, m.f(), nst, 3, 7, 0, phs.data(), rec.f(), st) == 0, "heun_record");
    check(llg_heun_vjp(h, rec.f(), nst, 3, 7, 0, ybar.f(), pgrad.d(), phs.data(), st) == 0, "heun_vjp");
    check(llg_vortex_core_position(h, m.f(), lam, nullptr, core.d(), st) == 0, "core position for vjp");
    const double rb[6] = {1.0, 0.5, 1.0, 0.5, 1.0, 0.5};
    HIP_OK(hipMemcpy(rbar.p, rb, sizeof rb, hipMemcpyHostToDevice));
    check(llg_core_position_vjp(h, m.f(), lam, core.d(), rbar.d(), ybar.f(), st) == 0, "core_position_vjp");
    {
        std::vector<double> gp(6);
        HIP_OK(hipMemcpy(gp.data(), pgrad.p, 48, hipMemcpyDeviceToHost));
        bool fin = true;
        for (double v : gp) fin = fin && std::isfinite(v);
        check(fin, "parameter gradients finite");
    }

    // tuning
    int ug = 0, nwg = 0, nt = 0, pol = 0;
    check(llg_tune(h, 2, 3, nullptr) == 0, "tune");
    check(llg_launch_shape(h, &ug, &nwg, &nt, &pol) == 0 && ug == 2 && pol == 3 && nt == 384, "launch_shape");
    double us = 0.0;
    check(llg_autotune(h, m.f(), ps.data(), 0, 3, st, &us) == 0 && us > 0.0, "autotune");
    check(llg_check(h, st) == 0, "check after everything");

    // ---- error paths
    llg_disk bad = nullptr;
    check(llg_build_kernels(30.3, 10.0, 2.0, 0, &bad) == LLG_EINVAL && !bad, "non-integer 2R/a refused");
    check(llg_build_kernels(100.0, 10.0, 2.0, 128, &bad) == LLG_EINVAL && !bad, "P < 2D-1 refused");
    check(llg_build_kernels(30.0, 10.0, 2.0, 96, &bad) == LLG_EUNSUPPORTED && !bad, "unsupported P refused");
    check(llg_rk4_step(nullptr, m.f(), 1, ps.data(), st) == LLG_EINVAL, "null handle refused");
    check(llg_rk4_step(h, nullptr, 1, ps.data(), st) == LLG_EINVAL, "null state refused");
    check(llg_rk4_vjp(h, rec.f(), nst, ybar.f(), pgrad.d(), nullptr, st) == LLG_EINVAL, "null params refused");
    check(llg_set_on_chip(h, 96) == LLG_EINVAL, "bad on-chip limit refused");
    check(llg_power_spectrum(series.d(), 1, 1, 24, 1, 0, 0, pwork.d(), spec.d(), st) == LLG_EINVAL,
          "non-power-of-two spectrum length refused");
    check(std::strlen(llg_last_error()) > 0, "last_error set");
    llg_destroy(h);

    // a lone disk through the single-disk constructor
    llg_disk one = nullptr;
    check(llg_build_kernels(30.0, 10.0, 2.0, 0, &one) == 0 && one, "build_kernels");
    if (one) {
        int D = 0, P = 0, nc = 0;
        check(llg_disk_info(one, 0, &D, &P, &nc) == 0 && D == 30 && P == 64 && nc == 716, "lone disk info");
        Dev m1(3 * 30 * 30 * 4);
        std::vector<float> v(3 * 30 * 30);
        vortex(30, 0.4, 0.3, v.data());
        HIP_OK(hipMemcpy(m1.p, v.data(), v.size() * 4, hipMemcpyHostToDevice));
        check(llg_rk4_step(one, m1.f(), 10, &p, st) == 0 && llg_check(one, st) == 0, "lone disk steps");
        llg_destroy(one);
    }
    HIP_OK(hipStreamDestroy(st));
    std::printf("abi_smoke: %d of %d checks passed\n", g_checks - g_failed, g_checks);
    std::fflush(stdout);
    // leak check now (it ends the process with status 23 on a leak outside the
    // suppressions), then leave without the HIP runtime's own teardown, which
    // the sanitizer's allocator does not survive
    LLG_LEAK_CHECK();
    std::fprintf(stderr, "abi_smoke: leak check done\n");
    _exit(g_failed ? 1 : 0);
}
