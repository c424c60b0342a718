// lib_llgdisk: host side of the C ABI declared in include/llgdisk.h.
//
// Owns geometry set-up (mask, thin-film kernel spectra in float64, twiddle
// tables), workspaces, the workgroup-to-disk map of the persistent launch and
// the parameter staging.  Every step of the hot path runs in the kernels of
// llg_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/llgdisk.h"
#include "llg_aux_kernels.hpp"

namespace llg {
// persistent-kernel instances, one translation unit per mode (kernels_*.hip)
const void* persistent_kernel_field(int UG, int RSEL, int PMAX);
const void* persistent_kernel_rk4(int UG, int RSEL, int PMAX);
const void* persistent_kernel_heun(int UG, int RSEL, int PMAX);
const void* persistent_kernel_vjp(int UG, int RSEL, int PMAX);
const void* persistent_kernel_heun_vjp(int UG, int RSEL, int PMAX);
const void* persistent_kernel_relax(int UG, int RSEL, int PMAX);
const void* persistent_kernel_rk4_series(int UG, int RSEL, int PMAX);
const void* persistent_kernel_heun_series(int UG, int RSEL, int PMAX);
}  // namespace llg

using namespace llg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(LLG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

// ------------------------------------------------------------------ geometry
// Thin-film kernels of Sec. II.B at displacement (u, v) in units of a, ell = L/a.
void green(double u, double v, double ell, double* kxx, double* kyy, double* kxy, double* kzz) {
    const double r2 = u * u + v * v;
    if (r2 == 0.0) {
        const double ro = 1.0 / std::sqrt(M_PI);
        const double so = std::sqrt(ell * ell + ro * ro);
        const double nz = (ell + ro - so) / ell;
        const double nx = (so - ro) / (2.0 * ell);
        *kxx = -nx;
        *kyy = -nx;
        *kxy = 0.0;
        *kzz = -nz;
        return;
    }
    const double r = std::sqrt(r2), s = std::sqrt(r2 + ell * ell);
    const double pre = ell / (2.0 * M_PI * r2 * r2);
    *kxx = pre * (u * u / s - v * v / (s + r));
    *kyy = pre * (v * v / s - u * u / (s + r));
    *kxy = pre * ((2.0 * s + r) / (s + r)) * (u * v / s);
    *kzz = -ell / (2.0 * M_PI * r * s * (s + r));
}

// In-place radix-2 complex FFT (forward, e^{-i}), float64, host.
void fft1d(std::complex<double>* x, int n, int stride) {
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[(size_t)i * stride], x[(size_t)j * stride]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * M_PI / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const std::complex<double> w(std::cos(ang * k), std::sin(ang * k));
                std::complex<double>& a = x[(size_t)(i + k) * stride];
                std::complex<double>& b = x[(size_t)(i + k + len / 2) * stride];
                const std::complex<double> t = w * b;
                b = a - t;
                a = a + t;
            }
    }
}

struct Geom {
    int D, P, n_cells;
    double ell;
    float* spec = nullptr;           // device [4][H][H]
    unsigned char* mask = nullptr;   // device [D][D]
};

// Quarter-plane real spectra / P^2 of the four wrapped kernels, [4][H][H].
std::vector<float> kernel_spectra(int D, int P, double ell) {
    const int H = P / 2 + 1;
    std::vector<float> out((size_t)4 * H * H);
    std::vector<std::complex<double>> w((size_t)P * P);
    for (int q = 0; q < 4; ++q) {
        std::fill(w.begin(), w.end(), std::complex<double>(0.0, 0.0));
        for (int v = -(D - 1); v <= D - 1; ++v)
            for (int u = -(D - 1); u <= D - 1; ++u) {
                double k[4];
                green(u, v, ell, &k[0], &k[1], &k[2], &k[3]);
                w[(size_t)((v + P) % P) * P + ((u + P) % P)] = k[q];
            }
        for (int row = 0; row < P; ++row) fft1d(&w[(size_t)row * P], P, 1);
        for (int col = 0; col < P; ++col) fft1d(&w[col], P, P);
        const double inv = 1.0 / ((double)P * P);
        for (int kx = 0; kx < H; ++kx)
            for (int ky = 0; ky < H; ++ky)
                out[((size_t)q * H + kx) * H + ky] = (float)(w[(size_t)ky * P + kx].real() * inv);
    }
    return out;
}

std::vector<unsigned char> disk_mask(int D, int* n_cells) {
    std::vector<unsigned char> m((size_t)D * D);
    const double c = (D - 1) / 2.0, r2 = (D / 2.0) * (D / 2.0);
    int n = 0;
    for (int j = 0; j < D; ++j)
        for (int i = 0; i < D; ++i) {
            const double x = i - c, y = j - c;
            const bool in = x * x + y * y <= r2;
            m[(size_t)j * D + i] = in;
            n += in;
        }
    *n_cells = n;
    return m;
}

// Transform policy: bit 0 = radix 8 everywhere (else radix 4 below P = 512),
// bit 1 = one lane group per column with all three components (else one
// wavefront per component).
int radix_for(int P, int RSEL) { return ((RSEL & 1) == 1 || P == 512) ? 8 : 4; }

}  // namespace

struct llg_disk_s {
    int device = 0;
    int n = 0;
    double a_nm = 2.0;
    std::vector<int> D, P, n_cells, G;
    std::vector<double> R_nm, L_nm;
    std::vector<long long> m_off;
    long long state_size = 0;
    std::vector<Geom> geoms;
    std::vector<int> geom_of;
    std::map<int, float2*> twiddles;
    std::vector<void*> allocs;
    DiskDesc* desc_dev = nullptr;
    DiskPrm* prm_dev = nullptr;
    DiskPrm* prm_pin = nullptr;
    std::vector<DiskPrm> prm_cache;
    bool prm_valid = false;
    hipEvent_t prm_event = nullptr;
    double* hint_dev = nullptr;
    double* hint_pin = nullptr;
    hipEvent_t hint_event = nullptr;
    static constexpr int N_MODES = 8;
    hipEvent_t time_ev[N_MODES][2] = {};          // opt-in launch timing (llg_timing), per mode
    bool time_valid[N_MODES] = {};                // a launch of that mode was timed since enabling
    bool timing = false;
    int* wg2disk = nullptr;
    int* wg2local = nullptr;
    int n_wg = 0;
    unsigned int* bars = nullptr;
    int n_bars = 0;
    int* err_dev = nullptr;
    unsigned long long* step_dev = nullptr;   // Heun step counter (LLG_STEP_COUNTER)
    CorePart* core_part = nullptr;    // per disk and plaquette-row strip: core-position candidates
    int core_strips = 1;              // strips per disk in core_part
    unsigned plan_modes = 0;          // modes whose co-residency the current plan was checked for
    unsigned plan_series_modes = 0;   // the same for the series instances of the integrators
    int UG = 1;                       // wavefront groups per workgroup of the persistent launch
    int RSEL = 0;                     // transform policy (radix and column strategy)
    int PMAX = 256;                   // largest FFT size of the handle's disks (kernel instance)
    int onchip_pmax = 0;              // disks with P <= this (64 or 128; 0: none) run on one workgroup, spectra in LDS
    unsigned spin_limit = SPIN_LIMIT; // polls of a group-barrier wait before it raises ERR_BARRIER
    unsigned onchip_lds = 0;          // dynamic LDS bytes of the on-chip capable launches (largest on-chip workspace)
    std::vector<DiskDesc> desc;       // host copy of the descriptors

    ~llg_disk_s() {
        for (void* p : allocs) (void)hipFree(p);
        if (prm_pin) (void)hipHostFree(prm_pin);
        if (hint_pin) (void)hipHostFree(hint_pin);
        if (prm_event) (void)hipEventDestroy(prm_event);
        if (hint_event) (void)hipEventDestroy(hint_event);
        for (auto& pair : time_ev)
            for (hipEvent_t e : pair)
                if (e) (void)hipEventDestroy(e);
    }
    template <typename T>
    int dalloc(T** p, size_t count) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) return fail(LLG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *p = static_cast<T*>(q);
        return 0;
    }
    void dfree(void* p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) {
            (void)hipFree(p);
            allocs.erase(it);
        }
    }
};

// An executable graph of one persistent launch (barrier reset, integrator,
// step-counter advance) with its own copies of the parameters and of the
// launch plan (workgroup maps, descriptors with their partial-sum buffers), so
// that a later re-plan of the handle leaves the graph's launch intact.
struct llg_graph_s {
    llg_disk h = nullptr;
    std::vector<void*> allocs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~llg_graph_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void* p : allocs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t dalloc(T** p, size_t count) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) {
            allocs.push_back(q);
            *p = static_cast<T*>(q);
        }
        return e;
    }
};

namespace {

const void* persistent_kernel(int mode, int UG, int RSEL, int PMAX, bool series = false) {
    if (series) return mode == MODE_HEUN ? persistent_kernel_heun_series(UG, RSEL, PMAX)
                                         : persistent_kernel_rk4_series(UG, RSEL, PMAX);
    switch (mode) {
        case MODE_RK4: return persistent_kernel_rk4(UG, RSEL, PMAX);
        case MODE_HEUN: return persistent_kernel_heun(UG, RSEL, PMAX);
        case MODE_RK4_VJP: return persistent_kernel_vjp(UG, RSEL, PMAX);
        case MODE_HEUN_VJP: return persistent_kernel_heun_vjp(UG, RSEL, PMAX);
        case MODE_RELAX: return persistent_kernel_relax(UG, RSEL, PMAX);
        default: return persistent_kernel_field(UG, RSEL, PMAX);
    }
}

constexpr unsigned ALL_MODES = (1u << MODE_DEMAG) | (1u << MODE_RK4) | (1u << MODE_HEUN) | (1u << MODE_RK4_VJP) |
                               (1u << MODE_HEUN_VJP) | (1u << MODE_RELAX);

// Largest on-chip spectra workspace: P = 128, D' = 64 (3 x 65 x 64 complex floats).
constexpr unsigned MAX_ONCHIP_LDS = 3u * 65u * 64u * 8u;

// Declare the largest dynamic LDS request of a kernel (the on-chip spectra of
// any handle, so that handles of different sizes never lower it for each
// other) before its occupancy query and launch.  A size the device cannot hold
// shows up as zero resident workgroups in the occupancy query, so the call's
// own status is not needed.
void allow_dynamic_lds(const void* k) {
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)MAX_ONCHIP_LDS);
    (void)hipGetLastError();
}

// Workgroups of the given shape that the kernels of every mode in `modes` (bit
// mask) can keep co-resident; the field and integrator kernels carry
// `onchip_lds` bytes of dynamic LDS (the spectra of on-chip disks).
int max_coresident_workgroups(int UG, int RSEL, int PMAX, int* out, unsigned modes = ALL_MODES,
                              unsigned onchip_lds = 0) {
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 1 << 30;
    for (int mode : {MODE_DEMAG, MODE_RK4, MODE_HEUN, MODE_RK4_VJP, MODE_HEUN_VJP, MODE_RELAX}) {
        if (!(modes & (1u << mode))) continue;
        const void* k = persistent_kernel(mode, UG, RSEL, PMAX);
        if (!k) return fail(LLG_EUNSUPPORTED, "no kernel instance for this launch shape");
        int b = 0;
        const unsigned dyn = on_chip_instance(mode, UG) ? onchip_lds : 0;
        if (dyn) allow_dynamic_lds(k);
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, WG_THREADS * UG, dyn));
        per_cu = std::min(per_cu, b);
    }
    *out = ncu * per_cu;
    return 0;
}

int choose_P(int D, int P_override, int* P) {
    const int need = 2 * D - 1;
    if (P_override == 0) {
        int p = 64;
        while (p < 2 * D) p *= 2;
        *P = p;
    } else {
        *P = P_override;
    }
    if (*P != 64 && *P != 128 && *P != 256 && *P != 512)
        return fail(LLG_EUNSUPPORTED, "FFT size " + std::to_string(*P) + " unsupported (64, 128, 256 or 512; disks up to D = 256)");
    if (*P < need) return fail(LLG_EINVAL, "P = " + std::to_string(*P) + " < 2D-1 = " + std::to_string(need));
    return 0;
}

// Units (transforms per component) a workgroup carries at once, for FFT size P.
int units_per_wg(int P, int UG, int RSEL) { return UG * (64 / (P / radix_for(P, RSEL))); }

int default_unit_groups(llg_disk) {
    // narrow workgroups spread a disk over the most CUs; measured best for a
    // lone D=100 disk (one transform per workgroup and phase) and for batches
    return 1;
}

// Workgroups per disk and the workgroup-to-disk map of the persistent launch.
//
// Without explicit counts the plan minimises the slowest disk's estimated
// stage time within a budget of scale x the co-resident workgroups: disk k on
// G workgroups takes ceil(ncb/G) column and ceil(nrb/G) row iterations of cost
// U P log2 P each (with lane-group columns, ceil(ncb3/G) column iterations of
// three times that, ncb3 = tiles of 3U columns) plus, for G > 1, two group
// barriers (2500 in the same units: the measured ratio of a barrier to a
// single-transform P = 256 column iteration); the smallest target T whose
// per-disk counts (the fewest workgroups that meet T) fit the budget is found
// by bisection.  Disks on chip (P <= h->onchip_pmax) take one workgroup each.
int plan(llg_disk h, int UG, int RSEL, const int* wg_per_disk, unsigned modes = ALL_MODES, double scale = 1.0) {
    if (UG != 1 && UG != 2 && UG != 4) return fail(LLG_EINVAL, "unit groups must be 1, 2 or 4");
    if (RSEL < 0 || RSEL > 3) return fail(LLG_EINVAL, "transform policy must be 0, 1, 2 or 3");
    const int n = h->n;
    if (h->onchip_pmax > 0 && UG != 1)
        return fail(LLG_EUNSUPPORTED, "spectra on chip need one unit group per workgroup");
    std::vector<char> oc(n, 0);
    unsigned oc_lds = 0;
    for (int k = 0; k < n; ++k) {
        oc[k] = h->onchip_pmax > 0 && h->P[k] <= h->onchip_pmax;
        if (oc[k]) oc_lds = std::max(oc_lds, (unsigned)(3 * (h->P[k] / 2 + 1) * h->desc[k].Dp * sizeof(float2)));
    }
    int cap = 0;
    int rc = max_coresident_workgroups(UG, RSEL, h->PMAX, &cap, modes, oc_lds);
    if (rc) return rc;
    if (cap <= 0)
        return fail(LLG_EUNSUPPORTED, "no workgroup of " + std::to_string(WG_THREADS * UG) + " threads fits a CU with " +
                                          std::to_string(oc_lds) + " bytes of on-chip spectra");
    std::vector<int> useful(n), G(n), ncb(n), nrb(n);
    std::vector<double> work(n), iter(n);
    for (int k = 0; k < n; ++k) {
        const int P = h->P[k], D = h->D[k];
        const int U = units_per_wg(P, UG, RSEL);
        const int H = P / 2 + 1;
        const int n_pairs = (D + 1) / 2;
        ncb[k] = (RSEL & 2) ? (H + 3 * U - 1) / (3 * U) : (H + U - 1) / U;
        nrb[k] = (n_pairs + U - 1) / U;
        useful[k] = std::max(ncb[k], nrb[k]);
        work[k] = (double)(n_pairs + H) * P * std::log2((double)P);
        iter[k] = (double)U * P * std::log2((double)P);
    }
    const int col_weight = (RSEL & 2) ? 3 : 1;
    auto stage_time = [&](int k, int g) {
        return (col_weight * ((ncb[k] + g - 1) / g) + (nrb[k] + g - 1) / g) * iter[k] + (g > 1 ? 5000.0 : 0.0);
    };
    // fewest workgroups for disk k that meet the target T (or all useful ones)
    auto g_for = [&](int k, double T) {
        if (oc[k]) return 1;
        int g = 1;
        while (g < useful[k] && stage_time(k, g) > T) ++g;
        return g;
    };
    if (wg_per_disk) {
        for (int k = 0; k < n; ++k) {
            if (wg_per_disk[k] < 1) return fail(LLG_EINVAL, "wg_per_disk must be >= 1");
            G[k] = oc[k] ? 1 : std::min(wg_per_disk[k], useful[k]);
        }
    } else {
        if (!(scale > 0.0 && scale <= 1.0)) return fail(LLG_EINVAL, "plan scale must be in (0, 1]");
        const long long budget = std::max<long long>(n, (long long)std::floor(cap * scale));
        double lo = 0.0, hi = 0.0;
        for (int k = 0; k < n; ++k) hi = std::max(hi, stage_time(k, 1));
        auto total = [&](double T) {
            long long t = 0;
            for (int k = 0; k < n; ++k) t += g_for(k, T);
            return t;
        };
        for (int it = 0; it < 60; ++it) {   // smallest T whose counts fit the budget
            const double mid = 0.5 * (lo + hi);
            if (total(mid) <= budget)
                hi = mid;
            else
                lo = mid;
        }
        for (int k = 0; k < n; ++k) G[k] = g_for(k, hi);
    }
    long long total = std::accumulate(G.begin(), G.end(), 0LL);
    while (total > cap) {  // trim the disks with the most workgroups
        int kmax = (int)(std::max_element(G.begin(), G.end()) - G.begin());
        if (G[kmax] <= 1) break;
        --G[kmax];
        --total;
    }
    if (total > cap)
        return fail(LLG_EUNSUPPORTED, "batch needs " + std::to_string(total) + " workgroups but only " +
                                          std::to_string(cap) + " can be co-resident");

    // Disks whose workgroups all fit one XCD stay on one XCD (workgroup w runs
    // on XCD w mod 8); larger disks take consecutive ids and span the XCDs.
    constexpr int NXCD = 8;
    std::vector<int> w2d, w2l;
    {
        std::vector<std::vector<std::pair<int, int>>> lanes(NXCD);
        std::vector<long long> load(NXCD, 0);
        std::vector<int> big;
        std::vector<int> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return G[x] > G[y]; });
        for (int k : order) {
            if (n > 1 && G[k] * NXCD <= cap) {
                const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                for (int l = 0; l < G[k]; ++l) lanes[x].push_back({k, l});
                load[x] += (long long)G[k] * (long long)work[k];
            } else {
                big.push_back(k);
            }
        }
        for (int k : big)
            for (int l = 0; l < G[k]; ++l) {
                w2d.push_back(k);
                w2l.push_back(l);
            }
        while (w2d.size() % NXCD) {
            w2d.push_back(-1);
            w2l.push_back(0);
        }
        size_t depth = 0;
        for (auto& l : lanes) depth = std::max(depth, l.size());
        for (size_t s = 0; s < depth; ++s)
            for (int x = 0; x < NXCD; ++x) {
                if (s < lanes[x].size()) {
                    w2d.push_back(lanes[x][s].first);
                    w2l.push_back(lanes[x][s].second);
                } else {
                    w2d.push_back(-1);
                    w2l.push_back(0);
                }
            }
        while (!w2d.empty() && w2d.back() < 0) {
            w2d.pop_back();
            w2l.pop_back();
        }
    }
    if ((int)w2d.size() > cap) {  // the XCD-aligned layout does not fit: consecutive ids
        w2d.clear();
        w2l.clear();
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < G[k]; ++l) {
                w2d.push_back(k);
                w2l.push_back(l);
            }
    }
    h->dfree(h->wg2disk);
    h->dfree(h->wg2local);
    h->wg2disk = h->wg2local = nullptr;
    if ((rc = h->dalloc(&h->wg2disk, w2d.size()))) return rc;
    if ((rc = h->dalloc(&h->wg2local, w2l.size()))) return rc;
    HIP_TRY(hipMemcpy(h->wg2disk, w2d.data(), w2d.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->wg2local, w2l.data(), w2l.size() * sizeof(int), hipMemcpyHostToDevice));
    h->n_wg = (int)w2d.size();
    for (int k = 0; k < n; ++k) {
        DiskDesc& d = h->desc[k];
        h->dfree(d.part);
        d.part = nullptr;
        if ((rc = h->dalloc(&d.part, (size_t)PART_STRIDE * G[k]))) return rc;
        d.G = G[k];
        d.onchip = oc[k];
    }
    h->onchip_lds = oc_lds;
    h->G = G;
    h->UG = UG;
    h->RSEL = RSEL;
    h->plan_modes = modes;
    h->plan_series_modes = 0;
    if (!h->desc_dev && (rc = h->dalloc(&h->desc_dev, n))) return rc;
    HIP_TRY(hipMemcpy(h->desc_dev, h->desc.data(), n * sizeof(DiskDesc), hipMemcpyHostToDevice));
    return 0;
}

int create(int n, const double* R_nm, const double* L_nm, double a_nm, const int* wg_per_disk,
           const int* P_override, llg_disk* out) {
    if (!out) return fail(LLG_EINVAL, "null output handle");
    *out = nullptr;
    if (n <= 0 || !R_nm || !L_nm) return fail(LLG_EINVAL, "need n >= 1 disks");
    if (!(a_nm > 0)) return fail(LLG_EINVAL, "cell edge must be positive");
    // owned until the end: every early return (HIP_TRY included) frees the partial handle
    std::unique_ptr<llg_disk_s> owner(new llg_disk_s());
    llg_disk h = owner.get();
    HIP_TRY(hipGetDevice(&h->device));
    h->n = n;
    h->a_nm = a_nm;
    std::map<std::tuple<int, int, long long>, int> geom_index;
    for (int k = 0; k < n; ++k) {
        const double dd = 2.0 * R_nm[k] / a_nm;
        const int D = (int)std::lround(dd);
        if (!(std::fabs(dd - D) <= 1e-9) || D < 1)
            return fail(LLG_EINVAL, "disk " + std::to_string(k) + ": 2R/a is not a positive integer");
        if (!(L_nm[k] > 0)) return fail(LLG_EINVAL, "disk " + std::to_string(k) + ": thickness must be positive");
        int P = 0;
        int rc = choose_P(D, P_override ? P_override[k] : 0, &P);
        if (rc) return rc;
        const double ell = L_nm[k] / a_nm;
        const auto key = std::make_tuple(D, P, (long long)std::llround(ell * 1e12));
        auto it = geom_index.find(key);
        int gi;
        if (it == geom_index.end()) {
            Geom g;
            g.D = D;
            g.P = P;
            g.ell = ell;
            std::vector<unsigned char> mk = disk_mask(D, &g.n_cells);
            std::vector<float> sp = kernel_spectra(D, P, ell);
            if ((rc = h->dalloc(&g.mask, mk.size()))) return rc;
            if ((rc = h->dalloc(&g.spec, sp.size()))) return rc;
            HIP_TRY(hipMemcpy(g.mask, mk.data(), mk.size(), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(g.spec, sp.data(), sp.size() * sizeof(float), hipMemcpyHostToDevice));
            gi = (int)h->geoms.size();
            h->geoms.push_back(g);
            geom_index[key] = gi;
        } else {
            gi = it->second;
        }
        if (!h->twiddles.count(P)) {
            std::vector<float2> tw(P);
            for (int e = 0; e < P; ++e)
                tw[e] = make_float2((float)std::cos(2.0 * M_PI * e / P), (float)(-std::sin(2.0 * M_PI * e / P)));
            float2* tdev = nullptr;
            if ((rc = h->dalloc(&tdev, P))) return rc;
            HIP_TRY(hipMemcpy(tdev, tw.data(), P * sizeof(float2), hipMemcpyHostToDevice));
            h->twiddles[P] = tdev;
        }
        h->geom_of.push_back(gi);
        h->D.push_back(D);
        h->P.push_back(P);
        h->n_cells.push_back(h->geoms[gi].n_cells);
        h->R_nm.push_back(R_nm[k]);
        h->L_nm.push_back(L_nm[k]);
        h->m_off.push_back(h->state_size);
        h->state_size += 3LL * D * D;
        if (P > h->PMAX) h->PMAX = P;
    }

    // ---- per-disk workspaces
    int rc = 0;
    h->n_bars = n * 32;  // one 128-byte line per disk
    if ((rc = h->dalloc(&h->bars, h->n_bars))) return rc;
    if ((rc = h->dalloc(&h->err_dev, 1))) return rc;
    HIP_TRY(hipMemset(h->err_dev, 0, sizeof(int)));
    if ((rc = h->dalloc(&h->step_dev, 1))) return rc;
    {
        int dmax = 1;
        for (int D : h->D) dmax = std::max(dmax, D);
        h->core_strips = std::max(1, (dmax - 1 + CORE_ROWS - 1) / CORE_ROWS);
        if ((rc = h->dalloc(&h->core_part, (size_t)n * h->core_strips))) return rc;
    }
    HIP_TRY(hipMemset(h->step_dev, 0, sizeof(unsigned long long)));
    h->desc.assign(n, DiskDesc{});
    for (int k = 0; k < n; ++k) {
        DiskDesc& d = h->desc[k];
        const Geom& g = h->geoms[h->geom_of[k]];
        d.D = h->D[k];
        d.P = h->P[k];
        d.H = d.P / 2 + 1;
        d.Dp = (d.D + SB - 1) / SB * SB;
        d.n_pairs = (d.D + 1) / 2;
        d.n_cells = g.n_cells;
        d.k = k;
        d.m_off = h->m_off[k];
        const size_t DD = (size_t)d.D * d.D;
        if ((rc = h->dalloc(&d.ya, 3 * DD))) return rc;
        if ((rc = h->dalloc(&d.yb, 3 * DD))) return rc;
        if ((rc = h->dalloc(&d.acc, 3 * DD))) return rc;
        if ((rc = h->dalloc(&d.aux, 3 * DD))) return rc;
        if ((rc = h->dalloc(&d.S, (size_t)3 * d.H * d.Dp))) return rc;
        HIP_TRY(hipMemset(d.S, 0, (size_t)3 * d.H * d.Dp * sizeof(float2)));
        d.spec = g.spec;
        d.mask = g.mask;
        d.tw = h->twiddles[d.P];
        d.bar = h->bars + 32 * k;
    }
    if ((rc = plan(h, default_unit_groups(h), 0, wg_per_disk))) return rc;
    if ((rc = h->dalloc(&h->prm_dev, n))) return rc;
    if ((rc = h->dalloc(&h->hint_dev, 2 * (size_t)n))) return rc;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->prm_pin), n * sizeof(DiskPrm), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->hint_pin), 2 * n * sizeof(double), hipHostMallocDefault));
    HIP_TRY(hipEventCreateWithFlags(&h->prm_event, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&h->hint_event, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(h->prm_event, 0));
    HIP_TRY(hipEventRecord(h->hint_event, 0));
    h->prm_cache.resize(n);
    HIP_TRY(hipDeviceSynchronize());
    *out = owner.release();
    return 0;
}

int upload_params(llg_disk h, const llg_params* p, hipStream_t st) {
    if (!p) return fail(LLG_EINVAL, "null params");
    std::vector<DiskPrm> v(h->n);
    std::memset(static_cast<void*>(v.data()), 0, v.size() * sizeof(DiskPrm));   // padding compares equal
    for (int k = 0; k < h->n; ++k) {
        const llg_params& q = p[k];
        if (!(q.dtau >= 0) || !(q.alpha >= 0) || !(q.temp >= 0) || !std::isfinite(q.c))
            return fail(LLG_EINVAL, "invalid parameters for disk " + std::to_string(k));
        const bool pulse = q.hpulse[0] != 0.0 || q.hpulse[1] != 0.0 || q.hpulse[2] != 0.0;
        const bool osc = q.hac[0] != 0.0 || q.hac[1] != 0.0 || q.hac[2] != 0.0;
        bool finite = std::isfinite(q.freq) && std::isfinite(q.phase) && std::isfinite(q.tpulse) &&
                      std::isfinite(q.wpulse) && std::isfinite(q.tau0);
        for (int c = 0; c < 3; ++c) finite = finite && std::isfinite(q.hac[c]) && std::isfinite(q.hpulse[c]) &&
                                             std::isfinite(q.hext[c]);
        if (!finite || (pulse && !(q.wpulse > 0)))
            return fail(LLG_EINVAL, "invalid driving field for disk " + std::to_string(k) +
                                        " (non-finite value, or a pulse without a positive width)");
        DiskPrm& d = v[k];
        d.alpha = (float)q.alpha;
        d.c = (float)q.c;
        d.hx = (float)q.hext[0];
        d.hy = (float)q.hext[1];
        d.hz = (float)q.hext[2];
        d.dtau = (float)q.dtau;
        double var = 2.0 * q.alpha * q.temp * q.dtau;
        double dvar = 2.0 * q.temp * q.dtau;   // d var / d alpha
        if (q.fd_factor) {
            const double s = 1.0 + q.alpha * q.alpha;
            var /= s;
            dvar *= (1.0 - q.alpha * q.alpha) / (s * s);
        }
        d.sigma = (float)std::sqrt(var);
        d.dsigma = var > 0.0 ? (float)(dvar / (2.0 * std::sqrt(var))) : 0.0f;
        d.renorm = q.renorm ? 1 : 0;
        d.c_d = q.c;
        d.hx_d = q.hext[0];
        d.hy_d = q.hext[1];
        d.hz_d = q.hext[2];
        d.dtau_d = q.dtau;
        d.tau0 = q.tau0;
        d.drive = (osc || pulse) ? 1 : 0;
        for (int c = 0; c < 3; ++c) {
            d.hac[c] = osc ? q.hac[c] : 0.0;
            d.hpulse[c] = pulse ? q.hpulse[c] : 0.0;
        }
        d.freq = q.freq;
        d.phase = q.phase;
        d.tpulse = q.tpulse;
        d.inv2w2 = pulse ? 1.0 / (2.0 * q.wpulse * q.wpulse) : 0.0;
        for (int c = 0; c < 3; ++c) {
            d.hacf[c] = (float)d.hac[c];
            d.hpulsef[c] = (float)d.hpulse[c];
        }
        const double prv = q.phase / (2.0 * M_PI);
        d.phase_rev = (float)(prv - std::floor(prv));
        if (d.phase_rev >= 1.0f) d.phase_rev = 0.0f;
        d.inv2w2_log2e = (float)(d.inv2w2 / std::log(2.0));
    }
    if (h->prm_valid && std::memcmp(v.data(), h->prm_cache.data(), v.size() * sizeof(DiskPrm)) == 0) return 0;
    HIP_TRY(hipEventSynchronize(h->prm_event));  // the staging buffer is free again
    std::memcpy(h->prm_pin, v.data(), v.size() * sizeof(DiskPrm));
    HIP_TRY(hipMemcpyAsync(h->prm_dev, h->prm_pin, v.size() * sizeof(DiskPrm), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(h->prm_event, st));
    h->prm_cache = v;
    h->prm_valid = true;
    return 0;
}

KArgs make_args(llg_disk h, const DiskPrm* prm, int mode, float* m, float* out, long long nsteps,
                unsigned long long seed, unsigned long long step0, unsigned int replica0,
                const unsigned long long* step_ptr, float* rec, const double* relax_x, double* relax_out,
                double kappa, double tol, double relax_cut2 = 0.0) {
    KArgs a;
    a.disks = h->desc_dev;
    a.prm = prm;
    a.wg2disk = h->wg2disk;
    a.wg2local = h->wg2local;
    a.m = m;
    a.out = out;
    a.rec = rec;
    a.relax_x = relax_x;
    a.relax_out = relax_out;
    a.kappa = kappa;
    a.tol = tol;
    a.relax_cut2 = relax_cut2;
    a.nsteps = nsteps;
    a.seed = seed;
    a.step0 = step0;
    a.step_ptr = step_ptr;
    a.replica0 = replica0;
    a.mode = mode;
    a.err = h->err_dev;
    a.series = nullptr;
    a.every = 0;
    a.n_disks = h->n;
    a.spin_limit = h->spin_limit;
    return a;
}

int launch(llg_disk h, int mode, float* m, float* out, long long nsteps, unsigned long long seed,
           unsigned long long step0, unsigned int replica0, hipStream_t st, float* rec = nullptr,
           const double* relax_x = nullptr, double* relax_out = nullptr, double kappa = 0.0, double tol = 0.0,
           const unsigned long long* step_ptr = nullptr, double relax_cut2 = 0.0,
           const DiskDesc* desc_override = nullptr, unsigned int* bars_override = nullptr,
           double* series = nullptr, long long every = 0) {
    const int kmode = (mode == MODE_RHS || mode == MODE_ENERGY) ? MODE_DEMAG : mode;   // kernel of the mode
    const unsigned dyn = on_chip_instance(kmode, h->UG) ? h->onchip_lds : 0;   // on-chip spectra
    if (!(h->plan_modes & (1u << kmode))) {
        int cap = 0;
        int rc = max_coresident_workgroups(h->UG, h->RSEL, h->PMAX, &cap, 1u << kmode, h->onchip_lds);
        if (rc) return rc;
        if (h->n_wg > cap)
            return fail(LLG_EUNSUPPORTED, "the launch plan (" + std::to_string(h->n_wg) +
                                              " workgroups, tuned for the integrator) exceeds what this mode keeps "
                                              "co-resident (" + std::to_string(cap) + "); re-plan with llg_tune");
        h->plan_modes |= 1u << kmode;   // checked once per plan
    }
    if (series && !(h->plan_series_modes & (1u << kmode))) {   // the series instance: its own co-residency, once per plan
        const void* k = persistent_kernel(mode, h->UG, h->RSEL, h->PMAX, true);
        if (!k) return fail(LLG_EUNSUPPORTED, "no series kernel instance for this launch shape");
        int dev = 0, ncu = 0, b = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if (dyn) allow_dynamic_lds(k);
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, WG_THREADS * h->UG, dyn));
        if (h->n_wg > ncu * b)
            return fail(LLG_EUNSUPPORTED, "the launch plan (" + std::to_string(h->n_wg) +
                                              " workgroups) exceeds what the series kernel keeps co-resident (" +
                                              std::to_string(ncu * b) + "); re-plan with llg_tune");
        h->plan_series_modes |= 1u << kmode;
    }
    const int nb = (h->n_bars + 255) / 256;
    hipLaunchKernelGGL(zero_u32, dim3(nb), dim3(256), 0, st, bars_override ? bars_override : h->bars, h->n_bars);
    HIP_TRY(hipGetLastError());
    KArgs a = make_args(h, h->prm_dev, mode, m, out, nsteps, seed, step0, replica0, step_ptr, rec, relax_x,
                        relax_out, kappa, tol, relax_cut2);
    if (desc_override) a.disks = desc_override;
    a.series = series;
    a.every = (int)every;
    void* args[] = {&a};
    if (h->timing) HIP_TRY(hipEventRecord(h->time_ev[mode][0], st));
    HIP_TRY(hipLaunchCooperativeKernel(persistent_kernel(mode, h->UG, h->RSEL, h->PMAX, series != nullptr),
                                       dim3(h->n_wg), dim3(WG_THREADS * h->UG), args, dyn, st));
    if (h->timing) {
        HIP_TRY(hipEventRecord(h->time_ev[mode][1], st));
        h->time_valid[mode] = true;
    }
    if (step_ptr) {
        hipLaunchKernelGGL(advance_u64, dim3(1), dim3(64), 0, st, h->step_dev, (unsigned long long)nsteps);
        HIP_TRY(hipGetLastError());
    }
    return 0;
}

// ---------------------------------------------------------------- fixed scratch array
// Workspaces of llg_rk4_step_noalloc: one array per GPU for the life of the
// process.  Layout (every block 256-byte aligned): the descriptor table of the
// handle's disks, the barrier counters (one 128-byte line per disk), then per
// disk the stage states A and B, the RK4 accumulator, the row/column spectra
// and the per-workgroup partial sums.
static __device__ __align__(256) unsigned char scratch[LLG_NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

__host__ __device__ inline unsigned long long align256(unsigned long long b) { return (b + 255ull) & ~255ull; }
__host__ __device__ inline unsigned long long scratch_head(int n) {
    return align256((unsigned long long)n * sizeof(DiskDesc)) + align256((unsigned long long)n * 32 * sizeof(unsigned));
}
__host__ __device__ inline unsigned long long scratch_disk_bytes(int D, int H, int Dp, int G) {
    const unsigned long long st = align256((unsigned long long)3 * D * D * sizeof(float));
    return 3 * st + align256((unsigned long long)3 * H * Dp * sizeof(float2)) +
           align256((unsigned long long)PART_STRIDE * G * sizeof(double));
}

// Descriptor table in the scratch array: disk k as in the handle's table, its
// workspaces redirected into its block (offsets summed over the disks before it).
__global__ void scratch_descriptors(const DiskDesc* src, int n, unsigned char* base) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    unsigned long long off = scratch_head(n);
    for (int q = 0; q < k; ++q) off += scratch_disk_bytes(src[q].D, src[q].H, src[q].Dp, src[q].G);
    DiskDesc d = src[k];
    const unsigned long long st = align256((unsigned long long)3 * d.D * d.D * sizeof(float));
    unsigned char* p = base + off;
    d.ya = reinterpret_cast<float*>(p);
    d.yb = reinterpret_cast<float*>(p + st);
    d.acc = reinterpret_cast<float*>(p + 2 * st);
    d.aux = nullptr;
    d.S = reinterpret_cast<float2*>(p + 3 * st);
    d.part = reinterpret_cast<double*>(p + 3 * st + align256((unsigned long long)3 * d.H * d.Dp * sizeof(float2)));
    d.bar = reinterpret_cast<unsigned int*>(base + align256((unsigned long long)n * sizeof(DiskDesc))) + 32 * k;
    reinterpret_cast<DiskDesc*>(base)[k] = d;
}

// Device address of this device's scratch array, looked up once per device.
int scratch_ptr(int dev, unsigned char** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LLG_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(LLG_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return 0;
}

int check_handle(llg_disk h) {
    if (!h) return fail(LLG_EINVAL, "null handle");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) return fail(LLG_EINVAL, "handle belongs to device " + std::to_string(h->device));
    return 0;
}

}  // namespace

extern "C" {

int llg_params_from_si(double A, double Ms, double gamma, double a_nm, double L_nm, double dt_ps, double T_K,
                       double alpha, llg_params* out, double* lambda_ex_nm) {
    if (!out) return fail(LLG_EINVAL, "null output");
    if (!(A > 0 && Ms > 0 && gamma > 0 && a_nm > 0 && L_nm > 0 && dt_ps >= 0 && T_K >= 0 && alpha >= 0))
        return fail(LLG_EINVAL, "material and grid parameters must be positive");
    const double mu0 = 4e-7 * M_PI, kB = 1.380649e-23;
    const double a = a_nm * 1e-9, L = L_nm * 1e-9;
    const double lam = std::sqrt(2.0 * A / (mu0 * Ms * Ms));
    const double B0 = 2.0 * A / (a * a * Ms);
    const double t0 = 1.0 / (gamma * B0);
    std::memset(out, 0, sizeof(*out));
    out->alpha = alpha;
    out->c = (a / lam) * (a / lam);
    out->temp = kB * T_K / (2.0 * A * L);
    out->dtau = dt_ps * 1e-12 / t0;
    if (lambda_ex_nm) *lambda_ex_nm = lam * 1e9;
    return 0;
}

int llg_build_kernels(double R_nm, double L_nm, double a_nm, int P_override, llg_disk* out) {
    return create(1, &R_nm, &L_nm, a_nm, nullptr, &P_override, out);
}

int llg_batch_create(int n, const double* R_nm, const double* L_nm, double a_nm, const int* wg_per_disk,
                     llg_disk* out) {
    return create(n, R_nm, L_nm, a_nm, wg_per_disk, nullptr, out);
}

int llg_disk_count(llg_disk h) { return h ? h->n : fail(LLG_EINVAL, "null handle"); }

int llg_disk_info(llg_disk h, int k, int* D, int* P, int* n_cells) {
    if (!h || k < 0 || k >= h->n) return fail(LLG_EINVAL, "bad handle or disk index");
    if (D) *D = h->D[k];
    if (P) *P = h->P[k];
    if (n_cells) *n_cells = h->n_cells[k];
    return 0;
}

long long llg_disk_offset(llg_disk h, int k) {
    if (!h || k < 0 || k >= h->n) return fail(LLG_EINVAL, "bad handle or disk index");
    return h->m_off[k];
}

long long llg_state_size(llg_disk h) { return h ? h->state_size : fail(LLG_EINVAL, "null handle"); }

int llg_disk_workgroups(llg_disk h, int k) {
    if (!h || k < 0 || k >= h->n) return fail(LLG_EINVAL, "bad handle or disk index");
    return h->G[k];
}

int llg_tune(llg_disk h, int unit_groups, int radix_policy, const int* wg_per_disk) {
    int rc = check_handle(h);
    if (rc) return rc;
    HIP_TRY(hipDeviceSynchronize());
    return plan(h, unit_groups, radix_policy, wg_per_disk);
}

int llg_set_on_chip(llg_disk h, int max_P) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (max_P != 0 && max_P != 64 && max_P != 128) return fail(LLG_EINVAL, "max_P must be 0, 64 or 128");
    HIP_TRY(hipDeviceSynchronize());
    const int old = h->onchip_pmax;
    h->onchip_pmax = max_P;
    if ((rc = plan(h, h->UG, h->RSEL, nullptr))) {
        h->onchip_pmax = old;   // the previous plan stays in force
        return rc;
    }
    return 0;
}

int llg_get_on_chip(llg_disk h) { return h ? h->onchip_pmax : fail(LLG_EINVAL, "null handle"); }

int llg_timing(llg_disk h, int enable) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (enable && !h->time_ev[0][0])
        for (auto& pair : h->time_ev)
            for (hipEvent_t& e : pair) HIP_TRY(hipEventCreate(&e));
    h->timing = enable != 0;
    for (bool& v : h->time_valid) v = false;
    return 0;
}

int llg_last_launch_ms(llg_disk h, int mode, float* ms) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!ms) return fail(LLG_EINVAL, "null output");
    if (mode < 0 || mode >= llg_disk_s::N_MODES) return fail(LLG_EINVAL, "mode out of range");
    if (!h->time_valid[mode]) return fail(LLG_EINVAL, "no launch of this mode timed since timing was enabled");
    HIP_TRY(hipEventSynchronize(h->time_ev[mode][1]));
    HIP_TRY(hipEventElapsedTime(ms, h->time_ev[mode][0], h->time_ev[mode][1]));
    return 0;
}

int llg_debug_spin_limit(llg_disk h, unsigned int polls) {
    if (!h) return fail(LLG_EINVAL, "null handle");
    h->spin_limit = polls ? polls : SPIN_LIMIT;
    return 0;
}

int llg_launch_shape(llg_disk h, int* unit_groups, int* workgroups, int* threads, int* radix_policy) {
    if (!h) return fail(LLG_EINVAL, "null handle");
    if (radix_policy) *radix_policy = h->RSEL;
    if (unit_groups) *unit_groups = h->UG;
    if (workgroups) *workgroups = h->n_wg;
    if (threads) *threads = WG_THREADS * h->UG;
    return 0;
}

int llg_autotune(llg_disk h, const float* m, const llg_params* p, int integrator, long long probe_steps,
                 void* stream, double* best_us) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !p) return fail(LLG_EINVAL, "null array");
    if (integrator != 0 && integrator != 1) return fail(LLG_EINVAL, "integrator: 0 = RK4, 1 = Heun");
    if (probe_steps < 1) return fail(LLG_EINVAL, "probe_steps < 1");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(st));
    // probe buffer and timing events, released on every return path
    struct Probe {
        float* work = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Probe() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (work) (void)hipFree(work);
        }
    } pr;
    HIP_TRY(hipMalloc(&pr.work, h->state_size * sizeof(float)));
    HIP_TRY(hipEventCreate(&pr.e0));
    HIP_TRY(hipEventCreate(&pr.e1));
    float* work = pr.work;
    hipEvent_t e0 = pr.e0, e1 = pr.e1;
    const int mode = integrator == 0 ? MODE_RK4 : MODE_HEUN;
    llg_params* pp = const_cast<llg_params*>(p);
    if ((rc = upload_params(h, pp, st))) return rc;
    // candidate plans: unit groups x transform policy x workgroup scale x spectra
    // on chip (off, and for P <= 64 / P <= 128 where the handle has such disks)
    const int pmin = *std::min_element(h->P.begin(), h->P.end());
    std::vector<int> ocs = {0};
    if (pmin <= 64) ocs.push_back(64);
    if (pmin <= 128 && std::count_if(h->P.begin(), h->P.end(), [](int P) { return P == 128; }) > 0) ocs.push_back(128);
    struct Cand { int UG, RSEL; double scale; int oc; };
    std::vector<Cand> cands;
    for (int ug : {1, 2, 4})
        for (int rs : {0, 1, 2, 3})
            for (double sc : {1.0, 0.5, 0.25}) cands.push_back({ug, rs, sc, 0});
    for (size_t q = 1; q < ocs.size(); ++q)   // on chip: one unit group, the full workgroup budget
        for (int rs : {0, 1, 2, 3}) cands.push_back({1, rs, 1.0, ocs[q]});
    double best = 1e300;
    Cand bestc{h->UG, h->RSEL, 1.0, h->onchip_pmax};
    for (const Cand& c : cands) {
        // the tuned plan must keep the integrator and the field kernel (observables) co-resident
        const unsigned modes = (1u << mode) | (1u << MODE_DEMAG);
        h->onchip_pmax = c.oc;
        if ((rc = plan(h, c.UG, c.RSEL, nullptr, modes, c.scale))) continue;
        float ms = 0.f;
        bool ok = true;
        for (int rep = 0; rep < 2 && ok; ++rep) {
            HIP_TRY(hipMemcpyAsync(work, m, h->state_size * sizeof(float), hipMemcpyDeviceToDevice, st));
            HIP_TRY(hipEventRecord(e0, st));
            if (launch(h, mode, work, nullptr, probe_steps, 1, 0, 0, st)) ok = false;
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        }
        int e = 0;
        HIP_TRY(hipMemcpy(&e, h->err_dev, sizeof(int), hipMemcpyDeviceToHost));
        if (e) {
            HIP_TRY(hipMemset(h->err_dev, 0, sizeof(int)));
            ok = false;
        }
        if (ok && ms > 0 && ms < best) {
            best = ms;
            bestc = c;
        }
    }
    h->onchip_pmax = bestc.oc;
    if ((rc = plan(h, bestc.UG, bestc.RSEL, nullptr, (1u << mode) | (1u << MODE_DEMAG), bestc.scale))) return rc;
    if (best_us) *best_us = best * 1e3 / (double)probe_steps;
    return 0;
}

int llg_demag_field(llg_disk h, const float* m, float* H, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !H) return fail(LLG_EINVAL, "null array");
    return launch(h, MODE_DEMAG, const_cast<float*>(m), H, 0, 0, 0, 0, (hipStream_t)stream);
}

int llg_rhs(llg_disk h, const float* m, float* dmdtau, const llg_params* p, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !dmdtau) return fail(LLG_EINVAL, "null array");
    if ((rc = upload_params(h, p, (hipStream_t)stream))) return rc;
    return launch(h, MODE_RHS, const_cast<float*>(m), dmdtau, 0, 0, 0, 0, (hipStream_t)stream);
}

int llg_rk4_step(llg_disk h, float* m, long long nsteps, const llg_params* p, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m) return fail(LLG_EINVAL, "null array");
    if (nsteps < 0) return fail(LLG_EINVAL, "nsteps < 0");
    if (nsteps == 0) return 0;
    if ((rc = upload_params(h, p, (hipStream_t)stream))) return rc;
    return launch(h, MODE_RK4, m, nullptr, nsteps, 0, 0, 0, (hipStream_t)stream);
}

long long llg_noalloc_bytes(llg_disk h) {
    if (!h) return fail(LLG_EINVAL, "null handle");
    unsigned long long b = scratch_head(h->n);
    for (const DiskDesc& d : h->desc) b += scratch_disk_bytes(d.D, d.H, d.Dp, d.G);
    return (long long)b;
}

int llg_rk4_step_noalloc(llg_disk h, float* m, long long nsteps, const llg_params* p, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m) return fail(LLG_EINVAL, "null array");
    if (nsteps < 0) return fail(LLG_EINVAL, "nsteps < 0");
    const long long need = llg_noalloc_bytes(h);
    if (need > (long long)LLG_NOALLOC_BYTES)
        return fail(LLG_EINVAL, "the handle's workspaces need " + std::to_string(need) + " bytes, more than the " +
                                    std::to_string((long long)LLG_NOALLOC_BYTES) +
                                    " bytes of the fixed scratch array; use llg_rk4_step");
    if (nsteps == 0) return 0;
    unsigned char* base = nullptr;
    if ((rc = scratch_ptr(h->device, &base))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = upload_params(h, p, st))) return rc;
    hipLaunchKernelGGL(scratch_descriptors, dim3((h->n + 63) / 64), dim3(64), 0, st, h->desc_dev, h->n, base);
    HIP_TRY(hipGetLastError());
    unsigned int* bars = reinterpret_cast<unsigned int*>(base + align256((unsigned long long)h->n * sizeof(DiskDesc)));
    return launch(h, MODE_RK4, m, nullptr, nsteps, 0, 0, 0, st, nullptr, nullptr, nullptr, 0.0, 0.0, nullptr, 0.0,
                  reinterpret_cast<const DiskDesc*>(base), bars);
}

int llg_rk4_record(llg_disk h, float* m, long long nsteps, const llg_params* p, float* rec, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !rec) return fail(LLG_EINVAL, "null array");
    if (nsteps < 1) return fail(LLG_EINVAL, "nsteps < 1");
    if ((rc = upload_params(h, p, (hipStream_t)stream))) return rc;
    return launch(h, MODE_RK4, m, nullptr, nsteps, 0, 0, 0, (hipStream_t)stream, rec);
}

int llg_rk4_vjp(llg_disk h, const float* rec, long long nsteps, float* ybar, double* pgrad, const llg_params* p,
                void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!rec || !ybar || !pgrad || !p) return fail(LLG_EINVAL, "null argument");
    if (nsteps < 1) return fail(LLG_EINVAL, "nsteps < 1");
    for (int k = 0; k < h->n; ++k)
        if (p[k].renorm) return fail(LLG_EUNSUPPORTED, "the adjoint covers RK4 without renormalisation");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = upload_params(h, p, st))) return rc;
    if ((rc = launch(h, MODE_RK4_VJP, ybar, nullptr, nsteps, 0, 0, 0, st, const_cast<float*>(rec)))) return rc;
    hipLaunchKernelGGL(grad_finalize, dim3((h->n + 63) / 64), dim3(64), 0, st, h->desc_dev, h->n, pgrad);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_heun_record(llg_disk h, float* m, long long nsteps, unsigned long long seed, unsigned long long step0,
                    unsigned int replica, const llg_params* p, float* rec, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !rec) return fail(LLG_EINVAL, "null array");
    if (nsteps < 1) return fail(LLG_EINVAL, "nsteps < 1");
    if (step0 == LLG_STEP_COUNTER) return fail(LLG_EINVAL, "the recorded Heun steps need an explicit step0");
    if ((rc = upload_params(h, p, (hipStream_t)stream))) return rc;
    return launch(h, MODE_HEUN, m, nullptr, nsteps, seed, step0, replica, (hipStream_t)stream, rec);
}

int llg_heun_vjp(llg_disk h, const float* rec, long long nsteps, unsigned long long seed, unsigned long long step0,
                 unsigned int replica, float* ybar, double* pgrad, const llg_params* p, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!rec || !ybar || !pgrad) return fail(LLG_EINVAL, "null array");
    if (nsteps < 1) return fail(LLG_EINVAL, "nsteps < 1");
    if (step0 == LLG_STEP_COUNTER) return fail(LLG_EINVAL, "the Heun adjoint needs an explicit step0");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = upload_params(h, p, st))) return rc;
    if ((rc = launch(h, MODE_HEUN_VJP, ybar, nullptr, nsteps, seed, step0, replica, st, const_cast<float*>(rec))))
        return rc;
    hipLaunchKernelGGL(grad_finalize, dim3((h->n + 63) / 64), dim3(64), 0, st, h->desc_dev, h->n, pgrad);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_core_position_vjp(llg_disk h, const float* m, double lambda_ex_nm, const double* core, const double* rbar,
                          float* mbar, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !core || !rbar || !mbar) return fail(LLG_EINVAL, "null array");
    if (!(lambda_ex_nm > 0)) return fail(LLG_EINVAL, "lambda_ex must be positive");
    hipLaunchKernelGGL(core_vjp_kernel, dim3(h->n), dim3(OBS_THREADS), 0, (hipStream_t)stream, h->desc_dev, m, core,
                       rbar, h->a_nm, 4.0 * lambda_ex_nm / h->a_nm, mbar);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_relax(llg_disk h, float* m, const double* X_nm, double cutoff_nm, double kappa, double tol,
              long long max_sweeps, const llg_params* p, double* out, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !X_nm || !out) return fail(LLG_EINVAL, "null array");
    if (!(kappa > 0) || !(tol > 0) || max_sweeps < 1) return fail(LLG_EINVAL, "need kappa > 0, tol > 0, max_sweeps >= 1");
    if (!(cutoff_nm >= 0)) return fail(LLG_EINVAL, "cutoff must be >= 0 (0 = whole disk)");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = upload_params(h, p, st))) return rc;
    // target positions in units of a from the disk centre, staged like the hints
    HIP_TRY(hipEventSynchronize(h->hint_event));
    for (int k = 0; k < 2 * h->n; ++k) h->hint_pin[k] = X_nm[k] / h->a_nm;
    HIP_TRY(hipMemcpyAsync(h->hint_dev, h->hint_pin, 2 * h->n * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(h->hint_event, st));
    const double rcut = cutoff_nm / h->a_nm;
    return launch(h, MODE_RELAX, m, nullptr, max_sweeps, 0, 0, 0, st, nullptr, h->hint_dev, out, kappa, tol, nullptr,
                  rcut * rcut);
}

int llg_rk4_series(llg_disk h, float* m, long long nsteps, const llg_params* p, long long sample_every,
                   double* series, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !series) return fail(LLG_EINVAL, "null array");
    if (nsteps < 0) return fail(LLG_EINVAL, "nsteps < 0");
    if (sample_every < 1 || sample_every > (1ll << 30)) return fail(LLG_EINVAL, "sample_every must be in [1, 2^30]");
    if (nsteps == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = upload_params(h, p, st))) return rc;
    return launch(h, MODE_RK4, m, nullptr, nsteps, 0, 0, 0, st, nullptr, nullptr, nullptr, 0.0, 0.0, nullptr, 0.0,
                  nullptr, nullptr, series, sample_every);
}

int llg_heun_series(llg_disk h, float* m, long long nsteps, unsigned long long seed, unsigned long long step0,
                    unsigned int replica, const llg_params* p, long long sample_every, double* series,
                    void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !series) return fail(LLG_EINVAL, "null array");
    if (nsteps < 0) return fail(LLG_EINVAL, "nsteps < 0");
    if (sample_every < 1 || sample_every > (1ll << 30)) return fail(LLG_EINVAL, "sample_every must be in [1, 2^30]");
    if (nsteps == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = upload_params(h, p, st))) return rc;
    const bool counter = step0 == LLG_STEP_COUNTER;
    return launch(h, MODE_HEUN, m, nullptr, nsteps, seed, counter ? 0 : step0, replica, st, nullptr, nullptr, nullptr,
                  0.0, 0.0, counter ? h->step_dev : nullptr, 0.0, nullptr, nullptr, series, sample_every);
}

int llg_power_spectrum(const double* x, int n_seq, long long bstride, long long len, long long tstride,
                       int remove_mean, int window, double* work, double* out, void* stream) {
    if (!x || !work || !out) return fail(LLG_EINVAL, "null array");
    if (n_seq < 1 || n_seq > 65535) return fail(LLG_EINVAL, "n_seq must be in [1, 65535]");
    if (len < 16 || len > (1ll << 24) || (len & (len - 1))) return fail(LLG_EINVAL, "len must be a power of two in [16, 2^24]");
    if (tstride < 1 || bstride < 0) return fail(LLG_EINVAL, "need tstride >= 1 and bstride >= 0");
    if (window != 0 && window != 1) return fail(LLG_EINVAL, "window: 0 = none, 1 = Hann");
    hipStream_t st = (hipStream_t)stream;
    double2* A = reinterpret_cast<double2*>(work);
    double2* B = A + (size_t)len * n_seq;
    const int half_blocks = (int)std::min<long long>((len / 2 + 255) / 256, 65535);
    const int full_blocks = (int)std::min<long long>((len + 255) / 256, 65535);
    hipLaunchKernelGGL(ps_mean, dim3(n_seq), dim3(256), 0, st, x, bstride, len, tstride, remove_mean, B);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(ps_load, dim3(full_blocks, n_seq), dim3(256), 0, st, x, bstride, len, tstride, window,
                       (const double2*)B, A);
    HIP_TRY(hipGetLastError());
    double2* in = A;
    double2* outb = B;
    for (long long Ns = 1; Ns < len; Ns *= 2) {
        hipLaunchKernelGGL(ps_pass, dim3(half_blocks, n_seq), dim3(256), 0, st, (const double2*)in, outb, len, Ns);
        HIP_TRY(hipGetLastError());
        std::swap(in, outb);
    }
    hipLaunchKernelGGL(ps_power, dim3(full_blocks, n_seq), dim3(256), 0, st, (const double2*)in, len, out);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_heun_step(llg_disk h, float* m, long long nsteps, unsigned long long seed, unsigned long long step0,
                  unsigned int replica, const llg_params* p, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m) return fail(LLG_EINVAL, "null array");
    if (nsteps < 0) return fail(LLG_EINVAL, "nsteps < 0");
    if (nsteps == 0) return 0;
    if ((rc = upload_params(h, p, (hipStream_t)stream))) return rc;
    if (step0 == LLG_STEP_COUNTER)
        return launch(h, MODE_HEUN, m, nullptr, nsteps, seed, 0, replica, (hipStream_t)stream, nullptr, nullptr,
                      nullptr, 0.0, 0.0, h->step_dev);
    return launch(h, MODE_HEUN, m, nullptr, nsteps, seed, step0, replica, (hipStream_t)stream);
}

int llg_step_counter_set(llg_disk h, unsigned long long step, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    hipLaunchKernelGGL(set_u64, dim3(1), dim3(64), 0, (hipStream_t)stream, h->step_dev, step);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_step_counter_get(llg_disk h, unsigned long long* step, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!step) return fail(LLG_EINVAL, "null output");
    HIP_TRY(hipMemcpyAsync(step, h->step_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    return 0;
}

int llg_graph_create(llg_disk h, int integrator, float* m, long long nsteps, const llg_params* p,
                     unsigned long long seed, unsigned int replica, llg_graph* out) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !p || !out) return fail(LLG_EINVAL, "null argument");
    if (integrator != 0 && integrator != 1) return fail(LLG_EINVAL, "integrator must be 0 (RK4) or 1 (Heun)");
    if (nsteps < 1) return fail(LLG_EINVAL, "nsteps < 1");
    *out = nullptr;
    std::unique_ptr<llg_graph_s> g(new llg_graph_s());
    g->h = h;
    // the graph keeps its own copy of the parameters
    if ((rc = upload_params(h, p, nullptr))) return rc;
    HIP_TRY(hipDeviceSynchronize());
    DiskPrm* gprm = nullptr;
    HIP_TRY(g->dalloc(&gprm, h->n));
    HIP_TRY(hipMemcpy(gprm, h->prm_dev, h->n * sizeof(DiskPrm), hipMemcpyDeviceToDevice));
    // ... and of the current launch plan
    int *gw2d = nullptr, *gw2l = nullptr;
    DiskDesc* gdesc = nullptr;
    HIP_TRY(g->dalloc(&gw2d, h->n_wg));
    HIP_TRY(g->dalloc(&gw2l, h->n_wg));
    HIP_TRY(hipMemcpy(gw2d, h->wg2disk, h->n_wg * sizeof(int), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(gw2l, h->wg2local, h->n_wg * sizeof(int), hipMemcpyDeviceToDevice));
    std::vector<DiskDesc> desc = h->desc;
    for (DiskDesc& d : desc) HIP_TRY(g->dalloc(&d.part, (size_t)PART_STRIDE * d.G));
    HIP_TRY(g->dalloc(&gdesc, h->n));
    HIP_TRY(hipMemcpy(gdesc, desc.data(), h->n * sizeof(DiskDesc), hipMemcpyHostToDevice));
    HIP_TRY(hipGraphCreate(&g->graph, 0));
    // node 1: clear the barrier counters (a kernel, not a memset node)
    int n_bars = h->n_bars;
    unsigned int* bars = h->bars;
    void* zargs[] = {&bars, &n_bars};
    hipKernelNodeParams zp{};
    zp.func = reinterpret_cast<void*>(zero_u32);
    zp.gridDim = dim3((h->n_bars + 255) / 256);
    zp.blockDim = dim3(256);
    zp.kernelParams = zargs;
    hipGraphNode_t nz, np, na;
    HIP_TRY(hipGraphAddKernelNode(&nz, g->graph, nullptr, 0, &zp));
    // node 2: the persistent cooperative launch
    const int mode = integrator == 0 ? MODE_RK4 : MODE_HEUN;
    KArgs a = make_args(h, gprm, mode, m, nullptr, nsteps, seed, 0, replica, integrator == 1 ? h->step_dev : nullptr,
                        nullptr, nullptr, nullptr, 0.0, 0.0);
    a.disks = gdesc;
    a.wg2disk = gw2d;
    a.wg2local = gw2l;
    void* pargs[] = {&a};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(persistent_kernel(mode, h->UG, h->RSEL, h->PMAX));
    kp.gridDim = dim3(h->n_wg);
    kp.blockDim = dim3(WG_THREADS * h->UG);
    kp.sharedMemBytes = h->onchip_lds;   // on-chip spectra of the plan (the descriptors' flags)
    kp.kernelParams = pargs;
    HIP_TRY(hipGraphAddKernelNode(&np, g->graph, &nz, 1, &kp));
    hipKernelNodeAttrValue coop{};
    coop.cooperative = 1;
    HIP_TRY(hipGraphKernelNodeSetAttribute(np, hipKernelNodeAttributeCooperative, &coop));
    // node 3 (Heun): advance the step counter so that the next replay continues the noise stream
    if (integrator == 1) {
        unsigned long long* sp = h->step_dev;
        unsigned long long ns = (unsigned long long)nsteps;
        void* aargs[] = {&sp, &ns};
        hipKernelNodeParams ap{};
        ap.func = reinterpret_cast<void*>(advance_u64);
        ap.gridDim = dim3(1);
        ap.blockDim = dim3(64);
        ap.kernelParams = aargs;
        HIP_TRY(hipGraphAddKernelNode(&na, g->graph, &np, 1, &ap));
    }
    HIP_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    *out = g.release();
    return 0;
}

int llg_graph_launch(llg_graph g, void* stream) {
    if (!g) return fail(LLG_EINVAL, "null graph");
    int rc = check_handle(g->h);
    if (rc) return rc;
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return 0;
}

void llg_graph_destroy(llg_graph g) { delete g; }

int llg_noise(llg_disk h, unsigned long long seed, unsigned long long step, unsigned int replica, float* w,
              void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!w) return fail(LLG_EINVAL, "null array");
    hipLaunchKernelGGL(noise_kernel, dim3(64, h->n), dim3(256), 0, (hipStream_t)stream, h->desc_dev, h->n, w, seed,
                       step, replica);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_energy(llg_disk h, const float* m, const llg_params* p, double* out, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !out) return fail(LLG_EINVAL, "null array");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = upload_params(h, p, st))) return rc;
    if ((rc = launch(h, MODE_ENERGY, const_cast<float*>(m), nullptr, 0, 0, 0, 0, st))) return rc;
    hipLaunchKernelGGL(energy_finalize, dim3((h->n + 63) / 64), dim3(64), 0, st, h->desc_dev, h->n, out);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_vortex_core_position(llg_disk h, const float* m, double lambda_ex_nm, const double* hint_nm, double* out,
                             void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !out) return fail(LLG_EINVAL, "null array");
    if (!(lambda_ex_nm > 0)) return fail(LLG_EINVAL, "lambda_ex must be positive");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipEventSynchronize(h->hint_event));
    for (int k = 0; k < 2 * h->n; ++k) h->hint_pin[k] = hint_nm ? hint_nm[k] : NAN;
    HIP_TRY(hipMemcpyAsync(h->hint_dev, h->hint_pin, 2 * h->n * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(h->hint_event, st));
    hipLaunchKernelGGL(core_scan_kernel, dim3(h->core_strips, h->n), dim3(OBS_THREADS), 0, st, h->desc_dev, m,
                       h->hint_dev, h->a_nm, h->core_strips, h->core_part);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(core_finish_kernel, dim3(h->n), dim3(OBS_THREADS), 0, st, h->desc_dev, m, h->a_nm,
                       4.0 * lambda_ex_nm / h->a_nm, h->core_strips, h->core_part, out);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_mean_m(llg_disk h, const float* m, double* out, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!m || !out) return fail(LLG_EINVAL, "null array");
    hipLaunchKernelGGL(mean_kernel, dim3(h->n), dim3(OBS_THREADS), 0, (hipStream_t)stream, h->desc_dev, m, out);
    HIP_TRY(hipGetLastError());
    return 0;
}

int llg_check(llg_disk h, void* stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int e = 0;
    HIP_TRY(hipMemcpy(&e, h->err_dev, sizeof(int), hipMemcpyDeviceToHost));
    if (e) {
        HIP_TRY(hipMemset(h->err_dev, 0, sizeof(int)));
        std::string msg = "device failure:";
        if (e & ERR_BARRIER) msg += " group barrier timed out;";
        if (e & ERR_NONFINITE) msg += " non-finite state;";
        return fail(LLG_EDEVICE, msg);
    }
    return 0;
}

void llg_destroy(llg_disk h) { delete h; }

const char* llg_last_error(void) { return g_err.c_str(); }

}  // extern "C"
