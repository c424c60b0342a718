// Small kernels of lib_llgdisk: barrier reset, per-disk float64 reductions
// (energy, adjoint parameter gradients, <m>, vortex core position and its
// cotangent) and the noise test hook.
#pragma once
#include "llg_device.hpp"

namespace llg {

__global__ void zero_u32(unsigned int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// The handle's Heun step counter: set, and advance after a launch that used it.
__global__ void set_u64(unsigned long long* p, unsigned long long v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}
__global__ void advance_u64(unsigned long long* p, unsigned long long n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p += n;
}

// E = E_ex + E_demag + E_ext per disk from the per-workgroup partials, summed in
// workgroup order (deterministic).
__global__ void energy_finalize(const DiskDesc* disks, int n, double* out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const DiskDesc d = disks[k];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int g = 0; g < d.G; ++g) {
        s0 += d.part[g * PART_STRIDE + 0];
        s1 += d.part[g * PART_STRIDE + 1];
        s2 += d.part[g * PART_STRIDE + 2];
    }
    out[4 * k + 0] = s0 + s1 + s2;
    out[4 * k + 1] = s0;
    out[4 * k + 2] = s1;
    out[4 * k + 3] = s2;
}

// Adjoint parameter gradients: pgrad[2k] += alpha_bar, pgrad[2k+1] += c_bar of disk k,
// summed over the per-workgroup partials in workgroup order.
__global__ void grad_finalize(const DiskDesc* disks, int n, double* pgrad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const DiskDesc d = disks[k];
    double s0 = 0.0, s1 = 0.0;
    for (int g = 0; g < d.G; ++g) {
        s0 += d.part[g * PART_STRIDE + 0];
        s1 += d.part[g * PART_STRIDE + 1];
    }
    pgrad[2 * k] += s0;
    pgrad[2 * k + 1] += s1;
}

// Noise field of one Heun step (test hook), packed like the state.
__global__ void noise_kernel(const DiskDesc* disks, int n, float* w, unsigned long long seed,
                             unsigned long long step, unsigned int replica0) {
    const int k = blockIdx.y;
    if (k >= n) return;
    const DiskDesc d = disks[k];
    const int DD = d.D * d.D;
    float* out = w + d.m_off;
    for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < DD; cell += gridDim.x * blockDim.x) {
        float3 v = make_float3(0.f, 0.f, 0.f);
        if (d.mask[cell]) {
            const int j = cell / d.D, i = cell - j * d.D;
            float3 ev, od;
            thermal_normals_pair(seed, step, (unsigned long long)((j >> 1) * d.D + i),
                                 (unsigned long long)(replica0 + d.k), ev, od);
            v = (j & 1) ? od : ev;
        }
        out[cell] = v.x;
        out[DD + cell] = v.y;
        out[2 * DD + cell] = v.z;
    }
}

constexpr int OBS_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < OBS_THREADS / 64; ++w) s += sh[w];
    return s;
}

// <m> per disk, float64.
__global__ __launch_bounds__(OBS_THREADS) void mean_kernel(const DiskDesc* disks, const float* m_base, double* out) {
    __shared__ double sh[OBS_THREADS / 64];
    const DiskDesc d = disks[blockIdx.x];
    const int DD = d.D * d.D;
    const float* m = m_base + d.m_off;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int c = threadIdx.x; c < DD; c += OBS_THREADS)
        if (d.mask[c]) {
            sx += m[c];
            sy += m[DD + c];
            sz += m[2 * DD + c];
        }
    sx = block_sum(sx, sh);
    sy = block_sum(sy, sh);
    sz = block_sum(sz, sh);
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x + 0] = sx / d.n_cells;
        out[3 * blockIdx.x + 1] = sy / d.n_cells;
        out[3 * blockIdx.x + 2] = sz / d.n_cells;
    }
}

// Vortex core position (Sec. IV) in two kernels.
//
// core_scan_kernel: block (s, k) scans the plaquette rows [CORE_ROWS s,
// CORE_ROWS (s + 1)) of disk k.  A plaquette counts when its four cells belong
// to the disk; its winding is the sum of the four counter-clockwise angle
// differences, each wrapped into [-pi, pi), over 2 pi, rounded.  The angles are
// taken in float32 first; only when a raw difference lies within
// CORE_WRAP_MARGIN of +-pi (where float32 rounding could flip the wrap) is the
// plaquette recomputed with float64 angles, so every decision equals the
// float64 one.  The block writes its count of +1 plaquettes and its best
// candidate (score: closeness to the hint, else the sum of m_z^2 over the
// corners; ties to the lower plaquette index) to part[k][s].
// core_finish_kernel: one block per disk picks r_v from the strips (same
// order), then forms the m_z^2-weighted centroid over the disk cells within
// the cutoff of r_v (scanning only the cutoff's bounding box) or, without a
// +1 plaquette, over the whole disk.  float64 throughout the reductions.
constexpr int CORE_ROWS = 8;
constexpr float CORE_WRAP_MARGIN = 1e-3f;

struct CorePart {
    double score;
    int count, idx;
};

__device__ __forceinline__ double wrap_pi(double x) {
    // x + pi reduced into [0, 2 pi), minus pi
    const double two_pi = 6.283185307179586476925286766559;
    const double pi = 3.1415926535897932384626433832795;
    double t = fmod(x + pi, two_pi);
    if (t < 0.0) t += two_pi;
    return t - pi;
}

// Winding of the plaquette with corners a, b, c, d (counter-clockwise).
__device__ __forceinline__ int plaquette_winding(const float* mx, const float* my, int ca, int cb, int cc, int cd) {
    const float pi_f = 3.14159265358979f;
    const float fa = atan2f(my[ca], mx[ca]), fb = atan2f(my[cb], mx[cb]);
    const float fc = atan2f(my[cc], mx[cc]), fd = atan2f(my[cd], mx[cd]);
    const float r0 = fb - fa, r1 = fc - fb, r2 = fd - fc, r3 = fa - fd;
    const float lo = pi_f - CORE_WRAP_MARGIN, hi = pi_f + CORE_WRAP_MARGIN;
    auto near_pi = [&](float r) {
        const float q = fabsf(r);
        return q > lo && q < hi;
    };
    if (!(near_pi(r0) || near_pi(r1) || near_pi(r2) || near_pi(r3))) {
        auto wrap = [&](float r) { return r >= pi_f ? r - 2.f * pi_f : (r < -pi_f ? r + 2.f * pi_f : r); };
        const float s = wrap(r0) + wrap(r1) + wrap(r2) + wrap(r3);
        return (int)rintf(s * 0.15915494309189535f);
    }
    const double two_pi = 6.283185307179586476925286766559;
    const double ga = atan2((double)my[ca], (double)mx[ca]), gb = atan2((double)my[cb], (double)mx[cb]);
    const double gc = atan2((double)my[cc], (double)mx[cc]), gd = atan2((double)my[cd], (double)mx[cd]);
    const double s = wrap_pi(gb - ga) + wrap_pi(gc - gb) + wrap_pi(gd - gc) + wrap_pi(ga - gd);
    return (int)rint(s / two_pi);
}

__device__ __forceinline__ bool core_better(double s, int i, double bs, int bi) {
    return s > bs || (s == bs && i < bi);
}

// hint: per disk (x, y) in nm, NaN = no hint.
__global__ __launch_bounds__(OBS_THREADS) void core_scan_kernel(const DiskDesc* disks, const float* m_base,
                                                                const double* hint, double a_nm, int n_strips,
                                                                CorePart* part) {
    __shared__ double s_score[OBS_THREADS / 64];
    __shared__ int s_idx[OBS_THREADS / 64], s_cnt[OBS_THREADS / 64];
    const int k = blockIdx.y, strip = blockIdx.x;
    const DiskDesc d = disks[k];
    const int D = d.D, DD = D * D, Dm = D - 1;
    const float* m = m_base + d.m_off;
    const double half = (D - 1) / 2.0;
    const double hx = hint[2 * k], hy = hint[2 * k + 1];
    const bool use_hint = !(isnan(hx) || isnan(hy));
    const int j0 = strip * CORE_ROWS, j1 = min(j0 + CORE_ROWS, Dm);
    double best = -INFINITY;
    int best_idx = 0x7fffffff, nplus = 0;
    const int nrow = j1 > j0 ? j1 - j0 : 0;
    for (int q = threadIdx.x; q < nrow * Dm; q += OBS_THREADS) {
        const int j = j0 + q / Dm, i = q % Dm;
        const int x0 = 2 * i - (D - 1), y0 = 2 * j - (D - 1);   // doubled centre coordinates of cell (j, i)
        const int x1 = x0 + 2, y1 = y0 + 2, DD2 = D * D;
        // the four corners belong to the disk (cell centre inside or on the circle)
        if (!(x0 * x0 + y0 * y0 <= DD2 && x1 * x1 + y0 * y0 <= DD2 && x1 * x1 + y1 * y1 <= DD2 &&
              x0 * x0 + y1 * y1 <= DD2))
            continue;
        const int ca = j * D + i, cb = ca + 1, cc = ca + D + 1, cd = ca + D;
        if (plaquette_winding(m, m + DD, ca, cb, cc, cd) != 1) continue;
        ++nplus;
        const int p = j * Dm + i;
        double score;
        if (use_hint) {
            const double ddx = ((double)i - half) + 0.5 - hx / a_nm, ddy = ((double)j - half) + 0.5 - hy / a_nm;
            score = -(ddx * ddx + ddy * ddy);
        } else {
            const double za = m[2 * DD + ca], zb = m[2 * DD + cb], zc = m[2 * DD + cc], zd = m[2 * DD + cd];
            score = za * za + zb * zb + zc * zc + zd * zd;
        }
        if (core_better(score, p, best, best_idx)) {
            best = score;
            best_idx = p;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double os = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(best_idx, o, 64);
        nplus += __shfl_xor(nplus, o, 64);
        if (core_better(os, oi, best, best_idx)) {
            best = os;
            best_idx = oi;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_score[wave] = best;
        s_idx[wave] = best_idx;
        s_cnt[wave] = nplus;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bs = s_score[0];
        int bi = s_idx[0], cnt = s_cnt[0];
        for (int w = 1; w < OBS_THREADS / 64; ++w) {
            cnt += s_cnt[w];
            if (core_better(s_score[w], s_idx[w], bs, bi)) {
                bs = s_score[w];
                bi = s_idx[w];
            }
        }
        part[k * n_strips + strip] = CorePart{bs, cnt, bi};
    }
}

__global__ __launch_bounds__(OBS_THREADS) void core_finish_kernel(const DiskDesc* disks, const float* m_base,
                                                                  double a_nm, double cutoff_cells, int n_strips,
                                                                  const CorePart* part, double* out) {
    __shared__ double sh[OBS_THREADS / 64];
    __shared__ double s_xv, s_yv;
    __shared__ int s_found;
    const int k = blockIdx.x;
    const DiskDesc d = disks[k];
    const int D = d.D, DD = D * D, Dm = D - 1;
    const float* m = m_base + d.m_off;
    const double half = (D - 1) / 2.0;
    if (threadIdx.x == 0) {
        double bs = -INFINITY;
        int bi = 0x7fffffff, np = 0;
        const int ns = (Dm + CORE_ROWS - 1) / CORE_ROWS;
        for (int s = 0; s < ns; ++s) {
            const CorePart c = part[k * n_strips + s];
            np += c.count;
            if (c.count > 0 && core_better(c.score, c.idx, bs, bi)) {
                bs = c.score;
                bi = c.idx;
            }
        }
        s_found = np;
        s_xv = NAN;
        s_yv = NAN;
        if (np > 0) {
            const int j = bi / Dm, i = bi - j * Dm;
            s_xv = ((double)i - half) + 0.5;
            s_yv = ((double)j - half) + 0.5;
        }
    }
    __syncthreads();
    const bool found = s_found > 0;
    const double xv = s_xv, yv = s_yv;
    const double c2 = cutoff_cells * cutoff_cells;
    // cells to visit: the cutoff circle's bounding box, or the whole box
    int i0 = 0, i1 = D - 1, j0 = 0, j1 = D - 1;
    if (found) {
        i0 = max(0, (int)floor(xv + half - cutoff_cells) - 1);
        i1 = min(D - 1, (int)ceil(xv + half + cutoff_cells) + 1);
        j0 = max(0, (int)floor(yv + half - cutoff_cells) - 1);
        j1 = min(D - 1, (int)ceil(yv + half + cutoff_cells) + 1);
    }
    const int wdt = i1 - i0 + 1, hgt = j1 - j0 + 1;
    double sw = 0.0, swx = 0.0, swy = 0.0;
    for (int q = threadIdx.x; q < wdt * hgt; q += OBS_THREADS) {
        const int j = j0 + q / wdt, i = i0 + q % wdt;
        const int xx = 2 * i - (D - 1), yy = 2 * j - (D - 1);
        if (xx * xx + yy * yy > D * D) continue;
        const double x = (double)i - half, y = (double)j - half;
        if (found) {
            const double ddx = x - xv, ddy = y - yv;
            if (!(ddx * ddx + ddy * ddy < c2)) continue;
        }
        const double z = m[2 * DD + j * D + i];
        const double w = z * z;
        sw += w;
        swx += w * x;
        swy += w * y;
    }
    sw = block_sum(sw, sh);
    swx = block_sum(swx, sh);
    swy = block_sum(swy, sh);
    if (threadIdx.x == 0) {
        out[5 * k + 0] = swx / sw * a_nm;
        out[5 * k + 1] = swy / sw * a_nm;
        out[5 * k + 2] = xv * a_nm;
        out[5 * k + 3] = yv * a_nm;
        out[5 * k + 4] = (double)s_found;
    }
}

// Cotangent of the core position r_c (Sec. IV) with the plaquette r_v and the
// cutoff set frozen at the values of `core` (the output of core_kernel for the
// same state): r_c = sum w_i r_i / W, w_i = m_z,i^2, so
// dL/dm_z,i += 2 m_z,i (rbar . (r_i - r_c)) / W for cells of the set.
// mbar is accumulated (packed like the state); positions in nm.
__global__ __launch_bounds__(OBS_THREADS) void core_vjp_kernel(const DiskDesc* disks, const float* m_base,
                                                               const double* core, const double* rbar, double a_nm,
                                                               double cutoff_cells, float* mbar_base) {
    __shared__ double sh[OBS_THREADS / 64];
    const int k = blockIdx.x;
    const DiskDesc d = disks[k];
    const int D = d.D, DD = D * D;
    const float* m = m_base + d.m_off;
    float* mbar = mbar_base + d.m_off;
    const double half = (D - 1) / 2.0;
    const bool found = core[5 * k + 4] > 0.5;
    const double xv = core[5 * k + 2] / a_nm, yv = core[5 * k + 3] / a_nm;
    const double xc = core[5 * k + 0], yc = core[5 * k + 1];
    const double rx = rbar[2 * k], ry = rbar[2 * k + 1];
    const double c2 = cutoff_cells * cutoff_cells;
    auto in_set = [&](int c, double& x, double& y) {
        if (!d.mask[c]) return false;
        const int j = c / D, i = c - j * D;
        x = (double)i - half;
        y = (double)j - half;
        if (!found) return true;
        const double ddx = x - xv, ddy = y - yv;
        return ddx * ddx + ddy * ddy < c2;
    };
    double W = 0.0;
    for (int c = threadIdx.x; c < DD; c += OBS_THREADS) {
        double x, y;
        if (!in_set(c, x, y)) continue;
        const double z = m[2 * DD + c];
        W += z * z;
    }
    W = block_sum(W, sh);
    for (int c = threadIdx.x; c < DD; c += OBS_THREADS) {
        double x, y;
        if (!in_set(c, x, y)) continue;
        const double z = m[2 * DD + c];
        const double g = 2.0 * z * (rx * (x * a_nm - xc) + ry * (y * a_nm - yc)) / W;
        mbar[2 * DD + c] += (float)g;
    }
}

// ---------------------------------------------------------------- power spectra
// Periodogram of real float64 sequences: mean, window, radix-2 Stockham passes
// in float64 through global memory (one launch per pass), |X_k|^2 / len.
// Sequence b is x[b * bstride + t * tstride]; block y = sequence.

// Mean of each sequence (or 0) into slot [b * len].x of buffer M.
__global__ __launch_bounds__(256) void ps_mean(const double* x, long long bstride, long long len,
                                               long long tstride, int remove_mean, double2* M) {
    __shared__ double sh[4];
    const int b = blockIdx.x;
    const double* xb = x + (long long)b * bstride;
    double s = 0.0;
    if (remove_mean)
        for (long long t = threadIdx.x; t < len; t += 256) s += xb[t * tstride];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) M[(long long)b * len] = make_double2((sh[0] + sh[1] + sh[2] + sh[3]) / (double)len, 0.0);
}

// A[b][t] = w[t] (x_b[t] - mean_b) as complex numbers; w = 1 or the Hann window sin^2(pi t / len).
__global__ __launch_bounds__(256) void ps_load(const double* x, long long bstride, long long len, long long tstride,
                                               int window, const double2* M, double2* A) {
    const int b = blockIdx.y;
    const double mean = M[(long long)b * len].x;
    const double* xb = x + (long long)b * bstride;
    for (long long t = blockIdx.x * 256ll + threadIdx.x; t < len; t += (long long)gridDim.x * 256) {
        double v = xb[t * tstride] - mean;
        if (window == 1) {
            const double sn = sinpi((double)t / (double)len);
            v *= sn * sn;
        }
        A[(long long)b * len + t] = make_double2(v, 0.0);
    }
}

// One radix-2 Stockham pass (sub-transforms of length Ns -> 2 Ns): for
// t < len/2, a = in[t], c = in[t + len/2] W^kk with kk = t mod Ns and
// W = exp(-i pi / Ns); out[2 (t - kk) + kk] = a + c, out[2 (t - kk) + kk + Ns] = a - c.
__global__ __launch_bounds__(256) void ps_pass(const double2* in, double2* out, long long len, long long Ns) {
    const int b = blockIdx.y;
    const double2* ib = in + (long long)b * len;
    double2* ob = out + (long long)b * len;
    const long long half = len / 2;
    for (long long t = blockIdx.x * 256ll + threadIdx.x; t < half; t += (long long)gridDim.x * 256) {
        const long long kk = t & (Ns - 1);
        const double2 a = ib[t], c0 = ib[t + half];
        double sw, cw;
        sincospi(-(double)kk / (double)Ns, &sw, &cw);
        const double2 c = make_double2(c0.x * cw - c0.y * sw, c0.x * sw + c0.y * cw);
        const long long base = 2 * (t - kk) + kk;
        ob[base] = make_double2(a.x + c.x, a.y + c.y);
        ob[base + Ns] = make_double2(a.x - c.x, a.y - c.y);
    }
}

// out[b * (len/2 + 1) + k] = |X_b[k]|^2 / len, k = 0 .. len/2.
__global__ __launch_bounds__(256) void ps_power(const double2* X, long long len, double* out) {
    const int b = blockIdx.y;
    const long long nk = len / 2 + 1;
    for (long long k = blockIdx.x * 256ll + threadIdx.x; k < nk; k += (long long)gridDim.x * 256) {
        const double2 v = X[(long long)b * len + k];
        out[(long long)b * nk + k] = (v.x * v.x + v.y * v.y) / (double)len;
    }
}

}  // namespace llg
