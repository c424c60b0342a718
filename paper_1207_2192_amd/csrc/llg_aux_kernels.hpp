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

__device__ __forceinline__ double wrap_pi(double x) {
    // x + pi reduced into [0, 2 pi), minus pi
    const double two_pi = 6.283185307179586476925286766559;
    const double pi = 3.1415926535897932384626433832795;
    double t = fmod(x + pi, two_pi);
    if (t < 0.0) t += two_pi;
    return t - pi;
}

// Vortex core position per disk, float64 (one workgroup per disk).
// hint: per disk (x, y) in nm, NaN = no hint.
__global__ __launch_bounds__(OBS_THREADS) void core_kernel(const DiskDesc* disks, const float* m_base,
                                                           const double* hint, double a_nm, double cutoff_cells,
                                                           double* out) {
    __shared__ double sh[OBS_THREADS / 64];
    __shared__ double s_score[OBS_THREADS / 64];
    __shared__ int s_idx[OBS_THREADS / 64];
    const int k = blockIdx.x;
    const DiskDesc d = disks[k];
    const int D = d.D, DD = D * D, Dm = D - 1;
    const float* m = m_base + d.m_off;
    const unsigned char* mask = d.mask;
    const double half = (D - 1) / 2.0;
    const double two_pi = 6.283185307179586476925286766559;
    const double hx = hint[2 * k], hy = hint[2 * k + 1];
    const bool use_hint = !(isnan(hx) || isnan(hy));

    double best = -INFINITY;
    int best_idx = 0x7fffffff;
    int nplus = 0;
    for (int p = threadIdx.x; p < Dm * Dm; p += OBS_THREADS) {
        const int j = p / Dm, i = p - j * Dm;
        const int ca = j * D + i, cb = ca + 1, cc = ca + D + 1, cd = ca + D;
        if (!(mask[ca] && mask[cb] && mask[cc] && mask[cd])) continue;
        const double fa = atan2((double)m[DD + ca], (double)m[ca]);
        const double fb = atan2((double)m[DD + cb], (double)m[cb]);
        const double fc = atan2((double)m[DD + cc], (double)m[cc]);
        const double fd = atan2((double)m[DD + cd], (double)m[cd]);
        const double s = wrap_pi(fb - fa) + wrap_pi(fc - fb) + wrap_pi(fd - fc) + wrap_pi(fa - fd);
        if ((int)rint(s / two_pi) != 1) continue;
        ++nplus;
        double score;
        const double cx = ((double)i - half) + 0.5, cy = ((double)j - half) + 0.5;
        if (use_hint) {
            const double ddx = cx - hx / a_nm, ddy = cy - hy / a_nm;
            score = -(ddx * ddx + ddy * ddy);
        } else {
            const double za = m[2 * DD + ca], zb = m[2 * DD + cb], zc = m[2 * DD + cc], zd = m[2 * DD + cd];
            score = za * za + zb * zb + zc * zc + zd * zd;
        }
        if (score > best || (score == best && p < best_idx)) {
            best = score;
            best_idx = p;
        }
    }
    // argmax (higher score, then lower index) over the workgroup
    for (int o = 32; o > 0; o >>= 1) {
        const double os = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(best_idx, o, 64);
        if (os > best || (os == best && oi < best_idx)) {
            best = os;
            best_idx = oi;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_score[wave] = best;
        s_idx[wave] = best_idx;
    }
    const double np = block_sum((double)nplus, sh);
    double bs = s_score[0];
    int bi = s_idx[0];
    for (int w = 1; w < OBS_THREADS / 64; ++w)
        if (s_score[w] > bs || (s_score[w] == bs && s_idx[w] < bi)) {
            bs = s_score[w];
            bi = s_idx[w];
        }
    const bool found = np > 0.5;
    double xv = NAN, yv = NAN;
    if (found) {
        const int j = bi / Dm, i = bi - j * Dm;
        xv = ((double)i - half) + 0.5;
        yv = ((double)j - half) + 0.5;
    }
    const double c2 = cutoff_cells * cutoff_cells;
    double sw = 0.0, swx = 0.0, swy = 0.0;
    for (int c = threadIdx.x; c < DD; c += OBS_THREADS) {
        if (!mask[c]) continue;
        const int j = c / D, i = c - j * D;
        const double x = (double)i - half, y = (double)j - half;
        if (found) {
            const double ddx = x - xv, ddy = y - yv;
            if (!(ddx * ddx + ddy * ddy < c2)) continue;
        }
        const double z = m[2 * DD + c];
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
        out[5 * k + 4] = np;
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
