// Stockham radix-R FFT of length P held in LDS, one transform per group of
// P/R lanes of one wavefront.  A transform never leaves its wavefront, and the
// LDS operations of a wavefront are performed in issue order, so the stages
// are separated by wavefront-scope fences (ordering for the compiler, no
// instruction); only the end of a transform is a workgroup barrier, because
// the callers then read the results across wavefronts.
//
// Forward: X[k] = sum_n x[n] exp(-2 pi i n k / P); inverse uses +i and is not
// normalised.  Twiddles come from a table W[e] = exp(-2 pi i e / P) computed in
// float64 on the host and rounded to float32.
#pragma once
#include <hip/hip_runtime.h>

namespace llg {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 d) {
    return INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
    float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
    float2 a2 = cadd(x1, x3), a3 = rot90<INV>(csub(x1, x3));
    x0 = cadd(a0, a2);
    x2 = csub(a0, a2);
    x1 = cadd(a1, a3);
    x3 = csub(a1, a3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* x) {
    // even/odd split into two 4-point transforms, combined with W8^k
    float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    const float r = 0.70710678118654752440f;
    // o1 *= W8^1, o2 *= W8^2, o3 *= W8^3 (conjugates for the inverse)
    float2 t1 = INV ? make_float2(r * (o1.x - o1.y), r * (o1.x + o1.y))
                    : make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));
    float2 t2 = rot90<INV>(o2);
    float2 t3 = INV ? make_float2(-r * (o3.x + o3.y), r * (o3.x - o3.y))
                    : make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));
    x[0] = cadd(e0, o0);
    x[4] = csub(e0, o0);
    x[1] = cadd(e1, t1);
    x[5] = csub(e1, t1);
    x[2] = cadd(e2, t2);
    x[6] = csub(e2, t2);
    x[3] = cadd(e3, t3);
    x[7] = csub(e3, t3);
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* x) {
    if constexpr (R == 2) {
        dft2<INV>(x[0], x[1]);
    } else if constexpr (R == 4) {
        dft4<INV>(x[0], x[1], x[2], x[3]);
    } else {
        static_assert(R == 8, "radix 2, 4 or 8");
        dft8<INV>(x);
    }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Order this lane's LDS accesses against those of the other lanes of its wavefront.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Powers w^1 .. w^(R-1) of one table twiddle by products of powers (at most
// three roundings deep for R = 8), so that a stage reads one twiddle from LDS
// instead of R-1.
template <int R>
__device__ __forceinline__ void twiddle_powers(float2 w1, float2 (&w)[R]) {
    w[1] = w1;
    if constexpr (R >= 4) {
        w[2] = cmul(w1, w1);
        w[3] = cmul(w1, w[2]);
    }
    if constexpr (R == 8) {
        w[4] = cmul(w[2], w[2]);
        w[5] = cmul(w1, w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
    }
}

// LDS layout of a transform buffer: one padding slot after every 8 complex
// values, so that the strided Stockham writes of every stage (lane strides of
// 8, 8 R and 1 elements) and the lane-consecutive reads of a 16-lane group land
// in 16 different bank pairs.
__device__ __forceinline__ int padb(int e) { return e + (e >> 3); }
template <int P>
constexpr int padded_len() { return P + P / 8; }

// One length-P transform by the lanes t = 0 .. P/R-1 of a lane group.
// On entry v[j] = x[t + j*(P/R)].  On exit buf holds X in natural order
// (element e at buf[padb(e)]).  buf may alias the input storage; tw is the P-entry twiddle table.
// buf is touched only by the lanes of this transform until the closing
// workgroup barrier, so every lane of the workgroup must call this the same
// number of times.
// With KEEP (only when P is a power of R) the last stage is not written back:
// v[j] then holds X[t + j*(P/R)] and no closing barrier is issued.  Without
// WGSYNC the buffer is private to the calling wavefront, and the closing
// barrier is a wavefront-scope fence.
template <int P, int R>
constexpr bool fft_whole_radix() {
    return (1 << ((ilog2(P) / ilog2(R)) * ilog2(R))) == P;
}

// Twiddle powers of the full radix-R stages 1 .. NFULL-1 of one lane: they
// depend only on the lane's position t in its transform, so a lane that runs
// many transforms computes them once (w[s-1][j-1] = w_s^j).
template <int P, int R>
struct StageTwiddles {
    static constexpr int NFULL = ilog2(P) / ilog2(R);
    float2 w[NFULL > 1 ? NFULL - 1 : 1][R - 1];
};
template <int P, int R>
__device__ __forceinline__ void stage_twiddles(StageTwiddles<P, R>& st, const float2* tw, int t) {
    int Ns = R;
#pragma unroll
    for (int s = 1; s < StageTwiddles<P, R>::NFULL; ++s) {
        float2 w[R];
        twiddle_powers<R>(tw[(t & (Ns - 1)) * (P / (Ns * R))], w);
#pragma unroll
        for (int j = 1; j < R; ++j) st.w[s - 1][j - 1] = w[j];
        Ns *= R;
    }
}

// ZHI: the inputs v[j], j >= R/2 (points at or past P/2) are known to be zero.
// ZHO: only the outputs below P/2 are needed; the last stage neither computes
// nor writes the others (buf keeps stale values there).
// st: precomputed stage twiddles of this lane (or null: computed per stage).
template <int P, int R, bool INV, bool KEEP = false, bool WGSYNC = true, bool ZHI = false, bool ZHO = false>
__device__ __forceinline__ void fft_run(float2 (&v)[R], float2* buf, const float2* tw, int t,
                                        const StageTwiddles<P, R>* st = nullptr) {
    constexpr int Tf = P / R;
    constexpr int LOGR = ilog2(R);
    constexpr int LOGP = ilog2(P);
    constexpr int NFULL = LOGP / LOGR;
    constexpr int REM = 1 << (LOGP - NFULL * LOGR);
    static_assert(!KEEP || REM == 1, "KEEP needs P = R^k");
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < NFULL; ++s) {
        if (s > 0) {
#pragma unroll
            for (int j = 0; j < R; ++j) v[j] = buf[padb(t + j * Tf)];
            float2 w[R];
            if (st) {
#pragma unroll
                for (int j = 1; j < R; ++j) w[j] = st->w[s - 1][j - 1];
            } else {
                const int kk = t & (Ns - 1);
                twiddle_powers<R>(tw[kk * (P / (Ns * R))], w);
            }
#pragma unroll
            for (int j = 1; j < R; ++j) v[j] = INV ? cmulc(v[j], w[j]) : cmul(v[j], w[j]);
        } else if constexpr (ZHI) {
#pragma unroll
            for (int j = R / 2; j < R; ++j) v[j] = make_float2(0.f, 0.f);
        }
        dftR<R, INV>(v);
        if (KEEP && s == NFULL - 1) break;
        const int kk = t & (Ns - 1);
        const int base = (t - kk) * R + kk;
        // in the last stage base = t and output j lands at t + j P/R
        constexpr int NW = (ZHO && REM == 1) ? R / 2 : R;
        wave_sync();
#pragma unroll
        for (int j = 0; j < (s == NFULL - 1 ? NW : R); ++j) buf[padb(base + j * Ns)] = v[j];
        if (WGSYNC && REM == 1 && s == NFULL - 1)
            __syncthreads();
        else
            wave_sync();
        Ns *= R;
    }
    if constexpr (REM > 1) {
        constexpr int NB = R / REM;
        float2 u[R];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int k = t + q * Tf;
            const int kk = k & (Ns - 1);
            float2 w[REM];
            twiddle_powers<REM>(tw[kk * (P / (Ns * REM))], w);
#pragma unroll
            for (int j = 0; j < REM; ++j) {
                float2 x = buf[padb(k + j * (P / REM))];
                if (j > 0) x = INV ? cmulc(x, w[j]) : cmul(x, w[j]);
                u[q * REM + j] = x;
            }
            dftR<REM, INV>(u + q * REM);
        }
        wave_sync();
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int k = t + q * Tf;
            const int kk = k & (Ns - 1);
            const int base = (k - kk) * REM + kk;
            // base = k and output j lands at k + j P/REM in this last stage
#pragma unroll
            for (int j = 0; j < (ZHO ? REM / 2 : REM); ++j) buf[padb(base + j * Ns)] = u[q * REM + j];
        }
        if constexpr (WGSYNC)
            __syncthreads();
        else
            wave_sync();
    }
}

}  // namespace llg
