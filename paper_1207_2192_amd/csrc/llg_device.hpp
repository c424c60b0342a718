// Device side of lib_llgdisk: descriptors shared with the host, Philox noise,
// the group barrier and the persistent field/integrator kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"

namespace llg {

constexpr int WG_THREADS = 192;   // one group of three wavefronts: components x, y, z (or packed row pairs)
constexpr int MAX_UG = 4;         // wavefront groups per workgroup
constexpr int MAX_P = 512;
constexpr int MAX_R = 8;
constexpr int LDS_FFT = 3 * 64 * MAX_R * 9 / 8 + 3 * 4 * 32;   // float2 per group: 3 waves x (64/Tf units) x padded P, bank skew
// The row/column spectra are stored in blocks of SB rows: for each spectral
// column kx the SB values of a block are contiguous (one 64-byte segment), so
// a column pass reads whole segments and a row pass over SB/2 row pairs
// writes whole segments.
constexpr int SB = 8;

// A compile-time flag passed as a value (for generic lambdas).
template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

// Per-disk descriptor (device memory, written once by the host).
struct DiskDesc {
    int D, P, H, Dp;          // box, FFT size, P/2+1, D rounded up to a multiple of SB
    int n_pairs, G, n_cells, k;  // row pairs, workgroups, masked cells, index in the batch
    int onchip;               // nonzero: G = 1 and the field kernel and integrators keep the spectra in LDS
    long long m_off;          // float offset of this disk in a packed state
    float* ya;                // stage state A  [3][D][D]
    float* yb;                // stage state B  [3][D][D]
    float* acc;               // RK4 accumulator / Heun m_n + Delta_1/2 / adjoint accumulator [3][D][D]
    float* aux;               // adjoint: direct part of the stage cotangent [3][D][D]
    float2* S;                // row/column spectra [3][Dp/SB][H][SB] (blocks of SB rows)
    const float* spec;        // kernel spectra quarter planes [4][H][H] (xx, yy, xy, zz) / P^2
    const unsigned char* mask;  // [D][D]
    const float2* tw;         // twiddles [P]
    unsigned int* bar;        // group barrier counter (own cache line)
    double* part;             // per-workgroup partial sums [G][PART_STRIDE]
};

// Per-disk parameters (device memory, refreshed when they change).
struct DiskPrm {
    float alpha, c, hx, hy, hz, dtau, sigma;
    float dsigma;          // d sigma / d alpha (Heun adjoint)
    int renorm;
    int drive;             // nonzero: h_ext has a time-dependent part
    double c_d, hx_d, hy_d, hz_d;
    double dtau_d, tau0;   // time step and the time at the start of the call
    double hac[3], freq, phase;      // h_ac sin(2 pi freq tau + phase)
    double hpulse[3], tpulse, inv2w2;   // h_pulse exp(-(tau - tpulse)^2 inv2w2), inv2w2 = 1/(2 w^2)
    float hacf[3], hpulsef[3];       // the same amplitudes in float32 (integrator kernels)
    float phase_rev;                 // phase / (2 pi), reduced to [0, 1)
    float inv2w2_log2e;              // inv2w2 / ln 2 (exponent for exp2)
};

// External field at time tau (the h_ext of eq. Hmm and eq. Bi, here allowed to
// depend on time): the constant part, an oscillation and a Gaussian pulse.
// float64; the oscillation's phase is reduced to one period before the sine.
struct Field3 {
    double x, y, z;
};
__device__ __forceinline__ Field3 hext_at(const DiskPrm& pr, double tau) {
    Field3 h{pr.hx_d, pr.hy_d, pr.hz_d};
    if (pr.drive) {
        double fr = pr.freq * tau;
        fr -= floor(fr);
        const double sn = sin(6.283185307179586476925286766559 * fr + pr.phase);
        const double u = tau - pr.tpulse;
        const double gs = pr.inv2w2 > 0.0 ? exp(-u * u * pr.inv2w2) : 0.0;
        h.x += pr.hac[0] * sn + pr.hpulse[0] * gs;
        h.y += pr.hac[1] * sn + pr.hpulse[1] * gs;
        h.z += pr.hac[2] * sn + pr.hpulse[2] * gs;
    }
    return h;
}

// The same field in float32 for the integrator kernels, where a float64 sine
// and exponential would raise the register count of the whole persistent
// kernel: the oscillation's phase is reduced to one period in float64, then
// the hardware sine of an angle in revolutions and the hardware exp2 (a few
// ulp each; the field enters the float32 induction anyway).
__device__ __forceinline__ void hext_at_f(const DiskPrm& pr, double tau, float& hx, float& hy, float& hz) {
    hx = pr.hx;
    hy = pr.hy;
    hz = pr.hz;
    if (pr.drive) {
        double fr = pr.freq * tau;
        fr -= floor(fr);
        float rv = (float)fr + pr.phase_rev;
        rv -= rv >= 1.0f ? 1.0f : 0.0f;
        const float sn = __builtin_amdgcn_sinf(rv);
        const float u = (float)(tau - pr.tpulse);
        const float gs = pr.inv2w2_log2e > 0.f ? __builtin_amdgcn_exp2f(-u * u * pr.inv2w2_log2e) : 0.f;
        hx += pr.hacf[0] * sn + pr.hpulsef[0] * gs;
        hy += pr.hacf[1] * sn + pr.hpulsef[1] * gs;
        hz += pr.hacf[2] * sn + pr.hpulsef[2] * gs;
    }
}

enum Mode : int {
    MODE_DEMAG = 0,
    MODE_RHS = 1,
    MODE_ENERGY = 2,
    MODE_RK4 = 3,
    MODE_HEUN = 4,
    MODE_RK4_VJP = 5,
    MODE_RELAX = 6,
    MODE_HEUN_VJP = 7
};

constexpr int PART_STRIDE = 8;  // doubles of per-workgroup partial sums

// Kernel instances that can keep a small disk's spectra in LDS: the field
// kernel and the integrators, with one group of three wavefronts per
// workgroup (wider workgroups would carry the extra code path at a higher
// register count in every plan, where it is never the faster choice); the
// adjoint and relaxation kernels always use the workspace in global memory,
// which every disk keeps.
constexpr bool on_chip_mode(int mode) { return mode == MODE_DEMAG || mode == MODE_RK4 || mode == MODE_HEUN; }
constexpr bool on_chip_instance(int mode, int UG) { return on_chip_mode(mode) && UG == 1; }

enum ErrBits : int { ERR_BARRIER = 1, ERR_NONFINITE = 2 };

struct KArgs {
    const DiskDesc* disks;
    const DiskPrm* prm;
    const int* wg2disk;   // -1 for idle workgroups
    const int* wg2local;
    float* m;             // packed state (input, or in/out for the integrators)
    float* out;           // packed output (demag field or rhs), may be null
    float* rec;           // RK4 stage record (stage states and demag fields), may be null
    long long nsteps;
    unsigned long long seed, step0;
    const unsigned long long* step_ptr;   // if set, the Heun step index is read here instead of step0
    unsigned int replica0;
    int mode;
    int* err;
    // constrained relaxation
    const double* relax_x;  // target vortex position per disk (2 doubles, units of a from the centre)
    double* relax_out;      // per disk: lambda_x, lambda_y, sweeps, residual, C_x, C_y, 0, 0
    double kappa, tol;
    double relax_cut2;      // squared constraint radius around the target (units of a^2); <= 0: whole disk
    // observable series of the integrators: every `every` steps (0 = none) the
    // state at the start of the step gives series[(sample * n_disks + k) * 4 + q] =
    // (<m_x>, <m_y>, <m_z>, E) in float64
    double* series;
    int every, n_disks;
    unsigned int spin_limit;   // polls of a group-barrier wait before it gives up (ERR_BARRIER)
};

// ---------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two 32x32->64
// multiplies mixed with the other counter words and the key; the key is bumped
// by two Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
            // bumped where used (scalar adds) rather than a precomputed schedule
            // of twenty long-lived scalar registers
            asm volatile("" : "+s"(k0), "+s"(k1));
        }
        // one 32 x 32 -> 64 multiply per product (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// Uniform in (0, 1) from the top 24 bits of a 32-bit word.
__device__ __forceinline__ float u24(uint32_t x) { return ((float)(x >> 8) + 0.5f) * 5.9604644775390625e-08f; }

// Six standard normals for the two cells (2p, ix), (2p+1, ix) of row pair p:
// two blocks with counters (s_lo, s_hi, 2q + h, replica), h = 0, 1, q = p*D + ix,
// key (seed_lo, seed_hi); the uniforms of block 0 and the first two of block 1
// give three Box-Muller pairs; the even row takes normals 0..2, the odd row 3..5.
__device__ __forceinline__ void thermal_normals_pair(unsigned long long seed, unsigned long long step,
                                                     unsigned long long q, unsigned long long replica,
                                                     float3& even, float3& odd) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t s0 = (uint32_t)step, s1 = (uint32_t)(step >> 32), rep = (uint32_t)replica;
    uint32_t a0 = s0, a1 = s1, a2 = (uint32_t)(2 * q), a3 = rep;
    philox4x32_10(a0, a1, a2, a3, k0, k1);
    uint32_t b0 = s0, b1 = s1, b2 = (uint32_t)(2 * q + 1), b3 = rep;
    philox4x32_10(b0, b1, b2, b3, k0, k1);
    // hardware transcendentals: log2, square root, and sine / cosine of an
    // angle given in revolutions (sin(2 pi u) for u in (0, 1)); each is within
    // a few ulp, far inside what the noise amplitude lets reach the state
    constexpr float M2LN2 = -1.38629436111989061f;   // -2 ln 2:  -2 ln u = -2 ln 2 log2 u
    const float ra = __builtin_amdgcn_sqrtf(M2LN2 * __builtin_amdgcn_logf(u24(a0)));
    const float rb = __builtin_amdgcn_sqrtf(M2LN2 * __builtin_amdgcn_logf(u24(a2)));
    const float rc = __builtin_amdgcn_sqrtf(M2LN2 * __builtin_amdgcn_logf(u24(b0)));
    const float ta = u24(a1), tb = u24(a3), tc = u24(b1);
    even = make_float3(ra * __builtin_amdgcn_cosf(ta), ra * __builtin_amdgcn_sinf(ta), rb * __builtin_amdgcn_cosf(tb));
    odd = make_float3(rb * __builtin_amdgcn_sinf(tb), rc * __builtin_amdgcn_cosf(tc), rc * __builtin_amdgcn_sinf(tc));
}

// ---------------------------------------------------------------- shared buffers
// Buffers that one workgroup writes and another reads inside a launch (row and
// column spectra, stage states) are accessed only through device-scope relaxed
// atomic loads and stores.  On gfx950 these carry the system-coherence bit:
// stores are written through to the device coherence point and loads are
// served from it, so no L2 write-back or invalidate is needed at a barrier;
// the barrier only has to drain the stores (s_waitcnt vmcnt(0)) before it
// signals arrival.  Read-only data (kernel spectra, masks, twiddles) keeps the
// normal cached path.
//
// Every such pointer refers to global memory; accesses go through it as a
// global-address-space pointer (gbl), so that they compile to global rather
// than flat instructions.  (A pending flat access makes the compiler wait for
// every outstanding memory operation at the next use of any loaded value,
// which would serialise prefetched loads.)
#define GLOBAL_AS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL_AS T* gbl(T* p) {
    return (GLOBAL_AS T*)p;
}
__device__ __forceinline__ float ld_sh(const float* p) {
    return __uint_as_float(__hip_atomic_load(gbl(reinterpret_cast<const unsigned int*>(p)), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_sh(float* p, float v) {
    __hip_atomic_store(gbl(reinterpret_cast<unsigned int*>(p)), __float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float2 ld_sh2(const float2* p) {
    const unsigned long long u = __hip_atomic_load(gbl(reinterpret_cast<const unsigned long long*>(p)),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((unsigned int)u), __uint_as_float((unsigned int)(u >> 32)));
}
__device__ __forceinline__ void st_sh2(float2* p, float2 v) {
    const unsigned long long u =
        (unsigned long long)__float_as_uint(v.x) | ((unsigned long long)__float_as_uint(v.y) << 32);
    __hip_atomic_store(gbl(reinterpret_cast<unsigned long long*>(p)), u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_shd(const double* p) {
    return __longlong_as_double((long long)__hip_atomic_load(gbl(reinterpret_cast<const unsigned long long*>(p)),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_shd(double* p, double v) {
    __hip_atomic_store(gbl(reinterpret_cast<unsigned long long*>(p)), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// read-only float2 through a global pointer
__device__ __forceinline__ float2 ldg2(const float2* p) {
    const unsigned long long u = *gbl(reinterpret_cast<const unsigned long long*>(p));
    return make_float2(__uint_as_float((unsigned int)u), __uint_as_float((unsigned int)(u >> 32)));
}
// raise an error flag of the launch
__device__ __forceinline__ void raise_err(int* err, int code) {
    __hip_atomic_fetch_or(gbl(err), code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float4 ld_sh4(const float2* p) {
    const float2 a = ld_sh2(p), b = ld_sh2(p + 1);
    return make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void st_sh4(float2* p, float4 v) {
    st_sh2(p, make_float2(v.x, v.y));
    st_sh2(p + 1, make_float2(v.z, v.w));
}

// Wide accesses to the same shared buffers go through buffer instructions whose
// cache-policy operand sets the same device-coherence bit (sc1) that the
// device-scope atomics above carry; the buffer resource also bounds every
// access to its range (out-of-range loads read 0, stores are dropped).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int CP_DEVICE = 16;   // cache policy: sc1
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
// An offset past the range of every buffer resource: a load there reads 0 and a
// store is dropped, without a memory access.  Loads guarded this way instead of
// by a branch are always issued, so the wait before the first use of a value
// counts only the accesses issued after it and prefetched data stays in flight.
constexpr int OOB = (int)0x80000000u;
// read-only data through the normal cached path (kernel spectra, own accumulator)
__device__ __forceinline__ float bld1c(__amdgpu_buffer_rsrc_t r, int off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ float bld1(__amdgpu_buffer_rsrc_t r, int off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, CP_DEVICE));
}
__device__ __forceinline__ float2 bld2(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CP_DEVICE));
}
__device__ __forceinline__ float4 bld4(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CP_DEVICE));
}
__device__ __forceinline__ void bst2(__amdgpu_buffer_rsrc_t r, int off, float2 v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, CP_DEVICE);
}
__device__ __forceinline__ void bst4(__amdgpu_buffer_rsrc_t r, int off, float4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, CP_DEVICE);
}

// Wait until every store this wave issued has completed (s_waitcnt vmcnt(0):
// vmcnt 0, expcnt 7, lgkmcnt 15 in the gfx9 encoding), as an instruction the
// compiler sees, so that its own wait bookkeeping starts afresh after it.
__device__ __forceinline__ void drain_stores() {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}

// The thread index, optionally passed through an empty asm statement: index
// arithmetic derived from it is then recomputed where it is used inside the
// persistent step loop, instead of being hoisted out of the loop and held in
// registers for the whole launch (which caps the resident wavefronts).  Worth
// it only where register pressure, not latency, limits the kernel.
template <bool OPAQUE>
__device__ __forceinline__ int tid() {
    int x = threadIdx.x;
    if constexpr (OPAQUE) asm volatile("" : "+v"(x));
    return x;
}

// ---------------------------------------------------------------- group barrier
// All workgroups that step one disk meet here.  The counter only grows during
// a launch (it is cleared before each launch); `target` = epoch * G.  A wait
// that exceeds the spin budget raises ERR_BARRIER and returns false so that
// every wave leaves the kernel.
constexpr unsigned int SPIN_LIMIT = 1u << 22;   // default budget (seconds of waiting)

__device__ __forceinline__ bool group_barrier(unsigned int* bar, unsigned int target, int G, int* err,
                                              unsigned int spin_limit) {
    drain_stores();
    __syncthreads();
    if (G == 1) return true;
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(gbl(bar), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned int spins = 0;
        int ok = 1;
        while (__hip_atomic_load(gbl(bar), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin_limit) {
                ok = 0;
                raise_err(err, (int)ERR_BARRIER);
                break;
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace llg
