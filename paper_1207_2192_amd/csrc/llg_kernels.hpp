// Kernels of lib_llgdisk.
//
// llg_persistent: one cooperative launch steps every disk of a batch.  Each
// disk is owned by G workgroups that meet at a per-disk group barrier; there
// is no device-wide barrier, so disks of different sizes progress
// independently.  One field evaluation (demag + exchange + torque) is three
// LDS-resident FFT passes fused into two phases:
//
//   column phase : for each spectral column kx: forward FFT along y of the
//                  three row spectra, multiply by the real kernel spectra,
//                  inverse FFT along y, keep the D rows of the disk.
//   row phase    : for each pair of rows: inverse FFT along x (two real rows
//                  and the packed z pair as three complex transforms), the
//                  exchange sum, the induction b, the torque, the RK4 or Heun
//                  stage update, and the forward FFT along x of the new stage
//                  state, unpacked into the row spectra for the next stage.
//
// The row spectra live in a [3][Dp/SB][P/2+1][SB] complex workspace per disk
// (blocks of SB rows, one 64-byte segment per spectral column and block), so a
// field evaluation moves them through L2/HBM twice per phase pair.  A disk of
// FFT size 64 or 128 that one workgroup steps alone can instead keep that
// workspace in the workgroup's LDS for the whole launch (ONCHIP): the two
// phases then exchange the spectra without leaving the CU, and the disk's
// barriers are workgroup barriers.
#pragma once
#include "llg_device.hpp"

namespace llg {

// Disk membership of cell (j, i) of a D x D box, in exact integer arithmetic:
// the cell centre ((i-(D-1)/2), (j-(D-1)/2)) lies inside or on the circle of
// radius D/2.  Same rule as the host-built mask; computed in registers so
// that no load sits in front of the state loads.
__device__ __forceinline__ bool in_disk(int j, int i, int D) {
    const int x = 2 * i - (D - 1), y = 2 * j - (D - 1);
    return x * x + y * y <= D * D;
}

// Rows staged in LDS per row iteration (the U row pairs and one row above and
// below) and the padded length of a staged row (one zero margin on each side).
template <int P, int R, int UG>
struct RowTile {
    static constexpr int U = UG * (64 / (P / R));
    static constexpr int HR = 2 * U + 2;
    static constexpr int HW = P / 2 + 2;
    static constexpr int floats = 3 * HR * HW;
};

template <int P, int R, int UG, int MODE, bool LARGE, bool SLOT, bool SER, bool ONCHIP>
__device__ __forceinline__ void run_disk(const KArgs& a, const DiskDesc& d, const DiskPrm& pr, int g,
                                         float2* lds, float2* ltw, float* halo, float2* sdyn) {
    constexpr int Tf = P / R;
    constexpr int U = UG * (64 / Tf);          // transforms per component in flight per workgroup
    // the adjoint keeps many values per cell in registers, the P = 512 kernels (LARGE) run
    // at higher occupancy, and four-group workgroups carry four tiles at once: recompute
    // their index arithmetic inside the loop instead of holding it in registers
    constexpr bool OPQ = MODE == MODE_RK4_VJP || MODE == MODE_HEUN_VJP || LARGE || UG != 2;
    constexpr int NT = WG_THREADS * UG;
    constexpr int H = P / 2 + 1;
    const int D = d.D, Dp = d.Dp, G = d.G;
    const int DD = D * D;
    const int wv = tid<OPQ>() >> 6, lane = tid<OPQ>() & 63;
    const int wave = wv % 3, grp = wv / 3;     // wave = component (or packed row) of the group
    const int u = grp * (64 / Tf) + lane / Tf, t = lane % Tf;
    constexpr int PS = padded_len<P>();
    // Row-pass lanes come in groups of UQ row pairs that share one SB-row
    // segment of the spectra; the UQ transform buffers of such a group start on
    // different LDS banks.
    constexpr int UQ = U < SB / 2 ? U : SB / 2;
    constexpr int PSK = UQ == 1 ? PS : PS + (((32 / UQ - PS) % 32) + 32) % 32;
    static_assert(3 * U * PSK <= LDS_FFT * UG, "transform buffers exceed the LDS reservation");
    static_assert(SB == 8, "segment indexing below assumes SB = 8");
    float2* const mybuf = lds + (wave * U + u) * PSK;
#define BUF(w, uu) (lds + ((w) * U + (uu)) * PSK)
    constexpr int HR = RowTile<P, R, UG>::HR, HW = RowTile<P, R, UG>::HW;

    for (int i = tid<OPQ>(); i < P; i += NT) ltw[i] = ldg2(d.tw + i);
    for (int r = tid<OPQ>(); r < 3 * HR; r += NT) {
        halo[r * HW] = 0.f;
        halo[r * HW + HW - 1] = 0.f;
    }
    __syncthreads();

    float* const m = a.m + d.m_off;
    float* const out = a.out ? a.out + d.m_off : nullptr;
    const unsigned char* __restrict__ mask = d.mask;
    float2* __restrict__ S = d.S;
    const int NJB = Dp >> 3;
    const unsigned s_bytes = (unsigned)(3 * H * Dp) * 8u;
    const __amdgpu_buffer_rsrc_t Srs = make_rsrc(S, s_bytes);
    // spectra accesses by byte offset: buffer instructions on the workspace in
    // global memory, or LDS (sdyn) for an on-chip disk; an offset out of range
    // (OOB) reads zero and drops the store in both
    auto sld2 = [&](int off) -> float2 {
        if constexpr (ONCHIP)
            return (unsigned)off < s_bytes ? sdyn[off >> 3] : make_float2(0.f, 0.f);
        else
            return bld2(Srs, off);
    };
    auto sld4 = [&](int off) -> float4 {
        if constexpr (ONCHIP)
            return (unsigned)off < s_bytes ? reinterpret_cast<const float4*>(sdyn)[off >> 4]
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
        else
            return bld4(Srs, off);
    };
    auto sst2 = [&](int off, float2 v) {
        if constexpr (ONCHIP) {
            if ((unsigned)off < s_bytes) sdyn[off >> 3] = v;
        } else {
            bst2(Srs, off, v);
        }
    };
    auto sst4 = [&](int off, float4 v) {
        if constexpr (ONCHIP) {
            if ((unsigned)off < s_bytes) reinterpret_cast<float4*>(sdyn)[off >> 4] = v;
        } else {
            bst4(Srs, off, v);
        }
    };
    if constexpr (ONCHIP) {   // rows no pass writes read as zeros, as in the cleared workspace
        for (int i = tid<OPQ>(); i < 3 * H * Dp; i += NT) sdyn[i] = make_float2(0.f, 0.f);
        __syncthreads();
    }
    const __amdgpu_buffer_rsrc_t Krs = make_rsrc(d.spec, (unsigned)(4 * H * H) * 4u);
    // byte offset of the spectrum of component c, column k, row j
    auto soff = [&](int c, int k, int j) { return ((((c * NJB + (j >> 3)) * H + k) << 3) + (j & 7)) * 8; };
    // row pass: item idx -> (row pair uu of the iteration, spectral column k)
    auto pair_map = [&](int idx, int& uu, int& k) {
        const int uq = idx % UQ, rest = idx / UQ;
        k = rest % H;
        uu = (rest / H) * UQ + uq;
    };
    const int n_rb = (d.n_pairs + U - 1) / U;
    const int n_cb_split = (H + U - 1) / U;       // column tiles of U columns (one wave per component)
    unsigned int epoch = 0;
    // the field kernel serves demag / rhs / energy at run time; the integrators are compiled per mode
    const int mode = (MODE == MODE_DEMAG) ? a.mode : MODE;
    // first Heun step index: from the handle's device counter when one is given
    const unsigned long long step0 = (MODE == MODE_HEUN && a.step_ptr) ? *gbl(a.step_ptr) : a.step0;

    // ---- packed rows of a state into LDS (masked), columns [0, D)
    auto load_state_rows = [&](int b, const float* src) {
        for (int idx = tid<OPQ>(); idx < U * D; idx += NT) {
            const int uu = idx / D, i = idx - uu * D;
            const int p = b * U + uu, j0 = 2 * p, j1 = j0 + 1;
            float x0 = 0.f, y0 = 0.f, z0 = 0.f, x1 = 0.f, y1 = 0.f, z1 = 0.f;
            if (p < d.n_pairs) {
                const int c0 = j0 * D + i;
                if (in_disk(j0, i, D)) {
                    x0 = ld_sh(src + c0);
                    y0 = ld_sh(src + DD + c0);
                    z0 = ld_sh(src + 2 * DD + c0);
                }
                if (j1 < D) {
                    const int c1 = j1 * D + i;
                    if (in_disk(j1, i, D)) {
                        x1 = ld_sh(src + c1);
                        y1 = ld_sh(src + DD + c1);
                        z1 = ld_sh(src + 2 * DD + c1);
                    }
                }
            }
            BUF(0, uu)[padb(i)] = make_float2(x0, y0);
            BUF(1, uu)[padb(i)] = make_float2(x1, y1);
            BUF(2, uu)[padb(i)] = make_float2(z0, z1);
        }
        __syncthreads();
    };

    // ---- forward transforms along x of the packed rows in LDS; unpack to S
    auto row_forward_store = [&](int b) {
        float2 v[R];   // columns at or past P/2 (>= D) are zero
#pragma unroll
        for (int j = 0; j < R / 2; ++j) {
            const int i = t + j * Tf;
            v[j] = (i < D) ? mybuf[padb(i)] : make_float2(0.f, 0.f);
        }
        fft_run<P, R, false, false, true, true>(v, mybuf, ltw, t);
        for (int idx = tid<OPQ>(); idx < U * H; idx += NT) {
            int uu, k;
            pair_map(idx, uu, k);
            const int p = b * U + uu;
            if (p >= d.n_pairs) continue;
            const int j0 = 2 * p;
            const int km = (P - k) & (P - 1);
            const float2 A0 = BUF(0, uu)[padb(k)], B0 = BUF(0, uu)[padb(km)];
            const float2 A1 = BUF(1, uu)[padb(k)], B1 = BUF(1, uu)[padb(km)];
            const float2 A2 = BUF(2, uu)[padb(k)], B2 = BUF(2, uu)[padb(km)];
            // two real rows packed as a + i b:  a^ = (A + conj B)/2,  b^ = (A - conj B)/(2i)
            const float4 sx = make_float4(0.5f * (A0.x + B0.x), 0.5f * (A0.y - B0.y),
                                          0.5f * (A1.x + B1.x), 0.5f * (A1.y - B1.y));
            const float4 sy = make_float4(0.5f * (A0.y + B0.y), -0.5f * (A0.x - B0.x),
                                          0.5f * (A1.y + B1.y), -0.5f * (A1.x - B1.x));
            const float4 sz = make_float4(0.5f * (A2.x + B2.x), 0.5f * (A2.y - B2.y),
                                          0.5f * (A2.y + B2.y), -0.5f * (A2.x - B2.x));
            sst4(soff(0, k, j0), sx);
            sst4(soff(1, k, j0), sy);
            sst4(soff(2, k, j0), sz);
        }
        __syncthreads();
    };

    // ---- column phase, one transform slot per column (for disks with several
    // column tiles per workgroup): each transform slot (lane group) takes one spectral
    // column kx with all three components: forward FFTs along y, the kernel
    // multiply in registers (x: Kxx mx + Kxy my, y: Kxy mx + Kyy my, z: Kzz mz),
    // inverse FFTs, and stores of the D rows of the disk.  A slot's LDS buffer
    // belongs to its wavefront alone, so the phase has no workgroup barrier;
    // where P is a power of the radix the forward results stay in registers in
    // exactly the order the inverse transform takes them.
    // Rows at or past P/2 (>= D) are zero on input and not needed on output,
    // so the points j >= R/2 of a lane are neither loaded nor stored.
    constexpr bool KEEP = fft_whole_radix<P, R>();
    constexpr int NSLOT = 3 * U;
    const int slot = wave * U + u;
    StageTwiddles<P, R> stw;
    auto col_fwd = [&](float2 (&v)[R]) {
        __builtin_amdgcn_sched_barrier(0);   // one transform at a time: bounds the live registers
        if constexpr (KEEP) {
            fft_run<P, R, false, true, true, true>(v, mybuf, ltw, t, &stw);
        } else {
            fft_run<P, R, false, false, false, true>(v, mybuf, ltw, t, &stw);
#pragma unroll
            for (int j = 0; j < R; ++j) v[j] = mybuf[padb(t + j * Tf)];
            wave_sync();
        }
    };
    auto col_inv_store = [&](int c, int kx, float2 (&v)[R]) {
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (KEEP) {
            fft_run<P, R, true, true>(v, mybuf, ltw, t, &stw);   // v[j] = column value at row t + j*Tf
#pragma unroll
            for (int j = 0; j < R / 2; ++j) {
                const int i = t + j * Tf;
                sst2(i < D ? soff(c, kx, i) : OOB, v[j]);
            }
        } else {
            fft_run<P, R, true, false, false, false, true>(v, mybuf, ltw, t, &stw);
#pragma unroll
            for (int j = 0; j < R / 2; ++j) {
                const int i = t + j * Tf;
                sst2(i < D ? soff(c, kx, i) : OOB, mybuf[padb(i)]);
            }
            wave_sync();
        }
    };
    // all columns of this workgroup.  At P = 512 (one transform slot per
    // wavefront) round r of the disk's workgroups takes the G * 3U columns from
    // r * G * 3U on, dealt to the workgroups in turn, so that the last, partial
    // round is spread over all of them, and a slot without a column skips it
    // (the phase has no workgroup barrier); below P = 512 a workgroup takes
    // tiles of 3U adjacent columns (tile b = g + r G), which measured faster for
    // the ragged ensemble, and a slot past the last column skips the tile.
    // Either way every column a slot transforms is a real one (kx < H).
    // z first (it needs only Kzz), while the x and y columns are still
    // arriving.  The kernel spectra are loaded ahead of the transform before
    // the one that needs them (Kzz with the columns, Kxx, Kyy and Kxy before
    // the z transform's inverse), so that no memory latency sits between two
    // transforms of a column.
    auto column_item = [&](int kx) {
        float2 X[R], Y[R], Z[R];
#pragma unroll
        for (int j = 0; j < R / 2; ++j) {
            const int i = t + j * Tf;
            Z[j] = sld2(i < D ? soff(2, kx, i) : OOB);
        }
#pragma unroll
        for (int j = 0; j < R / 2; ++j) {
            const int i = t + j * Tf;
            const bool ok = i < D;
            X[j] = sld2(ok ? soff(0, kx, i) : OOB);
            Y[j] = sld2(ok ? soff(1, kx, i) : OOB);
        }
        // kernel spectra at this lane's points: quarter-plane planes 0 = xx, 1 = yy, 2 = xy, 3 = zz
        auto kidx = [&](int j) {
            const int ky = t + j * Tf;
            return kx * H + (ky <= P / 2 ? ky : P - ky);
        };
        float kzz[R];
#pragma unroll
        for (int j = 0; j < R; ++j) kzz[j] = bld1c(Krs, (3 * H * H + kidx(j)) * 4);
        col_fwd(Z);
        float kxx[R], kyy[R], kxy[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int o = kidx(j);
            kxx[j] = bld1c(Krs, o * 4);
            kyy[j] = bld1c(Krs, (H * H + o) * 4);
            kxy[j] = bld1c(Krs, (2 * H * H + o) * 4);
        }
#pragma unroll
        for (int j = 0; j < R; ++j) Z[j] = make_float2(kzz[j] * Z[j].x, kzz[j] * Z[j].y);
        col_inv_store(2, kx, Z);
        col_fwd(X);
        col_fwd(Y);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float axy = t + j * Tf <= P / 2 ? kxy[j] : -kxy[j];   // K_xy is odd in ky
            const float2 x = X[j], y = Y[j];
            X[j] = make_float2(kxx[j] * x.x + axy * y.x, kxx[j] * x.y + axy * y.y);
            Y[j] = make_float2(axy * x.x + kyy[j] * y.x, axy * x.y + kyy[j] * y.y);
        }
        col_inv_store(0, kx, X);
        col_inv_store(1, kx, Y);
    };
    auto column_pass_slot = [&]() {
        stage_twiddles<P, R>(stw, ltw, t);
        if constexpr (P == 512) {
            for (int base = 0; base < H; base += G * NSLOT) {
                const int kx = base + slot * G + g;
                if (kx < H) column_item(kx);
            }
        } else {
            const int n_cb = (H + NSLOT - 1) / NSLOT;
            for (int b = g; b < n_cb; b += G) {
                const int kx = b * NSLOT + slot;
                if (kx < H) column_item(kx);
            }
        }
    };

    // ---- column phase, one wavefront per component (for disks with more
    // workgroups than column tiles): tile b holds the U columns kx = b*U + u and
    // wave c of a group transforms component c.  The multiply is fused into the
    // loads of the inverse transform: each lane forms its own inputs ky = t + j*Tf
    // from the three forward spectra (x wave: Kxx mx + Kxy my, y wave: Kxy mx +
    // Kyy my, z wave: Kzz mz), with the kernel spectra of those points loaded
    // together with the column.
    struct ColV {
        float2 v[R];          // this lane's column values
    };
    struct ColK {
        float k0[R], k1[R];   // kernel spectra at this lane's points (quarter-plane values)
    };
    // column values of tile b (zeros past the last column)
    auto col_load_v = [&](int b, ColV& c) {
        const int kx = b * U + u;
        const bool valid = kx < H;
#pragma unroll
        for (int j = 0; j < R / 2; ++j) {   // rows at or past P/2 (>= D) are zero
            const int i = t + j * Tf;
            c.v[j] = sld2((valid && i < D) ? soff(wave, kx, i) : OOB);
        }
    };
    auto col_load_k = [&](int b, ColK& c) {
        const int kx = b * U + u;
        const bool valid = kx < H;
        // planes: 0 = xx, 1 = yy, 2 = xy, 3 = zz
        const int pl0 = wave == 0 ? 0 : wave == 1 ? 2 : 3;
        const int pl1 = wave == 0 ? 2 : 1;
        const int o0 = (pl0 * H + kx) * H, o1 = (pl1 * H + kx) * H;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int ky = t + j * Tf;
            const int kq = ky <= P / 2 ? ky : P - ky;
            c.k0[j] = bld1c(Krs, valid ? (o0 + kq) * 4 : OOB);
            c.k1[j] = bld1c(Krs, (valid && wave < 2) ? (o1 + kq) * 4 : OOB);
        }
    };
    auto col_compute = [&](int b, ColV& c, const ColK& kk) {
        const int kx = b * U + u;
        const bool valid = kx < H;
        fft_run<P, R, false, false, true, true>(c.v, mybuf, ltw, t);   // ends with a workgroup barrier
        float2 v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int ky = t + j * Tf;
            const float sg = ky <= P / 2 ? 1.f : -1.f;   // K_xy is odd in ky
            const float2 A = BUF(wave == 2 ? 2 : 0, u)[padb(ky)];
            if (wave == 2) {
                v[j] = make_float2(kk.k0[j] * A.x, kk.k0[j] * A.y);
            } else {
                const float2 B = BUF(1, u)[padb(ky)];
                const float ka = wave == 0 ? kk.k0[j] : sg * kk.k0[j];
                const float kb = wave == 0 ? sg * kk.k1[j] : kk.k1[j];
                v[j] = make_float2(ka * A.x + kb * B.x, ka * A.y + kb * B.y);
            }
        }
        __syncthreads();   // every wave has its inputs before the transforms overwrite the spectra
        if constexpr (KEEP) {
            fft_run<P, R, true, true>(v, mybuf, ltw, t);   // v[j] = column value at row t + j*Tf
#pragma unroll
            for (int j = 0; j < R / 2; ++j) {
                const int i = t + j * Tf;
                sst2((valid && i < D) ? soff(wave, kx, i) : OOB, v[j]);
            }
        } else {
            fft_run<P, R, true, false, true, false, true>(v, mybuf, ltw, t);
#pragma unroll
            for (int j = 0; j < R / 2; ++j) {
                const int i = t + j * Tf;
                sst2((valid && i < D) ? soff(wave, kx, i) : OOB, mybuf[padb(i)]);
            }
        }
    };
    // all column tiles of this workgroup; the column values of the next tile are
    // loaded before the current tile is transformed, so their memory latency
    // overlaps the transforms (tiles write only their own columns)
    auto column_pass_split = [&]() {
        if (g >= n_cb_split) return;
        ColV cur;
        col_load_v(g, cur);
        for (int b = g; b < n_cb_split; b += G) {
            ColK kk;
            col_load_k(b, kk);
            ColV nxt;
            col_load_v(b + G, nxt);
            col_compute(b, cur, kk);
            cur = nxt;
        }
    };

    // The column strategy is part of the transform policy: one wavefront per
    // component (more lanes per column, for disks with few column tiles per
    // workgroup) or one lane group per column (less LDS traffic, no workgroup
    // barriers, for many tiles per workgroup).
    auto column_pass = [&]() {
        if constexpr (SLOT)
            column_pass_slot();
        else
            column_pass_split();
    };

    // ---- rebuild the full-length row spectra of a pair and transform back along x
    constexpr int IS = (U * H + NT - 1) / NT;
    struct SRow {
        float4 x, y, z;
    };
    auto row_load = [&](int b, SRow (&sv)[IS]) {
#pragma unroll
        for (int q = 0; q < IS; ++q) {
            const int idx = tid<OPQ>() + q * NT;
            int uu, k;
            pair_map(idx, uu, k);
            const int p = b * U + uu;
            const bool ok = idx < U * H && p < d.n_pairs;
            const int j0 = 2 * p;
            sv[q].x = sld4(ok ? soff(0, k, j0) : OOB);
            sv[q].y = sld4(ok ? soff(1, k, j0) : OOB);
            sv[q].z = sld4(ok ? soff(2, k, j0) : OOB);
        }
    };
    auto row_unpack_inverse = [&](const SRow (&sv)[IS]) {
#pragma unroll
        for (int q = 0; q < IS; ++q) {
            const int idx = tid<OPQ>() + q * NT;
            if (idx >= U * H) continue;
            int uu, k;
            pair_map(idx, uu, k);
            const float4 sx = sv[q].x, sy = sv[q].y, sz = sv[q].z;
            // Hx + i Hy of each row, Hz(j0) + i Hz(j1); mirrored half from Hermitian symmetry
            BUF(0, uu)[padb(k)] = make_float2(sx.x - sy.y, sx.y + sy.x);
            BUF(1, uu)[padb(k)] = make_float2(sx.z - sy.w, sx.w + sy.z);
            BUF(2, uu)[padb(k)] = make_float2(sz.x - sz.w, sz.y + sz.z);
            if (k > 0 && k < P / 2) {
                const int km = P - k;
                BUF(0, uu)[padb(km)] = make_float2(sx.x + sy.y, sy.x - sx.y);
                BUF(1, uu)[padb(km)] = make_float2(sx.z + sy.w, sy.z - sx.w);
                BUF(2, uu)[padb(km)] = make_float2(sz.x + sz.w, sz.z - sz.y);
            }
        }
        __syncthreads();
        float2 v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = mybuf[padb(t + j * Tf)];
        fft_run<P, R, true, false, true, false, true>(v, mybuf, ltw, t);   // only columns < P/2 (>= D) are read
    };
    auto row_inverse = [&](int b) {
        SRow sv[IS];
        row_load(b, sv);
        row_unpack_inverse(sv);
    };

    // ---- stage state rows 2bU-1 .. 2bU+2U of iteration b into LDS (masked; zero
    // outside the box), halo[(c*HR + rr)*HW + 1 + i] for row 2bU-1+rr and column i
    // Staged-row element q of this thread.  Where the index arithmetic is
    // recomputed inside the loop (OPQ) the rows are spread over the wavefronts,
    // one whole row per wavefront and round (row = wave + r * waves, uniform
    // across the wavefront) with lane l taking columns l + 64 v (coalesced), so
    // the per-element arithmetic is an add and the disk test; where it is
    // hoisted, elements run over rows x columns by thread index.
    constexpr int HC = P / 2;                    // staged columns (D <= P/2)
    constexpr int NWV = 3 * UG;                  // wavefronts of the workgroup
    constexpr int VW = HC >= 64 ? HC / 64 : 1;   // columns per lane and row
    constexpr int HQ = (3 * HR + NWV - 1) / NWV; // rounds of rows
    constexpr int IH = OPQ ? HQ * VW : (3 * HR * HC + NT - 1) / NT;
    auto halo_elem = [&](int q, int& row, int& i) {
        if constexpr (OPQ) {
            row = __builtin_amdgcn_readfirstlane(tid<OPQ>() >> 6) + (q / VW) * NWV;
            i = (tid<OPQ>() & 63) + 64 * (q % VW);
        } else {
            const int e = tid<OPQ>() + q * NT;
            row = e / HC;
            i = e % HC;
        }
    };
    // Cells outside the disk read as zero: a state this kernel wrote is zero
    // there already (every stage stores the whole box), so only a caller's
    // state (MASKED) needs the disk test.
    auto halo_load_t = [&](auto masked, int b, const float* Ys, float (&hv)[IH]) {
        constexpr bool MASKED = decltype(masked)::value;
        const __amdgpu_buffer_rsrc_t Yr = make_rsrc(Ys, (unsigned)(3 * DD) * 4u);
#pragma unroll
        for (int q = 0; q < IH; ++q) {
            int row, i;
            halo_elem(q, row, i);
            const int c = row / HR, rr = row - c * HR;
            const int j = 2 * b * U - 1 + rr;
            const bool ok = row < 3 * HR && i < D && j >= 0 && j < D && (!MASKED || in_disk(j, i, D));
            hv[q] = bld1(Yr, ok ? (c * DD + j * D + i) * 4 : OOB);
        }
    };
    auto halo_load = [&](int b, const float* Ys, float (&hv)[IH], bool masked) {
        if (masked)
            halo_load_t(BoolC<true>{}, b, Ys, hv);
        else
            halo_load_t(BoolC<false>{}, b, Ys, hv);
    };
    auto halo_store = [&](const float (&hv)[IH]) {
#pragma unroll
        for (int q = 0; q < IH; ++q) {
            int row, i;
            halo_elem(q, row, i);
            if (row < 3 * HR && i < HC) halo[row * HW + 1 + i] = hv[q];
        }
    };

    double e_ex = 0.0, e_dm = 0.0, e_ext = 0.0;
    const float cf = pr.c, al = pr.alpha, dt = pr.dtau;
    // external field of the stage being evaluated: constant, or set per stage
    // from its time when h_ext depends on time
    float hxf = pr.hx, hyf = pr.hy, hzf = pr.hz;
    double hxd = pr.hx_d, hyd = pr.hy_d, hzd = pr.hz_d;
    // (float64 for the field kernel's energy and the relaxation, both at tau0;
    // float32 hardware transcendentals in the integrators' stage loop)
    auto set_field = [&](double tau) {
        if (pr.drive) {
            if constexpr (MODE == MODE_RK4 || MODE == MODE_HEUN) {
                hext_at_f(pr, tau, hxf, hyf, hzf);
                hxd = hxf;
                hyd = hyf;
                hzd = hzf;
            } else {
                const Field3 h = hext_at(pr, tau);
                hxd = h.x;
                hyd = h.y;
                hzd = h.z;
                hxf = (float)h.x;
                hyf = (float)h.y;
                hzf = (float)h.z;
            }
        }
    };
    set_field(pr.tau0);
    // stage times as fractions of a step: RK4 (0, 1/2, 1/2, 1), Heun (0, 1)
    auto stage_frac = [](int nst, int s) { return nst == 4 ? (s == 0 ? 0.0 : s == 3 ? 1.0 : 0.5) : (double)s; };
    // observable series (kernel instances with SER only): float64 sums of m and
    // of the energy density of the state at the start of a sampled step (its
    // field is the stage-0 field), one slot per wavefront in LDS, so that no
    // register is held across the transforms
    constexpr bool SERIES = SER && (MODE == MODE_RK4 || MODE == MODE_HEUN);
    __shared__ double red4[SERIES ? 3 * MAX_UG : 1][4];

    // ---- per-cell work after the inverse transforms; new stage state back into LDS
    // stage s of step n; Ys = state whose field is in LDS; Yn = where the next stage state goes.
    // The stage state around the row pairs comes from LDS (staged rows); the
    // step's start state and the accumulator of the two cells of a column are
    // loaded into registers before the row spectra, so that all of the
    // iteration's loads share one memory latency.
    // (RK4: at stage 0 the state being evaluated is the start state itself, so
    // its values come from the staged rows and only later stages load it;
    // Heun: the corrector's base m_n + Delta_1/2 is kept in the accumulator)
    auto need_y0 = [&](int s) { return mode == MODE_RK4 && s > 0; };
    // stage record: per step, per stage, (stage state, demag field) of [3][D][D]
    constexpr int NST = (MODE == MODE_HEUN || MODE == MODE_HEUN_VJP) ? 2 : 4;
    float* const recd = a.rec ? a.rec + (size_t)a.nsteps * (2 * NST) * (size_t)d.m_off : nullptr;
    // Gathered values of one column of a row pair (registers).
    struct Gath {
        float y0[2][3], ac[2][3];
    };
    constexpr int IC = (U * (P / 2) + NT - 1) / NT;   // cell-update items per thread (D <= P/2)
    // Cell-update item idx -> (row pair uu of the iteration, column i).  Where
    // the index arithmetic is recomputed inside the loop (OPQ) the columns sit on
    // a stride of P/2 (shifts, no division by D); where it is hoisted, on a
    // stride of D (fewer idle items).
    auto cell_item = [&](int idx, int& uu, int& i) {
        if constexpr (OPQ) {
            uu = idx / (P / 2);
            i = idx % (P / 2);
            return uu < U && i < D;
        } else {
            uu = idx / D;
            i = idx - uu * D;
            return idx < U * D;
        }
    };
    Gath gv[IC];
    // this thread's cells of row iteration b (the cell-update items): m from the
    // staged rows, H from the inverse transforms, added to the wavefront's slots
    auto sample_pass = [&](int b) {
        double q4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < IC; ++q) {
            int uu, i;
            if (!cell_item(tid<OPQ>() + q * NT, uu, i)) continue;
            const int p = b * U + uu;
            if (p >= d.n_pairs) continue;
            const float2 hz2 = BUF(2, uu)[padb(i)];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = 2 * p + r;
                if (j >= D || !in_disk(j, i, D)) continue;
                const float2 hxy = BUF(r, uu)[padb(i)];
                const double H3[3] = {(double)hxy.x, (double)hxy.y, (double)(r == 0 ? hz2.x : hz2.y)};
                const double h3[3] = {hxd, hyd, hzd};
                double ex = 0.0, ed = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float* hr = halo + (c * HR + 2 * uu + r) * HW + 1 + i;   // row j - 1 of the stage
                    const double mc = hr[HW];
                    const double e3 = (double)hr[0] + (double)hr[2 * HW] + (double)hr[HW - 1] + (double)hr[HW + 1];
                    q4[c] += mc;
                    ex += mc * e3;
                    ed += mc * (h3[c] + 0.5 * H3[c]);
                }
                q4[3] += -0.5 * ex - pr.c_d * ed;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double v = wave_sum(q4[c]);
            if (lane == 0) red4[wv][c] += v;
        }
    };
    auto gather = [&](int b, int s) {
        const bool need_acc = (mode == MODE_RK4 && s > 0) || (mode == MODE_HEUN && s == 1);
        const bool ny0 = need_y0(s);
        const __amdgpu_buffer_rsrc_t Mrs = make_rsrc(m, (unsigned)(3 * DD) * 4u);
        const __amdgpu_buffer_rsrc_t Ars = make_rsrc(d.acc, (unsigned)(3 * DD) * 4u);
        // a stage that needs neither array issues no load at all (the
        // conditions are uniform); masked elements of a needed one read zero
#pragma unroll
        for (int q = 0; q < IC; ++q) {
            int uu, i;
            const bool item = cell_item(tid<OPQ>() + q * NT, uu, i);
            const int p = b * U + uu;
            const bool live = item && p < d.n_pairs;
            const int j0 = 2 * p;
            Gath& G_ = gv[q];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = j0 + r;
                const bool okc = live && j < D;   // values outside the disk are never used
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int cell = c * DD + j * D + i;
                    G_.y0[r][c] = 0.f;
                    G_.ac[r][c] = 0.f;
                    if (ny0) G_.y0[r][c] = bld1(Mrs, okc ? cell * 4 : OOB);
                    if (need_acc) G_.ac[r][c] = bld1c(Ars, okc ? cell * 4 : OOB);
                }
            }
        }
    };
    auto cell_update = [&](int b, int s, long long n, float* Yn) {
#pragma unroll
        for (int q = 0; q < IC; ++q) {
            int uu, i;
            if (!cell_item(tid<OPQ>() + q * NT, uu, i)) continue;   // same items as the gather
            const int p = b * U + uu;
            if (p >= d.n_pairs) continue;
            const int j0 = 2 * p;
            float col[4][3], lft[2][3], rgt[2][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float* hr = halo + (c * HR + 2 * uu) * HW + 1 + i;
#pragma unroll
                for (int r = 0; r < 4; ++r) col[r][c] = hr[r * HW];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    lft[r][c] = hr[(r + 1) * HW - 1];
                    rgt[r][c] = hr[(r + 1) * HW + 1];
                }
            }
            const float (&y0)[2][3] = gv[q].y0;
            const float (&ac)[2][3] = gv[q].ac;
            const float2 hz2 = BUF(2, uu)[padb(i)];
            float nxt[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
            float3 wn[2];
            // both Heun stages draw the step's noise from the same counters
            if (mode == MODE_HEUN && (in_disk(j0, i, D) || (j0 + 1 < D && in_disk(j0 + 1, i, D))))
                thermal_normals_pair(a.seed, step0 + (unsigned long long)n, (unsigned long long)(p * D + i),
                                     (unsigned long long)(a.replica0 + d.k), wn[0], wn[1]);
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = j0 + r;
                if (j >= D) break;
                const int cell = j * D + i;
                const bool in = in_disk(j, i, D);
                const float2 hxy = BUF(r, uu)[padb(i)];
                const float Hx = hxy.x, Hy = hxy.y, Hz = r == 0 ? hz2.x : hz2.y;
                if (mode == MODE_DEMAG) {
                    gbl(out)[cell] = in ? Hx : 0.f;
                    gbl(out)[DD + cell] = in ? Hy : 0.f;
                    gbl(out)[2 * DD + cell] = in ? Hz : 0.f;
                    continue;
                }
                const float mx = col[r + 1][0], my = col[r + 1][1], mz = col[r + 1][2];
                if (mode == MODE_ENERGY) {
                    if (!in) continue;
                    double e3[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        e3[c] = (double)col[r][c] + (double)col[r + 2][c] + (double)lft[r][c] + (double)rgt[r][c];
                    const double mxd = mx, myd = my, mzd = mz;
                    e_ex += -0.5 * (mxd * e3[0] + myd * e3[1] + mzd * e3[2]);
                    e_dm += -0.5 * pr.c_d * (mxd * (double)Hx + myd * (double)Hy + mzd * (double)Hz);
                    e_ext += -pr.c_d * (mxd * hxd + myd * hyd + mzd * hzd);
                    continue;
                }
                const float bx = (col[r][0] + col[r + 2][0] + lft[r][0] + rgt[r][0]) + cf * (hxf + Hx);
                const float by = (col[r][1] + col[r + 2][1] + lft[r][1] + rgt[r][1]) + cf * (hyf + Hy);
                const float bz = (col[r][2] + col[r + 2][2] + lft[r][2] + rgt[r][2]) + cf * (hzf + Hz);
                float nx = 0.f, ny = 0.f, nzv = 0.f;
                if (mode == MODE_RHS || mode == MODE_RK4) {
                    // f = m x b - alpha m x (m x b)
                    const float px = my * bz - mz * by, py = mz * bx - mx * bz, pz = mx * by - my * bx;
                    const float fx = px - al * (my * pz - mz * py);
                    const float fy = py - al * (mz * px - mx * pz);
                    const float fz = pz - al * (mx * py - my * px);
                    if (mode == MODE_RHS) {
                        gbl(out)[cell] = in ? fx : 0.f;
                        gbl(out)[DD + cell] = in ? fy : 0.f;
                        gbl(out)[2 * DD + cell] = in ? fz : 0.f;
                        continue;
                    }
                    if (recd) {
                        GLOBAL_AS float* rs = gbl(recd) + ((size_t)(n * 4 + s) * 2) * 3 * DD + cell;
                        rs[0] = in ? mx : 0.f;
                        rs[DD] = in ? my : 0.f;
                        rs[2 * DD] = in ? mz : 0.f;
                        rs[3 * DD] = in ? Hx : 0.f;
                        rs[4 * DD] = in ? Hy : 0.f;
                        rs[5 * DD] = in ? Hz : 0.f;
                    }
                    if (in) {
                        if (s < 3) {
                            const float w = (s == 0) ? 1.f : 2.f;
                            gbl(d.acc)[cell] = ac[r][0] + w * fx;
                            gbl(d.acc)[DD + cell] = ac[r][1] + w * fy;
                            gbl(d.acc)[2 * DD + cell] = ac[r][2] + w * fz;
                            const float h = (s == 2) ? dt : 0.5f * dt;
                            nx = (s == 0 ? mx : y0[r][0]) + h * fx;
                            ny = (s == 0 ? my : y0[r][1]) + h * fy;
                            nzv = (s == 0 ? mz : y0[r][2]) + h * fz;
                        } else {
                            const float h6 = dt * (1.0f / 6.0f);
                            nx = y0[r][0] + h6 * (ac[r][0] + fx);
                            ny = y0[r][1] + h6 * (ac[r][1] + fy);
                            nzv = y0[r][2] + h6 * (ac[r][2] + fz);
                            if (pr.renorm) {
                                const float rn = 1.0f / sqrtf(nx * nx + ny * ny + nzv * nzv);
                                nx *= rn;
                                ny *= rn;
                                nzv *= rn;
                            }
                            if (!(isfinite(nx) && isfinite(ny) && isfinite(nzv)))
                                raise_err(a.err, (int)ERR_NONFINITE);
                        }
                    }
                } else if (in) {  // MODE_HEUN
                    if (recd) {
                        GLOBAL_AS float* rs = gbl(recd) + ((size_t)(n * 2 + s) * 2) * 3 * DD + cell;
                        rs[0] = mx;
                        rs[DD] = my;
                        rs[2 * DD] = mz;
                        rs[3 * DD] = Hx;
                        rs[4 * DD] = Hy;
                        rs[5 * DD] = Hz;
                    }
                    const float3 w = wn[r];
                    const float sg = pr.sigma;
                    const float gx = bx * dt + sg * w.x, gy = by * dt + sg * w.y, gz = bz * dt + sg * w.z;
                    const float px = my * gz - mz * gy, py = mz * gx - mx * gz, pz = mx * gy - my * gx;
                    const float dx = px - al * (my * pz - mz * py);
                    const float dy = py - al * (mz * px - mx * pz);
                    const float dz = pz - al * (mx * py - my * px);
                    if (s == 0) {
                        // predictor m~ = m + Delta_1; m + Delta_1/2 kept for the corrector
                        gbl(d.acc)[cell] = mx + 0.5f * dx;
                        gbl(d.acc)[DD + cell] = my + 0.5f * dy;
                        gbl(d.acc)[2 * DD + cell] = mz + 0.5f * dz;
                        nx = mx + dx;
                        ny = my + dy;
                        nzv = mz + dz;
                    } else {
                        // corrector m' = (m + Delta_1/2) + Delta_2/2
                        nx = ac[r][0] + 0.5f * dx;
                        ny = ac[r][1] + 0.5f * dy;
                        nzv = ac[r][2] + 0.5f * dz;
                        if (pr.renorm) {
                            const float rn = 1.0f / sqrtf(nx * nx + ny * ny + nzv * nzv);
                            nx *= rn;
                            ny *= rn;
                            nzv *= rn;
                        }
                        if (!(isfinite(nx) && isfinite(ny) && isfinite(nzv)))
                            raise_err(a.err, (int)ERR_NONFINITE);
                    }
                }
                // integrators: store the next stage state (zero outside the disk)
                st_sh(Yn + cell, nx);
                st_sh(Yn + DD + cell, ny);
                st_sh(Yn + 2 * DD + cell, nzv);
                nxt[r][0] = nx;
                nxt[r][1] = ny;
                nxt[r][2] = nzv;
            }
            if (mode == MODE_RK4 || mode == MODE_HEUN) {
                BUF(0, uu)[padb(i)] = make_float2(nxt[0][0], nxt[0][1]);
                BUF(1, uu)[padb(i)] = make_float2(nxt[1][0], nxt[1][1]);
                BUF(2, uu)[padb(i)] = make_float2(nxt[0][2], nxt[1][2]);
            }
        }
        __syncthreads();
    };

    // ---- adjoint of RK4 (backward stage k finishes stage k-1 and starts stage k)
    // Backward stage k <-> step n = N-1-k/4, forward stage s = 3-k%4.  With the
    // recorded stage state Y and demag field H of that stage, the cotangent kb of
    // the stage slope gives (b = exchange(Y) + c (h + H)):
    //   direct part  mdir = b x kb - alpha [(Y x b) x kb + b x (kb x Y)]
    //   field part   bbar = kb x Y - alpha (kb x Y) x Y
    //   stage cotangent  Ybar = mdir + exchange(bbar) + c K bbar   (K: demag, self-adjoint)
    //   alpha_bar += kb . (-Y x (Y x b)),   c_bar += bbar . (h + H).
    // The slope cotangents follow RK4 backwards: kb_4 = dt/6 yb', kb_3 = dt/3 yb' + dt Ybar_4,
    // kb_2 = dt/3 yb' + dt/2 Ybar_3, kb_1 = dt/6 yb' + dt/2 Ybar_2;  yb = yb' + sum Ybar.
    auto vjp_update = [&](int b, long long k, long long K) {
        const long long N = a.nsteps;
        const bool fin = k > 0, sta = k < K;
        const long long nf = fin ? N - 1 - (k - 1) / 4 : 0, ns = sta ? N - 1 - k / 4 : 0;
        const int sf = fin ? 3 - (int)((k - 1) % 4) : 0, ss = sta ? 3 - (int)(k % 4) : 0;
        const float* Bf = ((k - 1) & 1) ? d.yb : d.ya;      // bbar of the finishing stage
        float* Bs = (k & 1) ? d.yb : d.ya;                  // bbar of the starting stage
        const GLOBAL_AS float* Yrec = gbl(recd) + ((size_t)(ns * 4 + ss) * 2) * 3 * DD;
        const GLOBAL_AS float* Hrec = Yrec + 3 * DD;
        const GLOBAL_AS float* Hfin = gbl(recd) + ((size_t)(nf * 4 + sf) * 2 + 1) * 3 * DD;
        // external field at the finishing and at the starting stage
        const Field3 hF = hext_at(pr, pr.tau0 + ((double)nf + stage_frac(4, sf)) * pr.dtau_d);
        const Field3 hS = hext_at(pr, pr.tau0 + ((double)ns + stage_frac(4, ss)) * pr.dtau_d);
        const float hh[3] = {(float)hF.x, (float)hF.y, (float)hF.z};
        const float hsx = (float)hS.x, hsy = (float)hS.y, hsz = (float)hS.z;
        for (int idx = tid<OPQ>(); idx < U * D; idx += NT) {
            const int uu = idx / D, i = idx - uu * D;
            const int p = b * U + uu;
            if (p >= d.n_pairs) continue;
            const int j0 = 2 * p;
            float bc[4][3], bl[2][3], br[2][3], yc[4][3], yl[2][3], yr[2][3];
            float ax[2][3], ac[2][3], hf[2][3], hs[2][3], yb0[2][3];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 - 1 + r;
                const bool ok = j >= 0 && j < D && in_disk(j, i, D);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    bc[r][c] = (fin && ok) ? ld_sh(Bf + c * DD + j * D + i) : 0.f;
                    yc[r][c] = (sta && ok) ? Yrec[c * DD + j * D + i] : 0.f;
                }
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = j0 + r;
                const bool okl = j < D && i > 0 && in_disk(j, i - 1, D);
                const bool okr = j < D && i + 1 < D && in_disk(j, i + 1, D);
                const bool okc = j < D && in_disk(j, i, D);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int cell = c * DD + j * D + i;
                    bl[r][c] = (fin && okl) ? ld_sh(Bf + cell - 1) : 0.f;
                    br[r][c] = (fin && okr) ? ld_sh(Bf + cell + 1) : 0.f;
                    yl[r][c] = (sta && okl) ? Yrec[cell - 1] : 0.f;
                    yr[r][c] = (sta && okr) ? Yrec[cell + 1] : 0.f;
                    ax[r][c] = (fin && okc) ? d.aux[cell] : 0.f;
                    ac[r][c] = (fin && okc) ? gbl(d.acc)[cell] : 0.f;
                    hf[r][c] = (fin && okc) ? Hfin[cell] : 0.f;
                    hs[r][c] = (sta && okc) ? Hrec[cell] : 0.f;
                    yb0[r][c] = (sta && okc) ? ld_sh(m + cell) : 0.f;
                }
            }
            const float2 hz2 = BUF(2, uu)[padb(i)];
            float nxt[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = j0 + r;
                if (j >= D) break;
                const int cell = j * D + i;
                if (!in_disk(j, i, D)) {
                    if (sta) {
                        st_sh(Bs + cell, 0.f);
                        st_sh(Bs + DD + cell, 0.f);
                        st_sh(Bs + 2 * DD + cell, 0.f);
                    }
                    continue;
                }
                float yprev[3] = {0.f, 0.f, 0.f};
                float ybar[3] = {yb0[r][0], yb0[r][1], yb0[r][2]};
                if (fin) {
                    const float2 kxy = BUF(r, uu)[padb(i)];
                    const float Kb[3] = {kxy.x, kxy.y, r == 0 ? hz2.x : hz2.y};
                    float accn[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float ex = bc[r][c] + bc[r + 2][c] + bl[r][c] + br[r][c];
                        yprev[c] = ax[r][c] + ex + cf * Kb[c];
                        accn[c] = ac[r][c] + yprev[c];
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) e_dm += (double)bc[r + 1][c] * ((double)hh[c] + (double)hf[r][c]);
                    if (sf == 0) {  // step nf complete: yb_nf = accumulated cotangent
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            st_sh(m + c * DD + cell, accn[c]);
                            ybar[c] = accn[c];
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < 3; ++c) gbl(d.acc)[c * DD + cell] = accn[c];
                    }
                }
                if (sta) {
                    if (ss == 3) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) gbl(d.acc)[c * DD + cell] = ybar[c];
                    }
                    const float w = (ss == 3 || ss == 0) ? dt * (1.0f / 6.0f) : dt * (1.0f / 3.0f);
                    const float v = (ss == 3) ? 0.f : (ss == 2) ? dt : 0.5f * dt;
                    const float kx = w * ybar[0] + v * yprev[0];
                    const float ky = w * ybar[1] + v * yprev[1];
                    const float kz = w * ybar[2] + v * yprev[2];
                    const float Yx = yc[r + 1][0], Yy = yc[r + 1][1], Yz = yc[r + 1][2];
                    const float bx = (yc[r][0] + yc[r + 2][0] + yl[r][0] + yr[r][0]) + cf * (hsx + hs[r][0]);
                    const float by = (yc[r][1] + yc[r + 2][1] + yl[r][1] + yr[r][1]) + cf * (hsy + hs[r][1]);
                    const float bz = (yc[r][2] + yc[r + 2][2] + yl[r][2] + yr[r][2]) + cf * (hsz + hs[r][2]);
                    // Y x b
                    const float px = Yy * bz - Yz * by, py = Yz * bx - Yx * bz, pz = Yx * by - Yy * bx;
                    // kb x Y
                    const float qx = ky * Yz - kz * Yy, qy = kz * Yx - kx * Yz, qz = kx * Yy - ky * Yx;
                    // mdir = b x kb - alpha [ (Y x b) x kb + b x (kb x Y) ]
                    const float m1x = by * kz - bz * ky, m1y = bz * kx - bx * kz, m1z = bx * ky - by * kx;
                    const float m2x = py * kz - pz * ky, m2y = pz * kx - px * kz, m2z = px * ky - py * kx;
                    const float m3x = by * qz - bz * qy, m3y = bz * qx - bx * qz, m3z = bx * qy - by * qx;
                    d.aux[cell] = m1x - al * (m2x + m3x);
                    d.aux[DD + cell] = m1y - al * (m2y + m3y);
                    d.aux[2 * DD + cell] = m1z - al * (m2z + m3z);
                    // bbar = kb x Y - alpha (kb x Y) x Y
                    const float gx = qx - al * (qy * Yz - qz * Yy);
                    const float gy = qy - al * (qz * Yx - qx * Yz);
                    const float gz = qz - al * (qx * Yy - qy * Yx);
                    st_sh(Bs + cell, gx);
                    st_sh(Bs + DD + cell, gy);
                    st_sh(Bs + 2 * DD + cell, gz);
                    // alpha_bar += kb . ( -Y x (Y x b) )
                    const float tx = Yy * pz - Yz * py, ty = Yz * px - Yx * pz, tz = Yx * py - Yy * px;
                    e_ex += -((double)kx * tx + (double)ky * ty + (double)kz * tz);
                    nxt[r][0] = gx;
                    nxt[r][1] = gy;
                    nxt[r][2] = gz;
                }
            }
            if (sta) {
                BUF(0, uu)[padb(i)] = make_float2(nxt[0][0], nxt[0][1]);
                BUF(1, uu)[padb(i)] = make_float2(nxt[1][0], nxt[1][1]);
                BUF(2, uu)[padb(i)] = make_float2(nxt[0][2], nxt[1][2]);
            }
        }
        __syncthreads();
    };


    // ---- adjoint of the Heun (H2) step with the noise replayed
    // Backward stage k <-> step n = N-1-k/2, forward stage s = 1-k%2 (s = 1: the
    // corrector's field at the predictor m~, s = 0: the field at m_n).  With the
    // recorded stage state Y, its demag field H and g = b(Y) dtau + sigma w, the
    // increment Delta(Y, g) = Y x g - alpha Y x (Y x g) has, for a cotangent c,
    //   direct part  mdir = g x c - alpha [(Y x g) x c + g x (c x Y)]
    //   g cotangent  gbar = c x Y - alpha (c x Y) x Y
    //   Y cotangent  mdir + dtau (exchange(gbar) + c_d K gbar)     (K: demag, symmetric)
    //   alpha_bar += c . (-Y x (Y x g)) + dsigma/dalpha gbar . w,   c_bar += dtau gbar . (h + H).
    // Step n: y = m_n + (Delta_1 + Delta_2)/2, m~ = m_n + Delta_1, m_{n+1} = y or y/|y|:
    //   ybar from m_{n+1}bar (through the normalisation), c_2 = ybar/2,
    //   m~bar = Y_2 cotangent, c_1 = m~bar + ybar/2, m_n bar = ybar + m~bar + Y_1 cotangent.
    // acc carries ybar (after s = 1 starts) and ybar + m~bar (after s = 0 starts);
    // aux carries mdir of the started stage; ya / yb carry gbar for its field.
    auto heun_vjp_update = [&](int b, long long k, long long K) {
        const long long N = a.nsteps;
        const bool fin = k > 0, sta = k < K;
        const long long nf = fin ? N - 1 - (k - 1) / 2 : 0, ns = sta ? N - 1 - k / 2 : 0;
        const int sf = fin ? 1 - (int)((k - 1) % 2) : 0, ss = sta ? 1 - (int)(k % 2) : 0;
        const float* Bf = ((k - 1) & 1) ? d.yb : d.ya;      // gbar of the finishing stage
        float* Bs = (k & 1) ? d.yb : d.ya;                  // gbar of the starting stage
        const GLOBAL_AS float* Yrec = gbl(recd) + ((size_t)(ns * 2 + ss) * 2) * 3 * DD;
        const GLOBAL_AS float* Hrec = Yrec + 3 * DD;
        const GLOBAL_AS float* Y0rec = gbl(recd) + ((size_t)(ns * 2) * 2) * 3 * DD;      // m_ns (stage 1 state)
        const GLOBAL_AS float* Hfin = gbl(recd) + ((size_t)(nf * 2 + sf) * 2 + 1) * 3 * DD;
        const float sg = pr.sigma, dsg = pr.dsigma;
        const Field3 hF = hext_at(pr, pr.tau0 + ((double)nf + (double)sf) * pr.dtau_d);
        const Field3 hS = hext_at(pr, pr.tau0 + ((double)ns + (double)ss) * pr.dtau_d);
        const float hh[3] = {(float)hF.x, (float)hF.y, (float)hF.z};
        const float hsv[3] = {(float)hS.x, (float)hS.y, (float)hS.z};
        for (int idx = tid<OPQ>(); idx < U * D; idx += NT) {
            const int uu = idx / D, i = idx - uu * D;
            const int p = b * U + uu;
            if (p >= d.n_pairs) continue;
            const int j0 = 2 * p;
            float3 wn[2] = {make_float3(0.f, 0.f, 0.f), make_float3(0.f, 0.f, 0.f)};
            if (sta && sg != 0.f && (in_disk(j0, i, D) || (j0 + 1 < D && in_disk(j0 + 1, i, D))))
                thermal_normals_pair(a.seed, step0 + (unsigned long long)ns, (unsigned long long)(p * D + i),
                                     (unsigned long long)(a.replica0 + d.k), wn[0], wn[1]);
            const float2 hz2 = BUF(2, uu)[padb(i)];
            float nxt[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = j0 + r;
                if (j >= D) break;
                const int cell = j * D + i;
                if (!in_disk(j, i, D)) {
                    if (sta) {
                        st_sh(Bs + cell, 0.f);
                        st_sh(Bs + DD + cell, 0.f);
                        st_sh(Bs + 2 * DD + cell, 0.f);
                    }
                    continue;
                }
                const bool okl = i > 0 && in_disk(j, i - 1, D), okr = i + 1 < D && in_disk(j, i + 1, D);
                const bool oku = j > 0 && in_disk(j - 1, i, D), okd = j + 1 < D && in_disk(j + 1, i, D);
                // ---- finish the stage whose gbar field is in LDS (Kb) and in Bf (exchange)
                float fin_tot[3] = {0.f, 0.f, 0.f};
                if (fin) {
                    const float2 kxy = BUF(r, uu)[padb(i)];
                    const float Kb[3] = {kxy.x, kxy.y, r == 0 ? hz2.x : hz2.y};
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int o = c * DD + cell;
                        const float gc = ld_sh(Bf + o);
                        const float ex = (oku ? ld_sh(Bf + o - D) : 0.f) + (okd ? ld_sh(Bf + o + D) : 0.f) +
                                         (okl ? ld_sh(Bf + o - 1) : 0.f) + (okr ? ld_sh(Bf + o + 1) : 0.f);
                        fin_tot[c] = d.aux[o] + dt * (ex + cf * Kb[c]);
                        e_dm += (double)dt * (double)gc * ((double)hh[c] + (double)Hfin[o]);
                    }
                }
                float ybar[3] = {0.f, 0.f, 0.f};     // cotangent of y (start of s = 1) or acc (s = 0)
                if (fin && sf == 0) {                // step nf complete: m_nf bar
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float v = gbl(d.acc)[c * DD + cell] + fin_tot[c];
                        st_sh(m + c * DD + cell, v);
                        ybar[c] = v;
                    }
                }
                if (!sta) continue;
                // ---- start stage (ns, ss)
                float Yv[3], bv[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int o = c * DD + cell;
                    Yv[c] = Yrec[o];
                    const float ex = (oku ? Yrec[o - D] : 0.f) + (okd ? Yrec[o + D] : 0.f) +
                                     (okl ? Yrec[o - 1] : 0.f) + (okr ? Yrec[o + 1] : 0.f);
                    bv[c] = ex + cf * (hsv[c] + Hrec[o]);
                }
                const float w3[3] = {r == 0 ? wn[0].x : wn[1].x, r == 0 ? wn[0].y : wn[1].y,
                                     r == 0 ? wn[0].z : wn[1].z};
                const float gx = bv[0] * dt + sg * w3[0], gy = bv[1] * dt + sg * w3[1], gz = bv[2] * dt + sg * w3[2];
                const float Yx = Yv[0], Yy = Yv[1], Yz = Yv[2];
                // Y x g and Delta(Y, g)
                const float px = Yy * gz - Yz * gy, py = Yz * gx - Yx * gz, pz = Yx * gy - Yy * gx;
                const float tx = Yy * pz - Yz * py, ty = Yz * px - Yx * pz, tz = Yx * py - Yy * px;   // Y x (Y x g)
                float cx, cy, cz;
                if (ss == 1) {
                    float yb[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) yb[c] = (k == 0) ? ld_sh(m + c * DD + cell) : ybar[c];
                    if (pr.renorm) {
                        // y = (m_n + m~)/2 + Delta_2/2;  ybar = (I - u u^T) m_{n+1}bar / |y|
                        float y3[3];
                        const float D2[3] = {px - al * tx, py - al * ty, pz - al * tz};
#pragma unroll
                        for (int c = 0; c < 3; ++c) y3[c] = 0.5f * (Y0rec[c * DD + cell] + Yv[c]) + 0.5f * D2[c];
                        const float nrm = sqrtf(y3[0] * y3[0] + y3[1] * y3[1] + y3[2] * y3[2]);
                        const float inv = 1.0f / nrm;
                        const float ux = y3[0] * inv, uy = y3[1] * inv, uz = y3[2] * inv;
                        const float pu = yb[0] * ux + yb[1] * uy + yb[2] * uz;
                        yb[0] = (yb[0] - pu * ux) * inv;
                        yb[1] = (yb[1] - pu * uy) * inv;
                        yb[2] = (yb[2] - pu * uz) * inv;
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) gbl(d.acc)[c * DD + cell] = yb[c];
                    cx = 0.5f * yb[0];
                    cy = 0.5f * yb[1];
                    cz = 0.5f * yb[2];
                } else {
                    // fin_tot = m~bar; acc holds ybar
                    float yb[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        yb[c] = gbl(d.acc)[c * DD + cell];
                        gbl(d.acc)[c * DD + cell] = yb[c] + fin_tot[c];
                    }
                    cx = fin_tot[0] + 0.5f * yb[0];
                    cy = fin_tot[1] + 0.5f * yb[1];
                    cz = fin_tot[2] + 0.5f * yb[2];
                }
                // c x Y
                const float qx = cy * Yz - cz * Yy, qy = cz * Yx - cx * Yz, qz = cx * Yy - cy * Yx;
                // mdir = g x c - alpha [ (Y x g) x c + g x (c x Y) ]
                const float m1x = gy * cz - gz * cy, m1y = gz * cx - gx * cz, m1z = gx * cy - gy * cx;
                const float m2x = py * cz - pz * cy, m2y = pz * cx - px * cz, m2z = px * cy - py * cx;
                const float m3x = gy * qz - gz * qy, m3y = gz * qx - gx * qz, m3z = gx * qy - gy * qx;
                d.aux[cell] = m1x - al * (m2x + m3x);
                d.aux[DD + cell] = m1y - al * (m2y + m3y);
                d.aux[2 * DD + cell] = m1z - al * (m2z + m3z);
                // gbar = c x Y - alpha (c x Y) x Y
                const float bx = qx - al * (qy * Yz - qz * Yy);
                const float by = qy - al * (qz * Yx - qx * Yz);
                const float bz = qz - al * (qx * Yy - qy * Yx);
                st_sh(Bs + cell, bx);
                st_sh(Bs + DD + cell, by);
                st_sh(Bs + 2 * DD + cell, bz);
                e_ex += -((double)cx * tx + (double)cy * ty + (double)cz * tz) +
                        (double)dsg * ((double)bx * w3[0] + (double)by * w3[1] + (double)bz * w3[2]);
                nxt[r][0] = bx;
                nxt[r][1] = by;
                nxt[r][2] = bz;
            }
            if (sta) {
                BUF(0, uu)[padb(i)] = make_float2(nxt[0][0], nxt[0][1]);
                BUF(1, uu)[padb(i)] = make_float2(nxt[1][0], nxt[1][1]);
                BUF(2, uu)[padb(i)] = make_float2(nxt[0][2], nxt[1][2]);
            }
        }
        __syncthreads();
    };

    // ---- constrained alignment relaxation (one sweep per field evaluation)
    // cur -> nxt: m <- (b + b^lam + kappa m)/|...| with b^lam = 2 m_z (lam . (r - X)) z-hat.
    // Thread sums (float64): q[0] = max residual |m x (b + b^lam)| of cur, q[1..2] = C(cur),
    // q[3..4] = C(nxt), q[5..7] = Jacobian entries (xx, xy, yy) of C(nxt) in lam.
    double rq[8];
    auto relax_update = [&](int b, const float* cur, float* nxt, double lx, double ly, double Xc, double Yc) {
        const double half = (D - 1) / 2.0;
        const float kap = (float)a.kappa;
        for (int idx = tid<OPQ>(); idx < U * D; idx += NT) {
            const int uu = idx / D, i = idx - uu * D;
            const int p = b * U + uu;
            if (p >= d.n_pairs) continue;
            const int j0 = 2 * p;
            float col[4][3], lft[2][3], rgt[2][3];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 - 1 + r;
                const bool ok = j >= 0 && j < D && in_disk(j, i, D);
#pragma unroll
                for (int c = 0; c < 3; ++c) col[r][c] = ok ? ld_sh(cur + c * DD + j * D + i) : 0.f;
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = j0 + r;
                const bool okl = j < D && i > 0 && in_disk(j, i - 1, D);
                const bool okr = j < D && i + 1 < D && in_disk(j, i + 1, D);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int cell = c * DD + j * D + i;
                    lft[r][c] = okl ? ld_sh(cur + cell - 1) : 0.f;
                    rgt[r][c] = okr ? ld_sh(cur + cell + 1) : 0.f;
                }
            }
            const float2 hz2 = BUF(2, uu)[padb(i)];
            float nxt_v[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = j0 + r;
                if (j >= D) break;
                const int cell = j * D + i;
                if (in_disk(j, i, D)) {
                    const float2 hxy = BUF(r, uu)[padb(i)];
                    const float Hz = r == 0 ? hz2.x : hz2.y;
                    const float mx = col[r + 1][0], my = col[r + 1][1], mz = col[r + 1][2];
                    double dx = ((double)i - half) - Xc, dy = ((double)j - half) - Yc;
                    if (a.relax_cut2 > 0.0 && !(dx * dx + dy * dy < a.relax_cut2)) dx = dy = 0.0;
                    const float bl = (float)(2.0 * (double)mz * (lx * dx + ly * dy));
                    const float bx = (col[r][0] + col[r + 2][0] + lft[r][0] + rgt[r][0]) + cf * (hxf + hxy.x);
                    const float by = (col[r][1] + col[r + 2][1] + lft[r][1] + rgt[r][1]) + cf * (hyf + hxy.y);
                    const float bz = (col[r][2] + col[r + 2][2] + lft[r][2] + rgt[r][2]) + cf * (hzf + Hz) + bl;
                    const float px = my * bz - mz * by, py = mz * bx - mx * bz, pz = mx * by - my * bx;
                    rq[0] = fmax(rq[0], (double)sqrtf(px * px + py * py + pz * pz));
                    const double w0 = (double)mz * (double)mz;
                    rq[1] += w0 * dx;
                    rq[2] += w0 * dy;
                    const float tx = bx + kap * mx, ty = by + kap * my, tz = bz + kap * mz;
                    const float tn = sqrtf(tx * tx + ty * ty + tz * tz);
                    const float inv = tn > 0.f ? 1.0f / tn : 0.f;
                    const float nx = tx * inv, ny = ty * inv, nz = tz * inv;
                    const double w1 = (double)nz * (double)nz;
                    rq[3] += w1 * dx;
                    rq[4] += w1 * dy;
                    const double gj = tn > 0.f ? 4.0 * w1 * (1.0 - w1) / (double)tn : 0.0;
                    rq[5] += gj * dx * dx;
                    rq[6] += gj * dx * dy;
                    rq[7] += gj * dy * dy;
                    nxt_v[r][0] = nx;
                    nxt_v[r][1] = ny;
                    nxt_v[r][2] = nz;
                }
                st_sh(nxt + cell, nxt_v[r][0]);
                st_sh(nxt + DD + cell, nxt_v[r][1]);
                st_sh(nxt + 2 * DD + cell, nxt_v[r][2]);
            }
            BUF(0, uu)[padb(i)] = make_float2(nxt_v[0][0], nxt_v[0][1]);
            BUF(1, uu)[padb(i)] = make_float2(nxt_v[1][0], nxt_v[1][1]);
            BUF(2, uu)[padb(i)] = make_float2(nxt_v[0][2], nxt_v[1][2]);
        }
        __syncthreads();
    };

    auto write_partials = [&](double s0v, double s1v, double s2v) {
        __shared__ double red[3 * MAX_UG][3];
        const double s0 = wave_sum(s0v), s1 = wave_sum(s1v), s2 = wave_sum(s2v);
        if (lane == 0) {
            red[wv][0] = s0;
            red[wv][1] = s1;
            red[wv][2] = s2;
        }
        __syncthreads();
        if (tid<OPQ>() < 3) {
            const int q = tid<OPQ>();
            double acc = 0.0;
            for (int w = 0; w < 3 * UG; ++w) acc += red[w][q];
            gbl(d.part)[g * PART_STRIDE + q] = acc;
        }
    };

    // ---------------------------------------------------------------- program
    if constexpr (MODE == MODE_RELAX) {
        for (int b = g; b < n_rb; b += G) {
            load_state_rows(b, m);
            row_forward_store(b);
        }
        if (!group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;
        const double Xc = a.relax_x[2 * d.k], Yc = a.relax_x[2 * d.k + 1];
        double lx = 0.0, ly = 0.0, res = 0.0, Cx = 0.0, Cy = 0.0;
        long long sweep = 0;
        float* cur = m;
        float* nxt = d.ya;
        __shared__ double red8[3 * MAX_UG][8];
        for (; sweep < a.nsteps; ++sweep) {
            column_pass();
            if (!group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;
            for (int q = 0; q < 8; ++q) rq[q] = 0.0;
            for (int b = g; b < n_rb; b += G) {
                row_inverse(b);
                relax_update(b, cur, nxt, lx, ly, Xc, Yc);
                row_forward_store(b);
            }
            // workgroup partials: max for the residual, sums for the rest
            {
                const double v0 = wave_max(rq[0]);
                double vs[7];
#pragma unroll
                for (int q = 1; q < 8; ++q) vs[q - 1] = wave_sum(rq[q]);
                if (lane == 0) {
                    red8[wv][0] = v0;
                    for (int q = 1; q < 8; ++q) red8[wv][q] = vs[q - 1];
                }
                __syncthreads();
                if (tid<OPQ>() < 8) {
                    const int q = tid<OPQ>();
                    double acc = 0.0;
                    for (int w = 0; w < 3 * UG; ++w) acc = (q == 0) ? fmax(acc, red8[w][q]) : acc + red8[w][q];
                    st_shd(d.part + g * PART_STRIDE + q, acc);
                }
            }
            if (!group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;
            // every workgroup of the disk reduces the same partials in the same order
            double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int gg = 0; gg < G; ++gg)
                for (int q = 0; q < 8; ++q) {
                    const double v = ld_shd(d.part + gg * PART_STRIDE + q);
                    t[q] = (q == 0) ? fmax(t[q], v) : t[q] + v;
                }
            res = t[0];
            Cx = t[1];
            Cy = t[2];
            if (res < a.tol && fabs(Cx) < a.tol && fabs(Cy) < a.tol) break;   // cur has converged
            const double jxx = t[5], jxy = t[6], jyy = t[7];
            const double det = jxx * jyy - jxy * jxy;
            if (det != 0.0) {
                lx -= (jyy * t[3] - jxy * t[4]) / det;
                ly -= (jxx * t[4] - jxy * t[3]) / det;
            }
            float* tmp = cur;
            cur = nxt;
            nxt = tmp;
        }
        // the result lives in cur; bring it back to m
        if (cur != m) {
            for (int b = g; b < n_rb; b += G)
                for (int idx = tid<OPQ>(); idx < U * D; idx += NT) {
                    const int uu = idx / D, i = idx - uu * D;
                    const int p = b * U + uu;
                    if (p >= d.n_pairs) continue;
                    for (int r = 0; r < 2; ++r) {
                        const int j = 2 * p + r;
                        if (j >= D) break;
                        for (int c = 0; c < 3; ++c) st_sh(m + c * DD + j * D + i, ld_sh(cur + c * DD + j * D + i));
                    }
                }
        }
        if (g == 0 && tid<OPQ>() == 0) {
            GLOBAL_AS double* o = gbl(a.relax_out) + 8 * d.k;
            o[0] = lx;
            o[1] = ly;
            o[2] = (double)sweep;
            o[3] = res;
            o[4] = Cx;
            o[5] = Cy;
            o[6] = 0.0;
            o[7] = 0.0;
        }
        return;
    } else if constexpr (MODE == MODE_RK4_VJP || MODE == MODE_HEUN_VJP) {
        const long long K = NST * a.nsteps;
        for (long long k = 0; k <= K; ++k) {
            for (int b = g; b < n_rb; b += G) {
                if (k > 0) row_inverse(b);
                if constexpr (MODE == MODE_RK4_VJP)
                    vjp_update(b, k, K);
                else
                    heun_vjp_update(b, k, K);
                if (k < K) row_forward_store(b);
            }
            if (k == K) break;
            if (!group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;
            column_pass();
            if (!group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;
        }
        write_partials(e_ex, e_dm, 0.0);
        return;
    } else {
        // field evaluation and integrators: the row spectra of the input state first
        for (int b = g; b < n_rb; b += G) {
            load_state_rows(b, m);
            row_forward_store(b);
        }
        if (!group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;

        // one row iteration of a field evaluation: issue every load, then stage, transform and update
        auto row_step = [&](int b, int s, long long n, const float* Ys, float* Yn) {
            float hv[IH];
            SRow sv[IS];
            halo_load(b, Ys, hv, true);
            gather(b, s);
            row_load(b, sv);
            halo_store(hv);
            row_unpack_inverse(sv);
            cell_update(b, s, n, Yn);
        };

        // all row iterations of a stage: the staged rows and row spectra of the
        // next iteration are loaded after the cell update of the current one, so
        // that they are in flight during its forward transforms and stores (at
        // P = 512 the staged rows are loaded before the cell update, so that
        // fewer loads queue behind its state stores); the start state and
        // accumulator are loaded at the top of the iteration
        // (iterations touch disjoint rows of the spectra and of the states they
        // write; a load past the last iteration reads zeros or unused rows)
        auto row_pass = [&](int s, long long n, const float* Ys, float* Yn, bool fwd, bool sample) {
            if (g >= n_rb) return;
            // the caller's state is read at the first stage of the launch only
            const bool masked = n == 0 && s == 0;
            float hv[IH];
            SRow sv[IS];
            halo_load(g, Ys, hv, masked);
            row_load(g, sv);
            for (int b = g; b < n_rb; b += G) {
                gather(b, s);
                halo_store(hv);
                row_unpack_inverse(sv);
                if constexpr (SERIES)
                    if (sample) sample_pass(b);
                if constexpr (P == 512) halo_load(b + G, Ys, hv, masked);
                cell_update(b, s, n, Yn);
                if constexpr (P != 512) halo_load(b + G, Ys, hv, masked);
                row_load(b + G, sv);
                if (fwd) row_forward_store(b);
            }
        };

        if constexpr (MODE == MODE_DEMAG) {
            column_pass();
            if (!group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;
            for (int b = g; b < n_rb; b += G) row_step(b, 0, 0, m, nullptr);
            if (mode == MODE_ENERGY) write_partials(e_ex, e_dm, e_ext);
        } else {
            constexpr int nst = (MODE == MODE_RK4) ? 4 : 2;
            for (long long n = 0; n < a.nsteps; ++n) {
                for (int s = 0; s < nst; ++s) {
                    column_pass();
                    if (!group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;
                    set_field(pr.tau0 + ((double)n + stage_frac(nst, s)) * pr.dtau_d);
                    const bool last = (n == a.nsteps - 1) && (s == nst - 1);
                    // state whose field is evaluated (Ys) and where the next stage state goes (Yn)
                    const float* Ys;
                    float* Yn;
                    if (nst == 4) {
                        Ys = (s == 0) ? m : (s == 2) ? d.yb : d.ya;
                        Yn = (s == 3) ? m : (s == 1) ? d.yb : d.ya;
                    } else {
                        Ys = (s == 0) ? m : d.ya;
                        Yn = (s == 0) ? d.ya : m;
                    }
                    const bool sampled = SERIES && s == 0 && n % a.every == 0;
                    if (sampled) {
                        if (tid<OPQ>() < 3 * UG * 4) red4[tid<OPQ>() >> 2][tid<OPQ>() & 3] = 0.0;
                        __syncthreads();
                    }
                    row_pass(s, n, Ys, Yn, !last, sampled);
                    if (sampled) {   // this workgroup's sums of the sample into its partial slots 4..7
                        __syncthreads();
                        if (tid<OPQ>() < 4) {
                            const int q = tid<OPQ>();
                            double acc = 0.0;
                            for (int w = 0; w < 3 * UG; ++w) acc += red4[w][q];
                            st_shd(d.part + g * PART_STRIDE + 4 + q, acc);
                        }
                    }
                    if (!last && !group_barrier(d.bar, ++epoch * G, G, a.err, a.spin_limit)) return;
                    // stage 0 is never the last stage: every workgroup's partials of a
                    // sample are visible here; workgroup 0 sums them in workgroup order
                    if (sampled && g == 0 && tid<OPQ>() < 4) {
                        const int q = tid<OPQ>();
                        double acc = 0.0;
                        for (int gg = 0; gg < G; ++gg) acc += ld_shd(d.part + gg * PART_STRIDE + 4 + q);
                        const long long smp = n / a.every;
                        gbl(a.series)[(smp * a.n_disks + d.k) * 4 + q] = q < 3 ? acc / (double)d.n_cells : acc;
                    }
                }
            }
        }
    }
#undef BUF
}

// Transform policy (the tuner picks one per handle): bit 0 selects the radix
// of the LDS transforms (0: radix 4, except radix 8 at P = 512 where 64 lanes
// must carry 512 points; 1: radix 8 for every size); bit 1 selects the column
// strategy (0: one wavefront per component, 1: one lane group per column with
// all three components).  The adjoint and relaxation kernels always use the
// first column strategy.
template <int P, int POL>
struct Radix {
    static constexpr int value = ((POL & 1) == 1 || P == 512) ? 8 : 4;
};
constexpr bool column_slots(int POL, int MODE) {
    return (POL & 2) != 0 && MODE != MODE_RK4_VJP && MODE != MODE_HEUN_VJP && MODE != MODE_RELAX;
}

// One persistent kernel per (workgroup shape UG, transform policy POL, mode,
// largest FFT size PMAX of the handle, observable series SER): each instance
// carries only the code and registers of its own path.  MODE_DEMAG stands for
// the field kernel (demag, rhs and energy, chosen at run time).
template <int UG, int POL>
constexpr int halo_floats(int PMAX) {
    int n = RowTile<64, Radix<64, POL>::value, UG>::floats;
    n = n > RowTile<128, Radix<128, POL>::value, UG>::floats ? n : RowTile<128, Radix<128, POL>::value, UG>::floats;
    n = n > RowTile<256, Radix<256, POL>::value, UG>::floats ? n : RowTile<256, Radix<256, POL>::value, UG>::floats;
    if (PMAX >= 512)
        n = n > RowTile<512, Radix<512, POL>::value, UG>::floats ? n : RowTile<512, Radix<512, POL>::value, UG>::floats;
    return n;
}

// The integrators keep three wavefronts per SIMD resident (the register
// budget the compiler must meet); the other modes take what they need.
constexpr int min_waves_per_simd(int mode) { return (mode == MODE_RK4 || mode == MODE_HEUN) ? 3 : 1; }

template <int UG, int POL, int MODE, int PMAX, bool SER>
__global__ __launch_bounds__(WG_THREADS* UG) __attribute__((amdgpu_waves_per_eu(min_waves_per_simd(MODE))))
void llg_persistent(KArgs a) {
    __shared__ float2 lds[LDS_FFT * UG];
    __shared__ float2 ltw[MAX_P];
    __shared__ float halo[halo_floats<UG, POL>(PMAX)];
    extern __shared__ float4 sdyn4[];   // on-chip spectra (launch-time size; empty when no disk is on chip)
    float2* const sdyn = reinterpret_cast<float2*>(sdyn4);
    const int wg = blockIdx.x;
    const int di = a.wg2disk[wg];
    if (di < 0) return;
    const int g = a.wg2local[wg];
    const DiskDesc d = a.disks[di];
    const DiskPrm pr = a.prm[di];
    constexpr bool L = PMAX >= 512, SL = column_slots(POL, MODE);
    constexpr bool OC = on_chip_instance(MODE, UG);
    switch (d.P) {
        case 64:
            if (OC && d.onchip)
                run_disk<64, Radix<64, POL>::value, UG, MODE, L, SL, SER, OC>(a, d, pr, g, lds, ltw, halo, sdyn);
            else
                run_disk<64, Radix<64, POL>::value, UG, MODE, L, SL, SER, false>(a, d, pr, g, lds, ltw, halo, sdyn);
            break;
        case 128:
            if (OC && d.onchip)
                run_disk<128, Radix<128, POL>::value, UG, MODE, L, SL, SER, OC>(a, d, pr, g, lds, ltw, halo, sdyn);
            else
                run_disk<128, Radix<128, POL>::value, UG, MODE, L, SL, SER, false>(a, d, pr, g, lds, ltw, halo, sdyn);
            break;
        case 256:
            run_disk<256, Radix<256, POL>::value, UG, MODE, L, SL, SER, false>(a, d, pr, g, lds, ltw, halo, sdyn);
            break;
        case 512:
            if constexpr (PMAX >= 512)
                run_disk<512, Radix<512, POL>::value, UG, MODE, L, SL, SER, false>(a, d, pr, g, lds, ltw, halo, sdyn);
            break;
        default: break;
    }
}

// Kernel pointer of the instance for (UG, POL, PMAX) of one mode; modes without
// the lane-group column strategy share the instances of policies 0 and 1.
template <int MODE, bool SER = false>
const void* persistent_instance(int UG, int POL, int PMAX) {
#define LLG_INST(ug, pl, pm)                                   \
    if (UG == ug && POL == pl && PMAX == pm)                   \
        return reinterpret_cast<const void*>(llg_persistent<ug, pl, MODE, pm, SER>);
    if (!column_slots(POL, MODE)) POL &= 1;
    LLG_INST(1, 0, 256) LLG_INST(2, 0, 256) LLG_INST(4, 0, 256)
    LLG_INST(1, 1, 256) LLG_INST(2, 1, 256) LLG_INST(4, 1, 256)
    LLG_INST(1, 0, 512) LLG_INST(2, 0, 512) LLG_INST(4, 0, 512)
    LLG_INST(1, 1, 512) LLG_INST(2, 1, 512) LLG_INST(4, 1, 512)
    if constexpr (column_slots(2, MODE)) {
        LLG_INST(1, 2, 256) LLG_INST(2, 2, 256) LLG_INST(4, 2, 256)
        LLG_INST(1, 3, 256) LLG_INST(2, 3, 256) LLG_INST(4, 3, 256)
        LLG_INST(1, 2, 512) LLG_INST(2, 2, 512) LLG_INST(4, 2, 512)
        LLG_INST(1, 3, 512) LLG_INST(2, 3, 512) LLG_INST(4, 3, 512)
    }
#undef LLG_INST
    return nullptr;
}

}  // namespace llg
