// Dense K x K block (K = D^k) on k adjacent qudits: psi[h, :, l] <- B psi[h, :, l]
// with the register viewed as [H][K][L].  This is a batched complex GEMM
// C[K x F] = B[K x K] X[K x F] over the F = H * L fibres.
//
// A workgroup owns a tile of NT fibres: it stages X[:, tile] in LDS (reads
// complete before any write, so the update is in place), then writes
// B X[:, tile] straight back to HBM.
#include "qf_internal.h"

namespace qf {
namespace {

constexpr int kBlock = 256;

struct FusedGeom {
    uint32_t K;       // block size D^k
    uint32_t L;       // stride of the block's last qudit
    uint32_t nfib;    // H * L
    uint32_t NT;      // fibres per tile
    FastDiv divL;
    FastDiv divK;
    FastDiv divNT;
};

__device__ inline uint32_t fibre_base(const FusedGeom& g, uint32_t f) {
    const uint32_t h = g.divL.div(f);
    const uint32_t l = f - h * g.L;
    return h * g.K * g.L + l;
}

// Stage X[:, tile] into LDS as xs[b * NT + i].
template <typename T>
__device__ inline void load_tile(const cplx<T>* __restrict__ psi, const FusedGeom& g, uint32_t f0,
                                 uint32_t nt, cplx<T>* xs) {
    const uint32_t cnt = g.K * nt;
    if (g.L == 1) {
        // the tile is nt whole fibres of K contiguous amplitudes
        const uint32_t base = f0 * g.K;
        for (uint32_t e = threadIdx.x; e < cnt; e += kBlock) {
            const uint32_t i = g.divK.div(e);
            const uint32_t b = e - i * g.K;
            xs[b * g.NT + i] = psi[base + e];
        }
    } else {
        // consecutive lanes take consecutive fibres (consecutive l when L >= NT)
        const uint32_t cnt_full = g.K * g.NT;
        for (uint32_t e = threadIdx.x; e < cnt_full; e += kBlock) {
            const uint32_t b = g.divNT.div(e);
            const uint32_t i = e - b * g.NT;
            if (i < nt) xs[b * g.NT + i] = psi[fibre_base(g, f0 + i) + b * g.L];
        }
    }
}

// VALU path: lane (i, r) accumulates rows a = r, r + RG, ... for fibre i.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fused_valu(cplx<T>* __restrict__ psi,
                                                       const cplx<T>* __restrict__ B, FusedGeom g) {
    extern __shared__ unsigned char smem[];
    cplx<T>* xs = reinterpret_cast<cplx<T>*>(smem);
    const uint32_t f0 = blockIdx.x * g.NT;
    const uint32_t nt = min(g.NT, g.nfib - f0);
    load_tile(psi, g, f0, nt, xs);
    __syncthreads();
    const uint32_t i = threadIdx.x % g.NT;
    const uint32_t rg = kBlock / g.NT;
    const uint32_t r0 = threadIdx.x / g.NT;
    if (i >= nt) return;
    const uint32_t base = fibre_base(g, f0 + i);
    constexpr int RA = 4;
    for (uint32_t a0 = r0; a0 < g.K; a0 += rg * RA) {
        cplx<T> acc[RA];
#pragma unroll
        for (int r = 0; r < RA; ++r) acc[r] = cmake<T>(0, 0);
        for (uint32_t b = 0; b < g.K; ++b) {
            const cplx<T> x = xs[b * g.NT + i];
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const uint32_t a = a0 + r * rg;
                if (a < g.K) cmac(acc[r], B[a * g.K + b], x);
            }
        }
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const uint32_t a = a0 + r * rg;
            if (a < g.K) psi[base + a * g.L] = acc[r];
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 matrix-core path (complex64, K >= 32).  Y = B X with
//   Y_re = B_re X_re - B_im X_im,  Y_im = B_re X_im + B_im X_re
// on v_mfma_f32_16x16x4f32 (A: 16 x 4, B: 4 x 16, C: 16 x 16).  Lane l of a
// wavefront supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// C[4 (l / 16) + r][l % 16] in accumulator register r.
//
// A workgroup owns NTM = 64 fibres.  X is staged in LDS as separate real and
// imaginary planes of Kp = ceil16(K) rows (rows >= K are zero), each row padded
// to 68 floats so that the four rows a wavefront reads per step fall in
// different banks.  B fragments are read from global memory (the K x K block
// stays in L2).  Wave w computes row blocks w, w + 4, ... against all four
// 16-fibre column blocks.  A real B (every imaginary part zero) skips the two
// products with B_im.
// ---------------------------------------------------------------------------

constexpr int NTM = 64;
constexpr int RS = NTM + 4;  // LDS row stride (floats)

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_fused_mfma(cplx<float>* __restrict__ psi,
                                                       const cplx<float>* __restrict__ B, FusedGeom g,
                                                       uint32_t Kp, int real) {
    extern __shared__ unsigned char smem[];
    float* xr = reinterpret_cast<float*>(smem);
    float* xi = xr + size_t(Kp) * RS;
    const uint32_t f0 = blockIdx.x * NTM;
    const uint32_t nt = min(uint32_t(NTM), g.nfib - f0);
    // stage X (zero rows >= K and columns >= nt)
    for (uint32_t e = threadIdx.x; e < Kp * NTM; e += kBlock) {
        const uint32_t b = e / NTM;
        const uint32_t i = e - b * NTM;
        cplx<float> v = cmake<float>(0.f, 0.f);
        if (b < g.K && i < nt) v = psi[fibre_base(g, f0 + i) + b * g.L];
        xr[b * RS + i] = v.re;
        xi[b * RS + i] = v.im;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15;  // A row / B column / C column inside a block
    const int lk = lane >> 4;  // A column / B row inside a k step; C row group
    const uint32_t nrb = Kp / 16;
    for (uint32_t rb = wave; rb < nrb; rb += kBlock / 64) {
        f32x4 cr[4], ci[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            cr[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            ci[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        const uint32_t arow = rb * 16 + lr;
        for (uint32_t k0 = 0; k0 < Kp; k0 += 4) {
            const uint32_t acol = k0 + lk;
            cplx<float> a = cmake<float>(0.f, 0.f);
            if (arow < g.K && acol < g.K) a = B[arow * g.K + acol];
            const float* xrr = xr + (k0 + lk) * RS + lr;
            const float* xir = xi + (k0 + lk) * RS + lr;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float br = xrr[j * 16];
                const float bi = xir[j * 16];
                cr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, br, cr[j], 0, 0, 0);
                ci[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, bi, ci[j], 0, 0, 0);
                if (!real) {
                    cr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.im, bi, cr[j], 0, 0, 0);
                    ci[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.im, br, ci[j], 0, 0, 0);
                }
            }
        }
        // write back rows rb*16 + 4*lk + r of the four column blocks
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t col = uint32_t(j * 16 + lr);
            if (col >= nt) continue;
            const uint32_t base = fibre_base(g, f0 + col);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t row = rb * 16 + uint32_t(4 * lk + r);
                if (row < g.K) psi[base + row * g.L] = cmake<float>(cr[j][r], ci[j][r]);
            }
        }
    }
}

// Persistent variant for Kp = 16 * NRB <= 128: wave w owns row blocks w and
// w + 4 and keeps their B fragments for every k step in registers, then loops
// over fibre tiles (grid-stride), so B is read once per workgroup.
// Template: NJ column blocks of 16 fibres per tile (NT = 16 NJ fibres; fewer
// make the LDS tile smaller, so more workgroups share a CU and one's staging
// overlaps another's products); REAL: the block's imaginary parts are zero,
// so their fragments are not held.
template <int NRB, int NJ, bool REAL>
__global__ __launch_bounds__(kBlock) void k_fused_mfma_regs(cplx<float>* __restrict__ psi,
                                                            const cplx<float>* __restrict__ B, FusedGeom g) {
    constexpr int Kp = 16 * NRB;
    constexpr int KS = Kp / 4;
    constexpr int RPW = (NRB + 3) / 4;  // row blocks per wave
    constexpr int NTR = 16 * NJ;        // fibres per tile
    constexpr int RSR = NTR + 4;        // LDS row stride (floats)
    typedef float fNJ __attribute__((ext_vector_type(NJ)));
    extern __shared__ unsigned char smem[];
    float* xr = reinterpret_cast<float*>(smem);
    float* xi = xr + size_t(Kp) * RSR;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15;
    const int lk = lane >> 4;
    float are[RPW][KS];
    float aim[REAL ? 1 : RPW][REAL ? 1 : KS];
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const uint32_t arow = uint32_t((wave + 4 * q) * 16 + lr);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const uint32_t acol = uint32_t(ks * 4 + lk);
            cplx<float> a = cmake<float>(0.f, 0.f);
            if (wave + 4 * q < NRB && arow < g.K && acol < g.K) a = B[arow * g.K + acol];
            are[q][ks] = a.re;
            if constexpr (!REAL) aim[q][ks] = a.im;
        }
    }
    const uint32_t ntiles = (g.nfib + NTR - 1) / NTR;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t f0 = tile * NTR;
        const uint32_t nt = min(uint32_t(NTR), g.nfib - f0);
        __syncthreads();
        // X[b][i] goes to position (i % 16) NJ + i / 16 of LDS row b, so that a
        // lane's NJ column blocks are one read
        if (g.L == 1) {
            // nt whole fibres of K contiguous amplitudes: consecutive lanes take
            // consecutive amplitudes
            const uint32_t cnt = g.K * nt;
            const cplx<float>* src = psi + size_t(f0) * g.K;
            for (uint32_t e = threadIdx.x; e < cnt; e += kBlock) {
                const uint32_t i = g.divK.div(e);
                const uint32_t b = e - i * g.K;
                const cplx<float> v = src[e];
                const uint32_t pos = b * RSR + (i & 15u) * NJ + (i >> 4);
                xr[pos] = v.re;
                xi[pos] = v.im;
            }
            // zero the padding: rows past K, columns past nt
            for (uint32_t e = threadIdx.x; e < uint32_t(Kp * NTR); e += kBlock) {
                const uint32_t b = e / NTR, i = e - b * NTR;
                if (b >= g.K || i >= nt) {
                    const uint32_t pos = b * RSR + (i & 15u) * NJ + (i >> 4);
                    xr[pos] = 0.f;
                    xi[pos] = 0.f;
                }
            }
        } else {
            // a lane keeps one fibre (its base computed once) and takes every
            // (kBlock / NT)-th row; consecutive lanes take consecutive fibres
            const uint32_t i = threadIdx.x & (NTR - 1);
            const bool have = i < nt;
            const uint32_t fb = have ? fibre_base(g, f0 + i) : 0u;
            const uint32_t col = (i & 15u) * NJ + (i >> 4);
            for (uint32_t b = threadIdx.x / NTR; b < uint32_t(Kp); b += kBlock / NTR) {
                cplx<float> v = cmake<float>(0.f, 0.f);
                if (have && b < g.K) v = psi[fb + b * g.L];
                xr[b * RSR + col] = v.re;
                xi[b * RSR + col] = v.im;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int rb = wave + 4 * q;
            if (rb >= NRB) continue;
            f32x4 cr[NJ], ci[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                cr[j] = f32x4{0.f, 0.f, 0.f, 0.f};
                ci[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const fNJ brv = *reinterpret_cast<const fNJ*>(xr + (ks * 4 + lk) * RSR + lr * NJ);
                const fNJ biv = *reinterpret_cast<const fNJ*>(xi + (ks * 4 + lk) * RSR + lr * NJ);
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const float br = brv[j];
                    const float bi = biv[j];
                    cr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(are[q][ks], br, cr[j], 0, 0, 0);
                    ci[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(are[q][ks], bi, ci[j], 0, 0, 0);
                    if constexpr (!REAL) {
                        cr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-aim[q][ks], bi, cr[j], 0, 0, 0);
                        ci[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[q][ks], br, ci[j], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const uint32_t col = uint32_t(j * 16 + lr);
                if (col >= nt) continue;
                const uint32_t base = fibre_base(g, f0 + col);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t row = uint32_t(rb * 16 + 4 * lk + r);
                    if (row < g.K) psi[base + row * g.L] = cmake<float>(cr[j][r], ci[j][r]);
                }
            }
        }
    }
}

template <int NRB, int NJ, bool REAL>
qf_status launch_mfma_regs(const StateView& s, const FusedGeom& g, const void* B, hipStream_t st) {
    constexpr int NTR = 16 * NJ;
    const size_t lds = size_t(2) * (16 * NRB) * (NTR + 4) * sizeof(float);
    const uint32_t ntiles = (g.nfib + NTR - 1) / NTR;
    const uint32_t grid = ntiles < 4096 ? ntiles : 4096;
    hipLaunchKernelGGL((k_fused_mfma_regs<NRB, NJ, REAL>), dim3(grid), dim3(kBlock), lds, st,
                       reinterpret_cast<cplx<float>*>(s.amps), reinterpret_cast<const cplx<float>*>(B), g);
    return check_launch("qf_apply_fused (matrix cores, persistent)");
}

// Real blocks: tiles of 32 fibres; complex blocks (twice the products per
// operand read): 16 (both measured best on the D = 10 and D = 7 pair blocks).
template <int NRB>
qf_status launch_mfma_regs_any(const StateView& s, const FusedGeom& g, const void* B, bool real, hipStream_t st) {
    return real ? launch_mfma_regs<NRB, 2, true>(s, g, B, st) : launch_mfma_regs<NRB, 1, false>(s, g, B, st);
}

}  // namespace

qf_status launch_fused(const StateView& s, int k, int q0, const void* B, hipStream_t st, bool real) {
    const uint32_t K = span(s, q0, k);
    FusedGeom g{};
    g.K = K;
    g.L = s.strides[q0 + k - 1];
    g.nfib = s.total / K;
    const size_t esz = s.dtype == QF_C64 ? 8 : 16;
    uint32_t nt = 64;
    while (nt > 1 && size_t(K) * nt * esz > 64 * 1024) nt >>= 1;
    g.NT = nt;
    g.divL.init(g.L);
    g.divK.init(K);
    g.divNT.init(nt);
    if (s.dtype == QF_C64 && K >= 32 && K <= 128) {
        switch ((K + 15) / 16) {
            case 2: return launch_mfma_regs_any<2>(s, g, B, real, st);
            case 3: return launch_mfma_regs_any<3>(s, g, B, real, st);
            case 4: return launch_mfma_regs_any<4>(s, g, B, real, st);
            case 5: return launch_mfma_regs_any<5>(s, g, B, real, st);
            case 6: return launch_mfma_regs_any<6>(s, g, B, real, st);
            case 7: return launch_mfma_regs_any<7>(s, g, B, real, st);
            case 8: return launch_mfma_regs_any<8>(s, g, B, real, st);
        }
    }
    if (s.dtype == QF_C64 && K >= 32 && K <= 256) {
        const uint32_t Kp = (K + 15) / 16 * 16;
        const size_t lds = size_t(2) * Kp * RS * sizeof(float);
        const uint32_t grid = (g.nfib + NTM - 1) / NTM;
        hipLaunchKernelGGL(k_fused_mfma, dim3(grid), dim3(kBlock), lds, st, reinterpret_cast<cplx<float>*>(s.amps),
                           reinterpret_cast<const cplx<float>*>(B), g, Kp, real ? 1 : 0);
        return check_launch("qf_apply_fused (matrix cores)");
    }
    const uint32_t grid = (g.nfib + nt - 1) / nt;
    const size_t lds = size_t(K) * nt * esz;
    if (s.dtype == QF_C64) {
        hipLaunchKernelGGL(k_fused_valu<float>, dim3(grid), dim3(kBlock), lds, st,
                           reinterpret_cast<cplx<float>*>(s.amps), reinterpret_cast<const cplx<float>*>(B), g);
    } else {
        hipLaunchKernelGGL(k_fused_valu<double>, dim3(grid), dim3(kBlock), lds, st,
                           reinterpret_cast<cplx<double>*>(s.amps), reinterpret_cast<const cplx<double>*>(B), g);
    }
    return check_launch("qf_apply_fused");
}

}  // namespace qf
