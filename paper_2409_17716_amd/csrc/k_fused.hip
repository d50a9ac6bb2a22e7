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

}  // namespace

qf_status launch_fused(const StateView& s, int k, int q0, const void* B, hipStream_t st) {
    const uint32_t K = ipow(s.D, k);
    FusedGeom g{};
    g.K = K;
    g.L = ipow(s.D, s.n - q0 - k);
    g.nfib = s.total / K;
    const size_t esz = s.dtype == QF_C64 ? 8 : 16;
    uint32_t nt = 64;
    while (nt > 1 && size_t(K) * nt * esz > 64 * 1024) nt >>= 1;
    g.NT = nt;
    g.divL.init(g.L);
    g.divK.init(K);
    g.divNT.init(nt);
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
