// Adjoint-method kernels.  For a one-qudit step U on axis q, one pass over the
// fibres of psi and lam (both taken just after U in the forward order):
//   * accumulates the D x D matrix M = sum_fibres psi_f lam_f^dagger in FP64
//     (every rotation folded into U gets its derivative from M on the host),
//   * un-applies U on both states: psi_f <- W psi_f, lam_f <- W lam_f with
//     W = U^dagger (passed in by the host).
// The reduction is deterministic: fixed per-workgroup tree, then a fixed-order
// sum over workgroups.
#include <type_traits>

#include "qf_internal.h"

namespace qf {
namespace {

constexpr int kFB = 128;  // fibres (= lanes) per workgroup

template <typename T, int D>
struct MatArgA {
    cplx<T> m[D * D];
};

template <typename T, int D>
__global__ __launch_bounds__(kFB) void k_adj_axis(cplx<T>* __restrict__ psi, cplx<T>* __restrict__ lam,
                                                  uint32_t nfib_reg, uint32_t blocks_per_reg, uint32_t N,
                                                  uint32_t L, FastDiv divL, MatArgA<T, D> W,
                                                  double* __restrict__ partial) {
    __shared__ cplx<T> sp[D][kFB];
    __shared__ cplx<T> sl[D][kFB];
    __shared__ double red[2][kFB];
    constexpr int E = D * D;
    const uint32_t b = blockIdx.x / blocks_per_reg;
    const uint32_t blk = blockIdx.x - b * blocks_per_reg;
    const uint32_t f = blk * kFB + threadIdx.x;
    const bool live = f < nfib_reg;
    cplx<T> vp[D], vl[D];
    if (live) {
        const uint32_t h = divL.div(f);
        const uint32_t l = f - h * L;
        const uint32_t base = b * N + h * (uint32_t(D) * L) + l;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            vp[d] = psi[base + uint32_t(d) * L];
            vl[d] = lam[base + uint32_t(d) * L];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            sp[d][threadIdx.x] = vp[d];
            sl[d][threadIdx.x] = vl[d];
        }
        cplx<T> wp[D], wl[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            wp[a] = cmake<T>(0, 0);
            wl[a] = cmake<T>(0, 0);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                cmac(wp[a], W.m[a * D + c], vp[c]);
                cmac(wl[a], W.m[a * D + c], vl[c]);
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            psi[base + uint32_t(d) * L] = wp[d];
            lam[base + uint32_t(d) * L] = wl[d];
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            sp[d][threadIdx.x] = cmake<T>(0, 0);
            sl[d][threadIdx.x] = cmake<T>(0, 0);
        }
    }
    __syncthreads();
    // M[a][c] = sum_i psi_i[a] conj(lam_i[c]); entry e = a*D + c.
    double* out = partial + size_t(blockIdx.x) * E * 2;
    if constexpr (E <= kFB) {
        constexpr int P = kFB / E;  // parts per entry
        const int e = threadIdx.x % E;
        const int part = threadIdx.x / E;
        double ar = 0.0, ai = 0.0;
        if (part < P) {
            const int a = e / D, c = e % D;
            for (int i = part; i < kFB; i += P) {
                const cplx<T> x = sp[a][i];
                const cplx<T> y = sl[c][i];
                ar += double(x.re) * double(y.re) + double(x.im) * double(y.im);
                ai += double(x.im) * double(y.re) - double(x.re) * double(y.im);
            }
        }
        red[0][threadIdx.x] = ar;
        red[1][threadIdx.x] = ai;
        __syncthreads();
        if (threadIdx.x < E) {
            double sr = 0.0, si = 0.0;
            for (int p = 0; p < P; ++p) {
                sr += red[0][p * E + threadIdx.x];
                si += red[1][p * E + threadIdx.x];
            }
            out[2 * threadIdx.x] = sr;
            out[2 * threadIdx.x + 1] = si;
        }
    } else {
        for (int e = threadIdx.x; e < E; e += kFB) {
            const int a = e / D, c = e % D;
            double ar = 0.0, ai = 0.0;
            for (int i = 0; i < kFB; ++i) {
                const cplx<T> x = sp[a][i];
                const cplx<T> y = sl[c][i];
                ar += double(x.re) * double(y.re) + double(x.im) * double(y.im);
                ai += double(x.im) * double(y.re) - double(x.re) * double(y.im);
            }
            out[2 * e] = ar;
            out[2 * e + 1] = ai;
        }
    }
}

// out[b][slot][e] = sum over the workgroups of register b: one workgroup per
// (b, e); lanes take workgroups k = lane, lane + 256, ..., then a fixed tree.
__global__ __launch_bounds__(256) void k_adj_reduce(const double* __restrict__ partial, uint32_t blocks_per_reg,
                                                    uint32_t E, uint32_t nslots, uint32_t slot, uint32_t slot_elems,
                                                    double* __restrict__ out) {
    __shared__ double sh[2][256];
    const uint32_t b = blockIdx.x / E;
    const uint32_t e = blockIdx.x - b * E;
    double sr = 0.0, si = 0.0;
    for (uint32_t k = threadIdx.x; k < blocks_per_reg; k += 256) {
        const double* p = partial + (size_t(b) * blocks_per_reg + k) * E * 2;
        sr += p[2 * e];
        si += p[2 * e + 1];
    }
    sh[0][threadIdx.x] = sr;
    sh[1][threadIdx.x] = si;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = out + ((size_t(b) * nslots + slot) * slot_elems + e) * 2;
        o[0] = sh[0][0];
        o[1] = sh[1][0];
    }
}

template <class F>
qf_status with_dim_a(uint32_t D, F&& f) {
    switch (D) {
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 6: return f(std::integral_constant<int, 6>{});
        case 7: return f(std::integral_constant<int, 7>{});
        case 8: return f(std::integral_constant<int, 8>{});
        case 9: return f(std::integral_constant<int, 9>{});
        case 10: return f(std::integral_constant<int, 10>{});
        case 11: return f(std::integral_constant<int, 11>{});
        case 12: return f(std::integral_constant<int, 12>{});
        case 13: return f(std::integral_constant<int, 13>{});
        case 14: return f(std::integral_constant<int, 14>{});
        case 15: return f(std::integral_constant<int, 15>{});
        case 16: return f(std::integral_constant<int, 16>{});
        default: return set_error(QF_EUNSUPPORTED, "dim %u outside 2..16", D);
    }
}

}  // namespace

size_t adj_axis_partial_doubles(const StateView& s) {
    const uint32_t nfib_reg = s.N / s.dmin;
    const uint32_t bpr = (nfib_reg + kFB - 1) / kFB;
    return size_t(bpr) * s.batch * s.dmax * s.dmax * 2;
}

qf_status launch_adj_axis(const StateView& s, void* lam, int q, const double* W, double* partial, double* mout,
                          uint32_t nslots, uint32_t slot, uint32_t slot_elems, hipStream_t st) {
    const uint32_t nfib_reg = s.N / s.dims[q];
    const uint32_t bpr = (nfib_reg + kFB - 1) / kFB;
    const uint32_t L = s.strides[q];
    auto body = [&](auto tag, auto dtag) -> qf_status {
        using T = decltype(tag);
        constexpr int D = decltype(dtag)::value;
        if constexpr (sizeof(MatArgA<T, D>) > 2048) {
            return set_error(QF_ERANGE, "dim %d too large for a complex128 adjoint matrix argument", D);
        } else {
            MatArgA<T, D> w;
            for (int i = 0; i < D * D; ++i) w.m[i] = cmake<T>(T(W[2 * i]), T(W[2 * i + 1]));
            hipLaunchKernelGGL((k_adj_axis<T, D>), dim3(bpr * s.batch), dim3(kFB), 0, st,
                               reinterpret_cast<cplx<T>*>(s.amps), reinterpret_cast<cplx<T>*>(lam), nfib_reg,
                               bpr, s.N, L, FastDiv(L), w, partial);
            QF_CHECK(check_launch("adjoint axis"));
            const uint32_t E = D * D;
            hipLaunchKernelGGL(k_adj_reduce, dim3(s.batch * E), dim3(256), 0, st, partial, bpr, E, nslots, slot,
                               slot_elems, mout);
            return check_launch("adjoint reduce");
        }
    };
    return with_dim_a(s.dims[q], [&](auto dtag) -> qf_status {
        if (s.dtype == QF_C64) return body(float{}, dtag);
        return body(double{}, dtag);
    });
}

}  // namespace qf
