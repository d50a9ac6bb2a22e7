// The differentiable controlled rotation sum_m |m><m|_c (x) R^{jk}_alpha(m theta)_t
// (arXiv:2409.17716, Appendix, subsection "Controlled Rotation Gate"), and
// without a control the plain two-level rotation as a slab sweep (the memory
// form of the paper's sparse rotation, subsection "Generalized rotation gate").
//
// The register is viewed as [H][D][L] for the target t (D = d_t, L = S_t, the
// product of the dimensions after t); a fibre is the D amplitudes
// psi[h, :, l], and its control digit m (0 <= m < d_c) is read from its index.  The x- and y-type rotations mix only target levels j and k, so a
// lane reads and writes just those two amplitudes of its fibre (2/D of the
// state); the z type scales levels 0..j.  Fibres at control level 0 are left
// alone.  Consecutive lanes take consecutive l, so for L >= 64 every access of
// a wavefront is one contiguous run.  The forward kernel gives each lane
// kFPL fibres, kCB apart, and issues all their loads before the first store:
// with one fibre a wavefront keeps only 1 KB of loads in flight when the two
// levels are contiguous slabs, too little to cover the HBM latency.
//
// Per control level m the kernels read a two-entry table: x, y types
// (cos(m theta / 2), sin(m theta / 2)) in one complex entry (the inverse
// negates the sine); z type the phase of levels below j and the phase of level
// j.  The adjoint kernel takes the inverse table, adds
//   m * Im <lam_f| S |psi_f>   (the slab generator is m S)
// over its fibres in FP64 (fixed tree per workgroup, then a fixed-order sum per
// register) and un-applies the gate on psi and lam.
#include <type_traits>

#include "qf_internal.h"

namespace qf {
namespace {

constexpr int kCB = 256;
constexpr int kFPL = 4;  // fibres per lane in the forward kernel

struct CrGeom {
    int32_t has_ctrl;    // 0: plain rotation, every fibre uses table entry 1
    uint32_t L;          // stride of the target qudit
    FastDiv divL;
    FastDiv cstride;     // stride of the control qudit
    FastDiv divDc;       // dimension of the control qudit
    uint32_t ntab;       // table entries: 2 per control level
    uint32_t nfib;       // fibres per register, N / d_t
    uint32_t N;          // amplitudes per register
    uint32_t bpr;        // workgroups per register (one fibre per lane: the adjoint)
    uint32_t bprf;       // workgroups per register of the forward kernel (kFPL fibres per lane)
    int32_t kind;        // 0 = x, 1 = y, 2 = z
    int32_t j, k;        // levels (z: j)
    double alpha;        // z: sqrt(2 / (j (j + 1)))
};

template <typename T>
struct CrTab {
    cplx<T> t[2 * kMaxDim];
};

template <typename T>
__device__ __forceinline__ void load_tab(const CrTab<T>& harg, const cplx<T>* __restrict__ dtab, size_t tab_stride,
                                         uint32_t b, uint32_t ntab, cplx<T>* tab) {
    if (threadIdx.x < ntab) tab[threadIdx.x] = dtab ? dtab[size_t(b) * tab_stride + threadIdx.x] : harg.t[threadIdx.x];
    __syncthreads();
}

__device__ __forceinline__ uint32_t ctrl_level(const CrGeom& g, uint32_t local) {
    if (!g.has_ctrl) return 1u;
    const uint32_t qv = g.cstride.div(local);
    return qv - g.divDc.div(qv) * g.divDc.d;
}

// The x- or y-type rotation of levels (j, k) with cs = (cos, sin) of half the
// angle, on the pair (a, b) = (psi_j, psi_k).
template <typename T>
__device__ __forceinline__ void rot_pair(int kind, cplx<T> cs, cplx<T>& a, cplx<T>& b) {
    const T c = cs.re, s = cs.im;
    const cplx<T> x = a, y = b;
    if (kind == 0) {  // [[c, -i s], [-i s, c]]
        a = cmake<T>(c * x.re + s * y.im, c * x.im - s * y.re);
        b = cmake<T>(c * y.re + s * x.im, c * y.im - s * x.re);
    } else {          // [[c, -s], [s, c]]
        a = cmake<T>(c * x.re - s * y.re, c * x.im - s * y.im);
        b = cmake<T>(s * x.re + c * y.re, s * x.im + c * y.im);
    }
}

// Applies the table's rotation for control level m to the fibre at base.
template <typename T, int D>
__device__ __forceinline__ void rotate(cplx<T>* __restrict__ psi, const CrGeom& g, uint32_t base, const cplx<T>* tab,
                                       uint32_t m) {
    if (g.kind == 2) {
        const cplx<T> p1 = tab[2 * m], p2 = tab[2 * m + 1];
        for (int d = 0; d < g.j; ++d) psi[base + uint32_t(d) * g.L] = cmul(psi[base + uint32_t(d) * g.L], p1);
        psi[base + uint32_t(g.j) * g.L] = cmul(psi[base + uint32_t(g.j) * g.L], p2);
        return;
    }
    const uint32_t ia = base + uint32_t(g.j) * g.L, ib = base + uint32_t(g.k) * g.L;
    cplx<T> a = psi[ia], b = psi[ib];
    rot_pair<T>(g.kind, tab[2 * m], a, b);
    psi[ia] = a;
    psi[ib] = b;
}

template <typename T, int D>
__global__ __launch_bounds__(kCB) void k_crot(cplx<T>* __restrict__ psi, CrGeom g, CrTab<T> harg,
                                              const cplx<T>* __restrict__ dtab, size_t tab_stride) {
    __shared__ cplx<T> tab[2 * kMaxDim];
    const uint32_t b = blockIdx.x / g.bprf;
    load_tab<T>(harg, dtab, tab_stride, b, g.ntab, tab);
    const uint32_t f0 = (blockIdx.x - b * g.bprf) * (kCB * kFPL) + threadIdx.x;
    cplx<T>* const p = psi + size_t(b) * g.N;
    uint32_t loc[kFPL], lev[kFPL];  // fibre base and control level (0: left alone)
#pragma unroll
    for (int i = 0; i < kFPL; ++i) {
        const uint32_t f = f0 + uint32_t(i) * kCB;
        loc[i] = 0;
        lev[i] = 0;
        if (f < g.nfib) {
            const uint32_t h = g.divL.div(f);
            loc[i] = h * (uint32_t(D) * g.L) + (f - h * g.L);
            lev[i] = ctrl_level(g, loc[i]);
        }
    }
    if (g.kind == 2) {
#pragma unroll
        for (int i = 0; i < kFPL; ++i)
            if (lev[i] != 0) rotate<T, D>(p, g, loc[i], tab, lev[i]);
        return;
    }
    const uint32_t oj = uint32_t(g.j) * g.L, ok = uint32_t(g.k) * g.L;
    cplx<T> va[kFPL], vb[kFPL];
#pragma unroll
    for (int i = 0; i < kFPL; ++i) {
        va[i] = cmake<T>(0, 0);
        vb[i] = cmake<T>(0, 0);
        if (lev[i] != 0) {
            va[i] = p[loc[i] + oj];
            vb[i] = p[loc[i] + ok];
        }
    }
#pragma unroll
    for (int i = 0; i < kFPL; ++i) {
        if (lev[i] == 0) continue;
        rot_pair<T>(g.kind, tab[2 * lev[i]], va[i], vb[i]);
        p[loc[i] + oj] = va[i];
        p[loc[i] + ok] = vb[i];
    }
}

// Deterministic workgroup sum (fixed tree).
__device__ inline double cr_block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kCB / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

template <typename T, int D>
__global__ __launch_bounds__(kCB) void k_crot_adj(cplx<T>* __restrict__ psi, cplx<T>* __restrict__ lam, CrGeom g,
                                                  CrTab<T> harg, const cplx<T>* __restrict__ dtab, size_t tab_stride,
                                                  double* __restrict__ partial) {
    __shared__ cplx<T> tab[2 * kMaxDim];
    __shared__ double sh[kCB];
    const uint32_t b = blockIdx.x / g.bpr;
    load_tab<T>(harg, dtab, tab_stride, b, g.ntab, tab);
    const uint32_t f = (blockIdx.x - b * g.bpr) * kCB + threadIdx.x;
    double acc = 0.0;
    if (f < g.nfib) {
        const uint32_t h = g.divL.div(f);
        const uint32_t local = h * (uint32_t(D) * g.L) + (f - h * g.L);
        const uint32_t m = ctrl_level(g, local);
        if (m != 0) {
            cplx<T>* p = psi + size_t(b) * g.N;
            cplx<T>* l = lam + size_t(b) * g.N;
            double im = 0.0;  // Im <lam_f| S |psi_f>
            if (g.kind == 2) {
                for (int d = 0; d <= g.j; ++d) {
                    const cplx<T> x = p[local + uint32_t(d) * g.L], y = l[local + uint32_t(d) * g.L];
                    const double w = d < g.j ? g.alpha : -g.alpha * g.j;
                    im += w * (double(y.re) * double(x.im) - double(y.im) * double(x.re));
                }
            } else {
                const uint32_t ia = local + uint32_t(g.j) * g.L, ib = local + uint32_t(g.k) * g.L;
                const cplx<T> pj = p[ia], pk = p[ib], lj = l[ia], lk = l[ib];
                // conj(lj) pk and conj(lk) pj
                const double r1 = double(lj.re) * pk.re + double(lj.im) * pk.im;
                const double i1 = double(lj.re) * pk.im - double(lj.im) * pk.re;
                const double r2 = double(lk.re) * pj.re + double(lk.im) * pj.im;
                const double i2 = double(lk.re) * pj.im - double(lk.im) * pj.re;
                im = g.kind == 0 ? i1 + i2 : r2 - r1;  // x: Im(z1 + z2); y: Im(-i z1 + i z2)
            }
            acc = double(m) * im;
            rotate<T, D>(p, g, local, tab, m);
            rotate<T, D>(l, g, local, tab, m);
        }
    }
    const double s = cr_block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[b * ostride] = sum of the bpr partials of register b (fixed order).
__global__ __launch_bounds__(kCB) void k_crot_reduce(const double* __restrict__ partial, uint32_t bpr,
                                                     double* __restrict__ out, uint32_t ostride) {
    __shared__ double sh[kCB];
    const uint32_t b = blockIdx.x;
    double s = 0.0;
    for (uint32_t i = threadIdx.x; i < bpr; i += kCB) s += partial[size_t(b) * bpr + i];
    s = cr_block_sum(s, sh);
    if (threadIdx.x == 0) out[size_t(b) * ostride] = s;
}

template <class F>
qf_status with_dim_c(uint32_t D, F&& f) {
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

CrGeom make_geom(const StateView& s, const CrotArgs& a) {
    CrGeom g{};
    g.has_ctrl = a.ctrl >= 0 ? 1 : 0;
    g.L = s.strides[a.tgt];
    g.divL.init(g.L);
    g.cstride.init(a.ctrl >= 0 ? s.strides[a.ctrl] : 1u);
    g.divDc.init(a.ctrl >= 0 ? s.dims[a.ctrl] : 2u);
    g.ntab = 2 * g.divDc.d;
    g.nfib = s.N / s.dims[a.tgt];
    g.N = s.N;
    g.bpr = (g.nfib + kCB - 1) / kCB;
    g.bprf = (g.nfib + kCB * kFPL - 1) / (kCB * kFPL);
    g.kind = a.kind;
    g.j = a.j;
    g.k = a.k;
    g.alpha = a.kind == 2 ? std::sqrt(2.0 / (double(a.j) * (a.j + 1))) : 0.0;
    return g;
}

template <typename T>
CrTab<T> host_tab(const double* htab, uint32_t ntab) {
    CrTab<T> t{};
    if (htab)
        for (uint32_t i = 0; i < ntab; ++i) t.t[i] = cmake<T>(T(htab[2 * i]), T(htab[2 * i + 1]));
    return t;
}

}  // namespace

size_t crot_partial_doubles(const StateView& s) {
    const uint32_t nfib = s.N / s.dmin;
    return size_t((nfib + kCB - 1) / kCB) * s.batch;
}

qf_status launch_crot(const StateView& s, const CrotArgs& a, const void* dtab, size_t tab_stride, const double* htab,
                      hipStream_t st) {
    const CrGeom g = make_geom(s, a);
    return with_dim_c(s.dims[a.tgt], [&](auto dtag) -> qf_status {
        constexpr int D = decltype(dtag)::value;
        if (s.dtype == QF_C64)
            hipLaunchKernelGGL((k_crot<float, D>), dim3(g.bprf * s.batch), dim3(kCB), 0, st,
                               reinterpret_cast<cplx<float>*>(s.amps), g, host_tab<float>(htab, g.ntab),
                               reinterpret_cast<const cplx<float>*>(dtab), tab_stride);
        else
            hipLaunchKernelGGL((k_crot<double, D>), dim3(g.bprf * s.batch), dim3(kCB), 0, st,
                               reinterpret_cast<cplx<double>*>(s.amps), g, host_tab<double>(htab, g.ntab),
                               reinterpret_cast<const cplx<double>*>(dtab), tab_stride);
        return check_launch("controlled rotation");
    });
}

qf_status launch_crot_adj(const StateView& s, void* lam, const CrotArgs& a, const void* dtab, size_t tab_stride,
                          const double* htab, double* partial, double* out, uint32_t ostride, hipStream_t st) {
    const CrGeom g = make_geom(s, a);
    return with_dim_c(s.dims[a.tgt], [&](auto dtag) -> qf_status {
        constexpr int D = decltype(dtag)::value;
        if (s.dtype == QF_C64)
            hipLaunchKernelGGL((k_crot_adj<float, D>), dim3(g.bpr * s.batch), dim3(kCB), 0, st,
                               reinterpret_cast<cplx<float>*>(s.amps), reinterpret_cast<cplx<float>*>(lam), g,
                               host_tab<float>(htab, g.ntab), reinterpret_cast<const cplx<float>*>(dtab), tab_stride,
                               partial);
        else
            hipLaunchKernelGGL((k_crot_adj<double, D>), dim3(g.bpr * s.batch), dim3(kCB), 0, st,
                               reinterpret_cast<cplx<double>*>(s.amps), reinterpret_cast<cplx<double>*>(lam), g,
                               host_tab<double>(htab, g.ntab), reinterpret_cast<const cplx<double>*>(dtab), tab_stride,
                               partial);
        QF_CHECK(check_launch("controlled rotation adjoint"));
        hipLaunchKernelGGL(k_crot_reduce, dim3(s.batch), dim3(kCB), 0, st, partial, g.bpr, out, ostride);
        return check_launch("controlled rotation gradient sum");
    });
}

}  // namespace qf
