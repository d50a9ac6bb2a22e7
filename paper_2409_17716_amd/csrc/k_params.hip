// Device-side parameter handling: fused gate matrices built from a device array
// of angles, and rotation gradients from the adjoint's M matrices.  Both run in
// FP64 (the same closed forms as the host builder) and need no host work, so a
// forward + adjoint step can be captured in a HIP graph and replayed with new
// angles.
#include <type_traits>

#include "qf_internal.h"

namespace qf {
namespace {

constexpr double kPi = 3.14159265358979323846;

template <int D>
struct DMat {
    cplx<double> m[D][D];
};

template <int D>
__device__ inline void dm_identity(DMat<D>& a) {
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) a.m[r][c] = cmake<double>(r == c ? 1.0 : 0.0, 0.0);
}

// out = G a for one forward gate G (inv: G^dagger a).
template <int D>
__device__ inline void dm_apply_gate(const DevGate& g, const double* theta, bool inv, DMat<D>& a) {
    DMat<D> o;
    const double t = g.param >= 0 ? theta[g.param] : 0.0;
    const double sg = inv ? -1.0 : 1.0;
    switch (g.kind) {
        case QF_OP_H: {
            // H is symmetric, H^dagger = conj(H)
            const double s = 1.0 / sqrt(double(D));
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) {
                    cplx<double> acc = cmake<double>(0.0, 0.0);
                    for (int m = 0; m < D; ++m) {
                        double sn, cs;
                        sincospi(2.0 * double((r * m) % D) / D, &sn, &cs);
                        cmac(acc, cmake<double>(s * cs, sg * s * sn), a.m[m][c]);
                    }
                    o.m[r][c] = acc;
                }
            a = o;
            return;
        }
        case QF_OP_CLOCK: {
            const int e = ((g.j % D) + D) % D;
            for (int r = 0; r < D; ++r) {
                double sn, cs;
                if (g.param >= 0)  // exponent from the angle array (any real value)
                    sincospi(2.0 * t * r / D, &sn, &cs);
                else
                    sincospi(2.0 * double((e * r) % D) / D, &sn, &cs);
                const cplx<double> ph = cmake<double>(cs, sg * sn);
                for (int c = 0; c < D; ++c) a.m[r][c] = cmul(ph, a.m[r][c]);
            }
            return;
        }
        case QF_OP_RZ: {
            const double al = sqrt(2.0 / (double(g.j) * (g.j + 1)));
            for (int r = 0; r <= g.j; ++r) {
                const double ang = (r < g.j ? -0.5 * t * al : 0.5 * t * al * g.j) * sg;
                double sn, cs;
                sincos(ang, &sn, &cs);
                const cplx<double> ph = cmake<double>(cs, sn);
                for (int c = 0; c < D; ++c) a.m[r][c] = cmul(ph, a.m[r][c]);
            }
            return;
        }
        case QF_OP_RX:
        case QF_OP_RY: {
            double sn, cs;
            sincos(0.5 * t, &sn, &cs);
            // rows j, k mix; R_x: [[c, -i s], [-i s, c]]; R_y: [[c, -s], [s, c]]; inverse: t -> -t
            const double s = sg * sn;
            for (int c = 0; c < D; ++c) {
                const cplx<double> x = a.m[g.j][c], y = a.m[g.k][c];
                if (g.kind == QF_OP_RX) {
                    a.m[g.j][c] = cmake<double>(cs * x.re + s * y.im, cs * x.im - s * y.re);
                    a.m[g.k][c] = cmake<double>(cs * y.re + s * x.im, cs * y.im - s * x.re);
                } else {
                    a.m[g.j][c] = cmake<double>(cs * x.re - s * y.re, cs * x.im - s * y.im);
                    a.m[g.k][c] = cmake<double>(cs * y.re + s * x.re, cs * y.im + s * x.im);
                }
            }
            return;
        }
    }
}

template <typename T, int D>
__global__ void k_build_mats(const DevGroup* __restrict__ groups, int ngroups, const DevGate* __restrict__ gates,
                             const double* __restrict__ theta, int64_t theta_stride, uint32_t batch,
                             cplx<T>* __restrict__ mats, size_t mat_stride) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= uint32_t(ngroups) * batch) return;
    const uint32_t b = t / uint32_t(ngroups);
    const DevGroup gr = groups[t - b * uint32_t(ngroups)];
    const double* th = theta + size_t(b) * size_t(theta_stride);
    cplx<T>* out = mats + size_t(b) * mat_stride + gr.mat_off;
    const double sg = gr.inv ? -1.0 : 1.0;
    if (gr.type == DG_U) {
        DMat<D> a;
        dm_identity<D>(a);
        for (int i = 0; i < gr.ng; ++i) dm_apply_gate<D>(gates[gr.g0 + i], th, gr.inv != 0, a);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) out[r * D + c] = cmake<T>(T(a.m[r][c].re), T(a.m[r][c].im));
    } else if (gr.type == DG_CR) {
        // controlled rotation table (layout in k_crot.hip); inverse: R(-m t)
        const DevGate& g = gates[gr.g0];
        const double t = th[g.param] * sg;
        for (int m = 0; m < D; ++m) {
            double sn, cs;
            if (g.kind == QF_OP_CRZ) {
                const double a = sqrt(2.0 / (double(g.j) * (g.j + 1)));
                sincos(-0.5 * m * t * a, &sn, &cs);
                out[2 * m] = cmake<T>(T(cs), T(sn));
                sincos(0.5 * m * t * a * g.j, &sn, &cs);
                out[2 * m + 1] = cmake<T>(T(cs), T(sn));
            } else {
                sincos(0.5 * m * t, &sn, &cs);
                out[2 * m] = cmake<T>(T(cs), T(sn));
                out[2 * m + 1] = cmake<T>(T(0), T(0));
            }
        }
    } else if (gr.type == DG_CZ) {
        for (int x = 0; x < D; ++x)
            for (int y = 0; y < D; ++y) {
                double sn, cs;
                sincospi(2.0 * double((x * y) % D) / D, &sn, &cs);
                out[x * D + y] = cmake<T>(T(cs), T(sg * sn));
            }
    } else {
        for (int e = 0; e < D; ++e) {
            double sn, cs;
            sincospi(2.0 * double(e) / D, &sn, &cs);
            out[e] = cmake<T>(T(cs), T(sg * sn));
        }
    }
}

// One thread per (register, run): V_i = product of the run's gates after gate
// i; contribution of rotation i = Im Tr(V_i S_i V_i^dagger M) = Im Tr(S_i W_i)
// with W_i = V_i^dagger M V_i.  Walking the run backwards, W starts as M and
// becomes G_i^dagger W G_i after gate i; rotations and phases touch two rows and
// columns or scale them, so a step costs O(D) or O(D^2) (the Fourier gate O(D^3)).
template <int D>
__device__ inline void dm_conj_diag(DMat<D>& w, const cplx<double> (&g)[D]) {
    // W <- diag(g)^dagger W diag(g)
    for (int r = 0; r < D; ++r)
        for (int q = 0; q < D; ++q) w.m[r][q] = cmul(cmul(cmake<double>(g[r].re, -g[r].im), w.m[r][q]), g[q]);
}

template <int D>
__device__ inline void dm_conj_gate(DMat<D>& w, const DevGate& gi, const double* th) {
    const double t = gi.param >= 0 ? th[gi.param] : 0.0;
    switch (gi.kind) {
        case QF_OP_RX:
        case QF_OP_RY: {
            double sn, cs;
            sincos(0.5 * t, &sn, &cs);
            // 2x2 block on levels (j, k): [[a, b], [c, d]]
            const cplx<double> a = cmake<double>(cs, 0.0), d = a;
            const cplx<double> bb = gi.kind == QF_OP_RX ? cmake<double>(0.0, -sn) : cmake<double>(-sn, 0.0);
            const cplx<double> cc = gi.kind == QF_OP_RX ? cmake<double>(0.0, -sn) : cmake<double>(sn, 0.0);
            const int j = gi.j, k = gi.k;
            for (int r = 0; r < D; ++r) {  // W <- W G (columns j, k)
                const cplx<double> x = w.m[r][j], y = w.m[r][k];
                w.m[r][j] = cadd(cmul(x, a), cmul(y, cc));
                w.m[r][k] = cadd(cmul(x, bb), cmul(y, d));
            }
            for (int q = 0; q < D; ++q) {  // W <- G^dagger W (rows j, k)
                const cplx<double> x = w.m[j][q], y = w.m[k][q];
                w.m[j][q] = cadd(cmul(cconj(a), x), cmul(cconj(cc), y));
                w.m[k][q] = cadd(cmul(cconj(bb), x), cmul(cconj(d), y));
            }
            return;
        }
        case QF_OP_RZ: {
            const double al = sqrt(2.0 / (double(gi.j) * (gi.j + 1)));
            cplx<double> g[D];
            for (int r = 0; r < D; ++r) {
                const double ang = r < gi.j ? -0.5 * t * al : r == gi.j ? 0.5 * t * al * gi.j : 0.0;
                double sn, cs;
                sincos(ang, &sn, &cs);
                g[r] = cmake<double>(cs, sn);
            }
            dm_conj_diag<D>(w, g);
            return;
        }
        case QF_OP_CLOCK: {
            const int e = ((gi.j % D) + D) % D;
            cplx<double> g[D];
            for (int r = 0; r < D; ++r) {
                double sn, cs;
                if (gi.param >= 0)
                    sincospi(2.0 * t * r / D, &sn, &cs);
                else
                    sincospi(2.0 * double((e * r) % D) / D, &sn, &cs);
                g[r] = cmake<double>(cs, sn);
            }
            dm_conj_diag<D>(w, g);
            return;
        }
        default: {
            // Fourier: H[x][q] = w^(xq) / sqrt(D); W <- H^dagger (W H), row by row then column by column
            const double s = 1.0 / sqrt(double(D));
            cplx<double> tmp[D];
            for (int r = 0; r < D; ++r) {
                for (int q = 0; q < D; ++q) {
                    cplx<double> acc = cmake<double>(0.0, 0.0);
                    for (int x = 0; x < D; ++x) {
                        double sn, cs;
                        sincospi(2.0 * double((x * q) % D) / D, &sn, &cs);
                        cmac(acc, w.m[r][x], cmake<double>(s * cs, s * sn));
                    }
                    tmp[q] = acc;
                }
                for (int q = 0; q < D; ++q) w.m[r][q] = tmp[q];
            }
            for (int q = 0; q < D; ++q) {
                for (int r = 0; r < D; ++r) {
                    cplx<double> acc = cmake<double>(0.0, 0.0);
                    for (int x = 0; x < D; ++x) {
                        double sn, cs;
                        sincospi(2.0 * double((x * r) % D) / D, &sn, &cs);
                        cmac(acc, cmake<double>(s * cs, -s * sn), w.m[x][q]);
                    }
                    tmp[r] = acc;
                }
                for (int r = 0; r < D; ++r) w.m[r][q] = tmp[r];
            }
            return;
        }
    }
}

template <int D>
__global__ void k_grad_contrib(const DevGradGroup* __restrict__ gg, int ngg, const DevGate* __restrict__ gates,
                               const double* __restrict__ theta, int64_t theta_stride, const double* __restrict__ M,
                               int nslots, uint32_t batch, double* __restrict__ contrib, int ncontrib) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= uint32_t(ngg) * batch) return;
    const uint32_t b = t / uint32_t(ngg);
    const DevGradGroup g = gg[t - b * uint32_t(ngg)];
    const double* th = theta + size_t(b) * size_t(theta_stride);
    const double* Mb = M + (size_t(b) * nslots + g.gslot) * D * D * 2;
    DMat<D> W;
    for (int r = 0; r < D; ++r)
        for (int q = 0; q < D; ++q) W.m[r][q] = cmake<double>(Mb[2 * (r * D + q)], Mb[2 * (r * D + q) + 1]);
    int c = g.c0;
    for (int i = g.ng - 1; i >= 0; --i) {
        const DevGate& gi = gates[g.g0 + i];
        if (gi.kind == QF_OP_RX) {
            contrib[size_t(b) * ncontrib + c++] = W.m[gi.k][gi.j].im + W.m[gi.j][gi.k].im;
        } else if (gi.kind == QF_OP_RY) {
            contrib[size_t(b) * ncontrib + c++] = W.m[gi.j][gi.k].re - W.m[gi.k][gi.j].re;
        } else if (gi.kind == QF_OP_RZ) {
            const double al = sqrt(2.0 / (double(gi.j) * (gi.j + 1)));
            double im = 0.0;
            for (int l = 0; l < gi.j; ++l) im += W.m[l][l].im;
            contrib[size_t(b) * ncontrib + c++] = al * im - al * gi.j * W.m[gi.j][gi.j].im;
        }
        dm_conj_gate<D>(W, gi, th);
    }
}

// grad[b][p] = scale * (sum of the contributions listed for p, in list order).
__global__ void k_grad_sum(const double* __restrict__ contrib, int ncontrib, const int32_t* __restrict__ p_off,
                           const int32_t* __restrict__ p_list, int nparams, uint32_t batch, double scale,
                           double* __restrict__ grad) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= uint32_t(nparams) * batch) return;
    const uint32_t b = t / uint32_t(nparams);
    const int p = int(t - b * uint32_t(nparams));
    double s = 0.0;
    for (int i = p_off[p]; i < p_off[p + 1]; ++i) s += contrib[size_t(b) * ncontrib + p_list[i]];
    grad[size_t(b) * nparams + p] = scale * s;
}

template <class F>
qf_status with_dim_p(int D, F&& f) {
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
        default: return set_error(QF_EUNSUPPORTED, "dim %d outside 2..16", D);
    }
}

}  // namespace

qf_status launch_build_mats(int D, int dtype, const DevGroup* groups, int ngroups, const DevGate* gates,
                            const double* theta, int64_t theta_stride, uint32_t batch, void* mats, size_t mat_stride,
                            hipStream_t st) {
    if (ngroups == 0) return QF_OK;
    const uint32_t n = uint32_t(ngroups) * batch;
    return with_dim_p(D, [&](auto dtag) -> qf_status {
        constexpr int DD = decltype(dtag)::value;
        if (dtype == QF_C64)
            hipLaunchKernelGGL((k_build_mats<float, DD>), dim3((n + 127) / 128), dim3(128), 0, st, groups, ngroups,
                               gates, theta, theta_stride, batch, reinterpret_cast<cplx<float>*>(mats), mat_stride);
        else
            hipLaunchKernelGGL((k_build_mats<double, DD>), dim3((n + 127) / 128), dim3(128), 0, st, groups, ngroups,
                               gates, theta, theta_stride, batch, reinterpret_cast<cplx<double>*>(mats), mat_stride);
        return check_launch("build matrices");
    });
}

qf_status launch_grad(int D, const DevGradGroup* gg, int ngg, const DevGate* gates, const double* theta,
                      int64_t theta_stride, const double* M, int nslots, uint32_t batch, double* contrib, int ncontrib,
                      const int32_t* p_off, const int32_t* p_list, int nparams, double scale, double* grad,
                      hipStream_t st) {
    if (nparams == 0) return QF_OK;
    if (ngg > 0) {
        const uint32_t n = uint32_t(ngg) * batch;
        qf_status r = with_dim_p(D, [&](auto dtag) -> qf_status {
            constexpr int DD = decltype(dtag)::value;
            hipLaunchKernelGGL((k_grad_contrib<DD>), dim3((n + 63) / 64), dim3(64), 0, st, gg, ngg, gates, theta,
                               theta_stride, M, nslots, batch, contrib, ncontrib);
            return check_launch("gradient contributions");
        });
        if (r != QF_OK) return r;
    }
    const uint32_t n = uint32_t(nparams) * batch;
    hipLaunchKernelGGL(k_grad_sum, dim3((n + 255) / 256), dim3(256), 0, st, contrib, ncontrib, p_off, p_list, nparams,
                       batch, scale, grad);
    return check_launch("gradient sum");
}

}  // namespace qf
