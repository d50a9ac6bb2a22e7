// Circuit plans: gate matrices built on the host in FP64 from closed forms,
// a schedule of kernel steps, the forward pass and the adjoint gradient.
//
// Gate conventions (arXiv:2409.17716, Appendix "Matrix form of the quantum
// gates"; levels 0-indexed):
//   Fourier      H_mn = w^(mn) / sqrt(D), w = exp(2 pi i / D)
//   clock Z^a    diag(w^(a m))
//   R_x^{jk}(t)  identity except [j][j] = [k][k] = cos(t/2), [j][k] = [k][j] = -i sin(t/2)
//   R_y^{jk}(t)  identity except [j][j] = [k][k] = cos(t/2), [j][k] = -sin(t/2), [k][j] = sin(t/2)
//   R_z^{j}(t)   diag: levels 0..j-1 get exp(-i t a / 2), level j gets exp(+i t a j / 2),
//                a = sqrt(2 / (j (j + 1))), all other levels 1
//   CSUM c->t    x_t -> x_t + x_c mod D (the index rule of the generalized CNOT)
//   CZ           phase w^(x_c x_t)
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <memory>
#include <vector>

#include "qf_internal.h"

namespace qf {

qf_status make_view(const qf_state* s, StateView& v);
qf_status combine_terms(const StateView& v, int32_t nterms, const int32_t* term_qudit, const double* term_diag,
                        std::vector<int>& active, std::vector<double>& table);
size_t adj_axis_partial_doubles(const StateView& s);
qf_status launch_adj_axis(const StateView& s, void* lam, int q, const double* W, double* partial, double* mout,
                          uint32_t nslots, uint32_t slot, hipStream_t st);

using cd = std::complex<double>;
using Mat = std::vector<cd>;  // row-major D x D

static Mat identity(int D) {
    Mat m(size_t(D) * D, cd(0, 0));
    for (int i = 0; i < D; ++i) m[size_t(i) * D + i] = 1.0;
    return m;
}

static Mat matmul(const Mat& A, const Mat& B, int D) {
    Mat C(size_t(D) * D, cd(0, 0));
    for (int i = 0; i < D; ++i)
        for (int k = 0; k < D; ++k) {
            const cd a = A[size_t(i) * D + k];
            if (a == cd(0, 0)) continue;
            for (int j = 0; j < D; ++j) C[size_t(i) * D + j] += a * B[size_t(k) * D + j];
        }
    return C;
}

static Mat dagger(const Mat& A, int D) {
    Mat C(size_t(D) * D);
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) C[size_t(j) * D + i] = std::conj(A[size_t(i) * D + j]);
    return C;
}

struct Gate {
    qf_op op;
    Mat mat;           // QF_OP_U: D^k x D^k
    void* dmat = nullptr;
    void* dmat_adj = nullptr;
};

static bool is_1q(int kind) {
    return kind == QF_OP_H || kind == QF_OP_CLOCK || kind == QF_OP_RX || kind == QF_OP_RY || kind == QF_OP_RZ;
}
static bool is_rot(int kind) { return kind == QF_OP_RX || kind == QF_OP_RY || kind == QF_OP_RZ; }

static Mat gate_matrix(const qf_op& g, int D, const double* theta) {
    const double pi = 3.14159265358979323846;
    Mat m = identity(D);
    switch (g.kind) {
        case QF_OP_H: {
            const double s = 1.0 / std::sqrt(double(D));
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) m[size_t(r) * D + c] = std::polar(s, 2 * pi * double((r * c) % D) / D);
            break;
        }
        case QF_OP_CLOCK:
            for (int r = 0; r < D; ++r) m[size_t(r) * D + r] = std::polar(1.0, 2 * pi * double(((g.j % D + D) % D) * r % D) / D);
            break;
        case QF_OP_RX: {
            const double t = theta[g.param];
            const double c = std::cos(t / 2), s = std::sin(t / 2);
            m[size_t(g.j) * D + g.j] = c;
            m[size_t(g.k) * D + g.k] = c;
            m[size_t(g.j) * D + g.k] = cd(0, -s);
            m[size_t(g.k) * D + g.j] = cd(0, -s);
            break;
        }
        case QF_OP_RY: {
            const double t = theta[g.param];
            const double c = std::cos(t / 2), s = std::sin(t / 2);
            m[size_t(g.j) * D + g.j] = c;
            m[size_t(g.k) * D + g.k] = c;
            m[size_t(g.j) * D + g.k] = -s;
            m[size_t(g.k) * D + g.j] = s;
            break;
        }
        case QF_OP_RZ: {
            const double t = theta[g.param];
            const double a = std::sqrt(2.0 / (double(g.j) * (g.j + 1)));
            for (int l = 0; l < g.j; ++l) m[size_t(l) * D + l] = std::polar(1.0, -0.5 * t * a);
            m[size_t(g.j) * D + g.j] = std::polar(1.0, 0.5 * t * a * g.j);
            break;
        }
        default:
            break;
    }
    return m;
}

// Hermitian generator S of a rotation (R = exp(-i t S / 2)).
static Mat generator(const qf_op& g, int D) {
    Mat m(size_t(D) * D, cd(0, 0));
    if (g.kind == QF_OP_RX) {
        m[size_t(g.j) * D + g.k] = 1.0;
        m[size_t(g.k) * D + g.j] = 1.0;
    } else if (g.kind == QF_OP_RY) {
        m[size_t(g.j) * D + g.k] = cd(0, -1);
        m[size_t(g.k) * D + g.j] = cd(0, 1);
    } else if (g.kind == QF_OP_RZ) {
        const double a = std::sqrt(2.0 / (double(g.j) * (g.j + 1)));
        for (int l = 0; l < g.j; ++l) m[size_t(l) * D + l] = a;
        m[size_t(g.j) * D + g.j] = -a * g.j;
    }
    return m;
}

enum StepType { ST_AXIS, ST_CTRL, ST_DIAG, ST_FUSED };

struct Step {
    StepType type;
    int q = 0;             // AXIS target; CTRL target; FUSED q0; DIAG first qudit
    int q2 = -1;           // CTRL control; DIAG second qudit
    int k = 1;             // FUSED qudit count
    std::vector<int> gates;  // gate indices folded into this step, in order
    bool has_param = false;
    int slot = -1;         // adjoint M slot
};

}  // namespace qf

struct qf_plan {
    int D = 0, n = 0, dtype = 0, nparams = 0;
    qf_plan_opts opts{};
    std::vector<qf::Gate> gates;
    std::vector<qf::Step> steps;
    int nslots = 0;
    ~qf_plan() {
        for (auto& g : gates) {
            if (g.dmat) (void)hipFree(g.dmat);
            if (g.dmat_adj) (void)hipFree(g.dmat_adj);
        }
    }
};

namespace qf {

static qf_status validate_op(const qf_op& o, int D, int n, int nparams) {
    auto qok = [&](int q) { return q >= 0 && q < n; };
    switch (o.kind) {
        case QF_OP_H:
            QF_RETURN_IF(!qok(o.q0), QF_EINVAL, "H on qudit %d outside [0, %d)", o.q0, n);
            break;
        case QF_OP_X:
        case QF_OP_CLOCK:
            QF_RETURN_IF(!qok(o.q0), QF_EINVAL, "qudit %d outside [0, %d)", o.q0, n);
            break;
        case QF_OP_RX:
        case QF_OP_RY:
            QF_RETURN_IF(!qok(o.q0), QF_EINVAL, "rotation qudit %d outside [0, %d)", o.q0, n);
            QF_RETURN_IF(!(o.j >= 0 && o.j < o.k && o.k < D), QF_EINVAL, "levels (%d, %d) need 0 <= j < k < D", o.j,
                         o.k);
            QF_RETURN_IF(o.param < 0 || o.param >= nparams, QF_EINVAL, "param %d outside [0, %d)", o.param, nparams);
            break;
        case QF_OP_RZ:
            QF_RETURN_IF(!qok(o.q0), QF_EINVAL, "rotation qudit %d outside [0, %d)", o.q0, n);
            QF_RETURN_IF(!(o.j >= 1 && o.j < D), QF_EINVAL, "R_z level j = %d needs 1 <= j < D", o.j);
            QF_RETURN_IF(o.param < 0 || o.param >= nparams, QF_EINVAL, "param %d outside [0, %d)", o.param, nparams);
            break;
        case QF_OP_CSUM:
        case QF_OP_CSHIFT:
        case QF_OP_CZ:
            QF_RETURN_IF(!qok(o.q0) || !qok(o.q1) || o.q0 == o.q1, QF_EINVAL, "two-qudit gate on (%d, %d)", o.q0,
                         o.q1);
            break;
        case QF_OP_U:
            QF_RETURN_IF(o.q1 < 1 || o.q0 < 0 || o.q0 + o.q1 > n, QF_EINVAL, "U on qudits %d..%d", o.q0,
                         o.q0 + o.q1 - 1);
            QF_RETURN_IF(ipow(D, o.q1) > 1024, QF_ERANGE, "U block D^k > 1024");
            QF_RETURN_IF(o.mat == nullptr, QF_EINVAL, "U matrix is NULL");
            break;
        default:
            return set_error(QF_EINVAL, "unknown op kind %d", o.kind);
    }
    return QF_OK;
}

// Schedule: one-qudit gates accumulate per qudit (gates on different qudits
// commute) and are flushed as one D x D step right before the next
// multi-qudit gate that touches the qudit, or at the end.
static void build_schedule(qf_plan* p) {
    std::vector<std::vector<int>> pending(p->n);
    auto flush = [&](int q) {
        if (pending[q].empty()) return;
        Step s;
        s.type = ST_AXIS;
        s.q = q;
        s.gates = pending[q];
        for (int gi : s.gates) s.has_param = s.has_param || is_rot(p->gates[gi].op.kind);
        p->steps.push_back(s);
        pending[q].clear();
    };
    const bool fuse = p->opts.fuse != 1;
    for (int gi = 0; gi < int(p->gates.size()); ++gi) {
        const qf_op& o = p->gates[gi].op;
        if (is_1q(o.kind)) {
            pending[o.q0].push_back(gi);
            if (!fuse) flush(o.q0);
            continue;
        }
        Step s;
        s.gates = {gi};
        switch (o.kind) {
            case QF_OP_X:
                flush(o.q0);
                s.type = ST_CTRL;
                s.q = o.q0;
                s.q2 = -1;
                break;
            case QF_OP_CSUM:
            case QF_OP_CSHIFT:
                flush(o.q0);
                flush(o.q1);
                s.type = ST_CTRL;
                s.q = o.q1;
                s.q2 = o.q0;
                break;
            case QF_OP_CZ:
                flush(o.q0);
                flush(o.q1);
                s.type = ST_DIAG;
                s.q = o.q0;
                s.q2 = o.q1;
                break;
            case QF_OP_U:
                for (int q = o.q0; q < o.q0 + o.q1; ++q) flush(q);
                s.type = ST_FUSED;
                s.q = o.q0;
                s.k = o.q1;
                break;
        }
        p->steps.push_back(s);
    }
    for (int q = 0; q < p->n; ++q) flush(q);
    p->nslots = 0;
    for (auto& s : p->steps)
        if (s.type == ST_AXIS && s.has_param) s.slot = p->nslots++;
}

static void to_interleaved(const Mat& m, std::vector<double>& out) {
    out.resize(m.size() * 2);
    for (size_t i = 0; i < m.size(); ++i) {
        out[2 * i] = m[i].real();
        out[2 * i + 1] = m[i].imag();
    }
}

static Mat step_matrix(const qf_plan* p, const Step& s, const double* theta) {
    Mat U = identity(p->D);
    for (int gi : s.gates) U = matmul(gate_matrix(p->gates[gi].op, p->D, theta), U, p->D);
    return U;
}

static void ctrl_shifts(const qf_plan* p, const Step& s, bool inverse, int32_t* sh) {
    const qf_op& o = p->gates[s.gates[0]].op;
    const int D = p->D;
    for (int c = 0; c < D; ++c) {
        int v = 0;
        if (o.kind == QF_OP_X) v = (c == 0) ? o.j : 0;
        if (o.kind == QF_OP_CSUM) v = c;
        if (o.kind == QF_OP_CSHIFT) v = o.shifts[c];
        v = ((v % D) + D) % D;
        sh[c] = inverse ? (D - v) % D : v;
    }
}

static void cz_table(int D, bool inverse, std::vector<double>& out) {
    const double pi = 3.14159265358979323846;
    out.resize(size_t(D) * D * 2);
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            const double ang = 2 * pi * double((a * b) % D) / D * (inverse ? -1.0 : 1.0);
            out[2 * (a * D + b)] = std::cos(ang);
            out[2 * (a * D + b) + 1] = std::sin(ang);
        }
}

static qf_status run_step(const qf_plan* p, const Step& s, const StateView& v, const double* theta, bool inverse,
                          hipStream_t st) {
    std::vector<double> buf;
    switch (s.type) {
        case ST_AXIS: {
            Mat U = step_matrix(p, s, theta);
            if (inverse) U = dagger(U, p->D);
            to_interleaved(U, buf);
            return launch_apply_1q(v, s.q, buf.data(), st);
        }
        case ST_CTRL: {
            int32_t sh[kMaxDim];
            ctrl_shifts(p, s, inverse, sh);
            return launch_ctrl(v, s.q2, s.q, sh, st);
        }
        case ST_DIAG: {
            cz_table(p->D, inverse, buf);
            const int32_t qs[2] = {s.q, s.q2};
            return launch_diag(v, 2, qs, buf.data(), st);
        }
        case ST_FUSED: {
            const Gate& g = p->gates[s.gates[0]];
            return launch_fused(v, s.k, s.q, inverse ? g.dmat_adj : g.dmat, st);
        }
    }
    return QF_OK;
}

static qf_status check_plan_state(const qf_plan* p, const qf_state* s, StateView& v) {
    QF_RETURN_IF(p == nullptr, QF_EINVAL, "plan is NULL");
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(int(v.D) != p->D || int(v.n) != p->n || v.dtype != p->dtype, QF_EINVAL,
                 "state (dim %u, n %u, dtype %d) does not match the plan (dim %d, n %d, dtype %d)", v.D, v.n, v.dtype,
                 p->D, p->n, p->dtype);
    return QF_OK;
}

}  // namespace qf

using namespace qf;

extern "C" {

qf_status qf_plan_create(int32_t dim, int32_t n, int32_t dtype, const qf_op* ops, int32_t nops, int32_t nparams,
                         const qf_plan_opts* opts, qf_plan** out) {
    QF_RETURN_IF(out == nullptr, QF_EINVAL, "out is NULL");
    *out = nullptr;
    QF_RETURN_IF(dim < 2 || dim > kMaxDim, QF_ERANGE, "dim %d outside 2..%d", dim, kMaxDim);
    QF_RETURN_IF(n < 1, QF_EINVAL, "n = %d < 1", n);
    QF_RETURN_IF(dtype != QF_C64 && dtype != QF_C128, QF_EDTYPE, "unknown dtype %d", dtype);
    QF_RETURN_IF(nops < 0 || (nops > 0 && ops == nullptr), QF_EINVAL, "bad op list");
    QF_RETURN_IF(nparams < 0, QF_EINVAL, "nparams < 0");
    for (int i = 0; i < nops; ++i) {
        qf_status st = validate_op(ops[i], dim, n, nparams);
        if (st != QF_OK) return set_error(st, "op %d: %s", i, qf_last_error());
    }
    std::unique_ptr<qf_plan> p(new (std::nothrow) qf_plan);
    QF_RETURN_IF(!p, QF_ENOMEM, "plan allocation failed");
    p->D = dim;
    p->n = n;
    p->dtype = dtype;
    p->nparams = nparams;
    if (opts) p->opts = *opts;
    p->gates.resize(nops);
    for (int i = 0; i < nops; ++i) {
        Gate& g = p->gates[i];
        g.op = ops[i];
        g.op.mat = nullptr;
        if (ops[i].kind == QF_OP_U) {
            const size_t K = ipow(dim, ops[i].q1);
            g.mat.resize(K * K);
            for (size_t e = 0; e < K * K; ++e) g.mat[e] = cd(ops[i].mat[2 * e], ops[i].mat[2 * e + 1]);
            const size_t esz = dtype == QF_C64 ? 8 : 16;
            std::vector<unsigned char> a(K * K * esz), b(K * K * esz);
            for (size_t r = 0; r < K; ++r)
                for (size_t c = 0; c < K; ++c) {
                    const cd x = g.mat[r * K + c];
                    const cd y = std::conj(g.mat[c * K + r]);
                    if (dtype == QF_C64) {
                        float* fa = reinterpret_cast<float*>(a.data()) + 2 * (r * K + c);
                        float* fb = reinterpret_cast<float*>(b.data()) + 2 * (r * K + c);
                        fa[0] = float(x.real()); fa[1] = float(x.imag());
                        fb[0] = float(y.real()); fb[1] = float(y.imag());
                    } else {
                        double* da = reinterpret_cast<double*>(a.data()) + 2 * (r * K + c);
                        double* db = reinterpret_cast<double*>(b.data()) + 2 * (r * K + c);
                        da[0] = x.real(); da[1] = x.imag();
                        db[0] = y.real(); db[1] = y.imag();
                    }
                }
            QF_HIP_CHECK(hipMalloc(&g.dmat, a.size()));
            QF_HIP_CHECK(hipMalloc(&g.dmat_adj, b.size()));
            QF_HIP_CHECK(hipMemcpy(g.dmat, a.data(), a.size(), hipMemcpyHostToDevice));
            QF_HIP_CHECK(hipMemcpy(g.dmat_adj, b.data(), b.size(), hipMemcpyHostToDevice));
        }
    }
    build_schedule(p.get());
    *out = p.release();
    return QF_OK;
}

int32_t qf_plan_num_stages(const qf_plan* plan) { return plan ? int32_t(plan->steps.size()) : -1; }

qf_status qf_plan_forward(qf_plan* plan, const qf_state* s, const double* theta, void* stream) {
    StateView v;
    QF_CHECK(check_plan_state(plan, s, v));
    QF_RETURN_IF(plan->nparams > 0 && theta == nullptr, QF_EINVAL, "theta is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (const Step& step : plan->steps) QF_CHECK(run_step(plan, step, v, theta, false, st));
    return QF_OK;
}

qf_status qf_adjoint_grad(qf_plan* plan, const qf_state* psi, const qf_state* lam, const double* theta,
                          int32_t nterms, const int32_t* term_qudit, const double* term_diag, double* grad,
                          void* stream) {
    StateView v, vl;
    QF_CHECK(check_plan_state(plan, psi, v));
    QF_CHECK(check_plan_state(plan, lam, vl));
    QF_RETURN_IF(vl.batch != v.batch, QF_EINVAL, "psi and lam batch differ");
    QF_RETURN_IF(psi->amps == lam->amps, QF_EINVAL, "psi and lam must not alias");
    QF_RETURN_IF(grad == nullptr, QF_EINVAL, "grad is NULL");
    QF_RETURN_IF(plan->nparams > 0 && theta == nullptr, QF_EINVAL, "theta is NULL");
    std::vector<int> active;
    std::vector<double> table;
    QF_CHECK(combine_terms(v, nterms, term_qudit, term_diag, active, table));
    std::vector<double> table_re(active.size() * v.D);
    for (size_t i = 0; i < table_re.size(); ++i) table_re[i] = table[2 * i];
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int D = plan->D;
    const size_t E = size_t(D) * D;

    // lam = H_O psi with H_O the Hermitian part of O
    QF_CHECK(launch_diag_observable(v, lam->amps, active, table_re, st));

    double* partial = nullptr;
    double* mdev = nullptr;
    const size_t mcount = size_t(v.batch) * std::max(plan->nslots, 1) * E * 2;
    QF_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&partial),
                                std::max<size_t>(adj_axis_partial_doubles(v), 1) * sizeof(double), st));
    QF_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&mdev), mcount * sizeof(double), st));
    qf_status rs = QF_OK;
    for (int si = int(plan->steps.size()) - 1; si >= 0 && rs == QF_OK; --si) {
        const Step& s = plan->steps[si];
        if (s.type == ST_AXIS && s.has_param) {
            Mat W = dagger(step_matrix(plan, s, theta), D);
            std::vector<double> buf;
            to_interleaved(W, buf);
            rs = launch_adj_axis(v, lam->amps, s.q, buf.data(), partial, mdev, plan->nslots, s.slot, st);
        } else {
            rs = run_step(plan, s, v, theta, true, st);
            if (rs == QF_OK) rs = run_step(plan, s, vl, theta, true, st);
        }
    }
    std::vector<double> mhost(mcount);
    if (rs == QF_OK && plan->nslots > 0) {
        hipError_t e = hipMemcpyAsync(mhost.data(), mdev, mcount * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) rs = set_error(QF_EHIP, "copy of M matrices failed: %s", hipGetErrorString(e));
    }
    (void)hipFreeAsync(partial, st);
    (void)hipFreeAsync(mdev, st);
    hipError_t e = hipStreamSynchronize(st);
    if (rs != QF_OK) return rs;
    QF_RETURN_IF(e != hipSuccess, QF_EHIP, "stream synchronisation failed: %s", hipGetErrorString(e));

    // dL/dtheta_i = Im Tr(V_i S_i V_i^dagger M) with V_i the product of the
    // step's gates after gate i and M = sum_f psi_f lam_f^dagger after the step.
    std::memset(grad, 0, sizeof(double) * size_t(v.batch) * plan->nparams);
    for (const Step& s : plan->steps) {
        if (!(s.type == ST_AXIS && s.has_param)) continue;
        const int m = int(s.gates.size());
        std::vector<Mat> suffix(m + 1);
        suffix[m] = identity(D);
        for (int i = m - 1; i >= 0; --i)
            suffix[i] = matmul(suffix[i + 1], gate_matrix(plan->gates[s.gates[i]].op, D, theta), D);
        for (int i = 0; i < m; ++i) {
            const qf_op& o = plan->gates[s.gates[i]].op;
            if (!is_rot(o.kind)) continue;
            const Mat& V = suffix[i + 1];
            const Mat A = matmul(matmul(V, generator(o, D), D), dagger(V, D), D);
            for (uint32_t b = 0; b < v.batch; ++b) {
                const double* M = mhost.data() + ((size_t(b) * plan->nslots + s.slot) * E) * 2;
                cd tr(0, 0);
                for (int r = 0; r < D; ++r)
                    for (int c = 0; c < D; ++c) tr += A[size_t(r) * D + c] * cd(M[2 * (c * D + r)], M[2 * (c * D + r) + 1]);
                grad[size_t(b) * plan->nparams + o.param] += tr.imag();
            }
        }
    }
    return QF_OK;
}

void qf_plan_destroy(qf_plan* plan) { delete plan; }

}  // extern "C"
