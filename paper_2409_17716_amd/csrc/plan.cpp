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
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "qf_internal.h"

namespace qf {

qf_status make_view(const qf_state* s, StateView& v);
qf_status combine_terms(const StateView& v, int32_t nterms, const int32_t* term_qudit, const double* term_diag,
                        std::vector<int>& active, std::vector<double>& table);
size_t adj_axis_partial_doubles(const StateView& s);
qf_status launch_adj_axis(const StateView& s, void* lam, int q, const double* W, double* partial, double* mout,
                          uint32_t nslots, uint32_t slot, uint32_t slot_elems, hipStream_t st);

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
    bool real = false; // QF_OP_U: every imaginary part is zero
};

// A two-qudit dense block made of the one-qudit runs of qudits q0 and q0 + 1
// (pair mode, forward only): U_run0 (x) U_run1, rebuilt from theta per call.
struct Synth {
    qf_op op;                 // kind QF_OP_U on q0, q0 + 1
    std::vector<int> run0, run1;
    bool real = false;
};

static bool is_1q(int kind) {
    return kind == QF_OP_H || kind == QF_OP_CLOCK || kind == QF_OP_RX || kind == QF_OP_RY || kind == QF_OP_RZ;
}
static bool is_rot(int kind) { return kind == QF_OP_RX || kind == QF_OP_RY || kind == QF_OP_RZ; }
static bool is_crot(int kind) { return kind == QF_OP_CRX || kind == QF_OP_CRY || kind == QF_OP_CRZ; }
// Gates that never enter an LDS tile: each makes a pass of its own (dense
// blocks, controlled rotations).
static bool pass_gate(int kind) {
    return kind == QF_OP_U || is_crot(kind) || kind == QF_OP_SWAP || kind == QF_OP_MCX;
}
static CrotArgs crot_args(const qf_op& o) { return CrotArgs{o.kind - QF_OP_CRX, o.q0, o.q1, o.j, o.k}; }
// A lone rotation as a controlled rotation whose every fibre takes table
// entry m = 1 (the two-level slab kernel).
static qf_op slab_op(const qf_op& o) {
    qf_op t = o;
    t.kind = QF_OP_CRX + (o.kind - QF_OP_RX);
    t.q1 = o.q0;
    t.q0 = -1;
    return t;
}

// Table of a controlled rotation for control levels m = 0..nlev-1 (2 nlev
// complex entries, interleaved FP64; layout in k_crot.hip): x, y types
// (cos(m t / 2), sin(m t / 2)) at 2m; z type exp(-i m t a / 2) (levels below
// j) at 2m and exp(+i m t a j / 2) (level j) at 2m + 1, a = sqrt(2/(j(j+1))).
// The inverse is R(-m t).
static void crot_table(const qf_op& o, int nlev, const double* theta, bool inverse, std::vector<double>& out) {
    out.assign(size_t(4) * nlev, 0.0);
    const double t = theta[o.param] * (inverse ? -1.0 : 1.0);
    for (int m = 0; m < nlev; ++m) {
        if (o.kind == QF_OP_CRZ) {
            const double a = std::sqrt(2.0 / (double(o.j) * (o.j + 1)));
            out[4 * m] = std::cos(-0.5 * m * t * a);
            out[4 * m + 1] = std::sin(-0.5 * m * t * a);
            out[4 * m + 2] = std::cos(0.5 * m * t * a * o.j);
            out[4 * m + 3] = std::sin(0.5 * m * t * a * o.j);
        } else {
            out[4 * m] = std::cos(0.5 * m * t);
            out[4 * m + 1] = std::sin(0.5 * m * t);
        }
    }
}

// SWAP and multi-controlled shifts (inverse: the shift subtracts; SWAP is its own inverse).
static qf_status launch_perm_gate(const StateView& v, const qf_op& o, bool inverse, hipStream_t st) {
    if (o.kind == QF_OP_SWAP) return launch_swap(v, o.q0, o.q1, st);
    return launch_mcx(v, o.j, o.shifts, o.q1, inverse, st);
}

static qf_status check_finite_theta(const double* theta, int nparams) {
    for (int i = 0; i < nparams; ++i)
        QF_RETURN_IF(!std::isfinite(theta[i]), QF_EINVAL, "theta[%d] is not finite", i);
    return QF_OK;
}

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
            if (g.param >= 0) {  // exponent a = theta[param] (any real value)
                for (int r = 0; r < D; ++r) m[size_t(r) * D + r] = std::polar(1.0, 2 * pi * theta[g.param] * r / D);
            } else {
                for (int r = 0; r < D; ++r)
                    m[size_t(r) * D + r] = std::polar(1.0, 2 * pi * double(((g.j % D + D) % D) * r % D) / D);
            }
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

// ---------------------------------------------------------------------------
// Per-gate schedule (opts.fuse = 1: one kernel per gate; 2: one kernel per run
// of one-qudit gates on a qudit).
// ---------------------------------------------------------------------------

enum StepType { ST_AXIS, ST_CTRL, ST_DIAG, ST_FUSED, ST_CROT, ST_PERM };

struct Step {
    StepType type;
    int q = 0;               // AXIS target; CTRL target; FUSED q0; DIAG first qudit
    int q2 = -1;             // CTRL control; DIAG second qudit
    int k = 1;               // FUSED qudit count
    std::vector<int> gates;  // gate indices folded into this step, in order
    bool has_param = false;
    int slot = -1;           // adjoint M slot
    int cr_slot = -1;        // ST_CROT, slab steps: index among the gradient outputs
    bool slab = false;       // ST_AXIS holding one rotation: run as a two-level slab sweep
};

// ---------------------------------------------------------------------------
// Stage schedule (opts.fuse = 0).
// ---------------------------------------------------------------------------

struct GRef {
    int gi;
    bool inv;
};

// A stage op before its matrices exist.
struct HOp {
    int type;                // SOP_U / SOP_SHIFT / SOP_PHASE
    int q = -1;              // U, SHIFT: tile qudit acted on
    int ctrl = -1;           // SHIFT: control qudit or -1
    std::vector<GRef> g;     // U: fused run in application order; SHIFT: one gate; PHASE: factors
    int slot = -1;           // adjoint: stage-local M slot
    int gslot = -1;          // adjoint: plan-wide M slot
};

struct Pass {
    bool tile = true;
    std::vector<int> T;      // tile qudits, ascending
    StageGeom geom{};
    std::vector<HOp> ops;
    int nslots = 0, slot0 = 0;
    int op_off = 0, nops = 0;
    size_t mat_off = 0, nmat = 0;  // complex elements
    GRef fused{-1, false};   // !tile: the dense block gate
    int seg = 0;             // checkpoint segment
    int round_off = 0, nrounds = 0;  // register rounds (forward); nrounds = 0: op-by-op kernel
    int cr_slot = -1;        // !tile controlled rotation: its index among the list's controlled rotations
};

struct PassList {
    std::vector<Pass> passes;
    std::vector<StageOp> hops;
    std::vector<RoundDesc> hrounds;
    RoundDesc* drounds = nullptr;
    std::vector<DevGroup> hgroups;   // bound mode: matrices built on the device
    DevGroup* dgroups = nullptr;
    void* dmats_b = nullptr;         // bound mode: batch x nmats matrices
    size_t nmats = 0;
    int nslots = 0;
    int ncr = 0;                     // controlled-rotation passes
    StageOp* dops = nullptr;
    void* dmats = nullptr;
    void* hmats = nullptr;
    hipEvent_t copied = nullptr, done = nullptr;
    bool copied_valid = false, done_valid = false;
    void release_bound() {
        if (dgroups) (void)hipFree(dgroups);
        if (dmats_b) (void)hipFree(dmats_b);
        dgroups = nullptr;
        dmats_b = nullptr;
    }
    void release() {
        release_bound();
        if (drounds) (void)hipFree(drounds);
        drounds = nullptr;
        if (dops) (void)hipFree(dops);
        if (dmats) (void)hipFree(dmats);
        if (hmats) (void)hipHostFree(hmats);
        if (copied) (void)hipEventDestroy(copied);
        if (done) (void)hipEventDestroy(done);
        dops = nullptr;
        dmats = hmats = nullptr;
        copied = done = nullptr;
    }
};

struct ProfRec {
    int family;
    double bytes;
    hipEvent_t a, b;
};

}  // namespace qf

struct qf_plan {
    int D = 0, n = 0, dtype = 0, nparams = 0;  // D = 0: the qudits' dimensions differ
    std::vector<int> dims;            // per-qudit dimensions (all D for a uniform register)
    int group = 1;                    // register-round group size
    qf_plan_opts opts{};
    std::vector<qf::Gate> gates;
    std::vector<qf::Synth> synth;     // fuse = 3
    std::vector<qf::Step> steps;      // fuse = 1, 2
    int nslots = 0;                   // fuse = 1, 2
    int ncr_steps = 0;                // fuse = 1, 2: controlled rotations
    std::vector<int> cr_contrib;      // bound mode: contribution slot of each reverse controlled rotation
    qf::PassList fwd, rev;            // fuse = 0
    std::vector<int> seg_end;         // gate index where each checkpoint segment ends
    void* ckpt = nullptr;             // (nseg - 1) saved states
    size_t ckpt_bytes = 0;
    const void* ckpt_amps = nullptr;  // state and batch of the forward that wrote the checkpoints
    uint32_t ckpt_batch = 0;
    bool profiling = false;
    std::vector<qf::ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    // bound (device-parameter) mode
    uint32_t bound = 0;
    std::vector<qf::DevGate> hgates;
    qf::DevGate* dgates = nullptr;
    std::vector<qf::DevGradGroup> hgg;
    qf::DevGradGroup* dgg = nullptr;
    int32_t* d_poff = nullptr;
    int32_t* d_plist = nullptr;
    int ncontrib = 0;
    double* w_partial = nullptr;
    double* w_m = nullptr;
    double* w_contrib = nullptr;
    double* w_expect = nullptr;
    void release_bound() {
        for (void* q : {static_cast<void*>(dgates), static_cast<void*>(dgg), static_cast<void*>(d_poff),
                        static_cast<void*>(d_plist), static_cast<void*>(w_partial), static_cast<void*>(w_m),
                        static_cast<void*>(w_contrib), static_cast<void*>(w_expect)})
            if (q) (void)hipFree(q);
        dgates = nullptr;
        dgg = nullptr;
        d_poff = d_plist = nullptr;
        w_partial = w_m = w_contrib = w_expect = nullptr;
        fwd.release_bound();
        rev.release_bound();
        bound = 0;
    }
    qf_plan() = default;
    qf_plan(const qf_plan&) = delete;
    qf_plan& operator=(const qf_plan&) = delete;
    // Exchanges everything, including the ownership of device buffers and events.
    void swap_with(qf_plan& o) {
        std::swap(D, o.D);
        dims.swap(o.dims);
        std::swap(n, o.n);
        std::swap(dtype, o.dtype);
        std::swap(nparams, o.nparams);
        std::swap(group, o.group);
        std::swap(opts, o.opts);
        gates.swap(o.gates);
        synth.swap(o.synth);
        steps.swap(o.steps);
        std::swap(nslots, o.nslots);
        std::swap(ncr_steps, o.ncr_steps);
        cr_contrib.swap(o.cr_contrib);
        std::swap(fwd, o.fwd);
        std::swap(rev, o.rev);
        seg_end.swap(o.seg_end);
        std::swap(ckpt, o.ckpt);
        std::swap(ckpt_bytes, o.ckpt_bytes);
        std::swap(ckpt_amps, o.ckpt_amps);
        std::swap(ckpt_batch, o.ckpt_batch);
        std::swap(profiling, o.profiling);
        prof.swap(o.prof);
        ev_pool.swap(o.ev_pool);
        std::swap(ev_used, o.ev_used);
        std::swap(bound, o.bound);
        hgates.swap(o.hgates);
        std::swap(dgates, o.dgates);
        hgg.swap(o.hgg);
        std::swap(dgg, o.dgg);
        std::swap(d_poff, o.d_poff);
        std::swap(d_plist, o.d_plist);
        std::swap(ncontrib, o.ncontrib);
        std::swap(w_partial, o.w_partial);
        std::swap(w_m, o.w_m);
        std::swap(w_contrib, o.w_contrib);
        std::swap(w_expect, o.w_expect);
    }
    ~qf_plan() {
        release_bound();
        for (auto& g : gates) {
            if (g.dmat) (void)hipFree(g.dmat);
            if (g.dmat_adj) (void)hipFree(g.dmat_adj);
        }
        fwd.release();
        rev.release();
        if (ckpt) (void)hipFree(ckpt);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
};

namespace qf {

// fuse 0 (LDS stages) and 3 (stages + two-qudit blocks) use pass lists.
static bool staged(const qf_plan* p) { return p->opts.fuse == 0 || p->opts.fuse == 3; }

// Register group of the adjoint rounds: psi and lam sub-tiles are both live, so
// at most 2 qudits; 1 for D >= 5 (measured faster) and for complex128 with
// D >= 4 (register budget).
static int adj_group(const qf_plan* p) {
    if (p->D >= 5 || (p->dtype == QF_C128 && p->D >= 4)) return 1;
    return std::min(p->group, 2);
}

static const char* kFamilies[] = {"stage", "stage_adj", "fused", "axis", "ctrl", "diag", "adj_axis", "checkpoint",
                                  "crot", "crot_adj"};
enum Family { F_STAGE, F_STAGE_ADJ, F_FUSED, F_AXIS, F_CTRL, F_DIAG, F_ADJ_AXIS, F_CKPT, F_CROT, F_CROT_ADJ, F_COUNT };

static qf_status validate_op(const qf_op& o, const std::vector<int>& dims, int nparams) {
    const int n = int(dims.size());
    auto qok = [&](int q) { return q >= 0 && q < n; };
    switch (o.kind) {
        case QF_OP_H:
            QF_RETURN_IF(!qok(o.q0), QF_EINVAL, "H on qudit %d outside [0, %d)", o.q0, n);
            break;
        case QF_OP_X:
        case QF_OP_CLOCK:
            QF_RETURN_IF(!qok(o.q0), QF_EINVAL, "qudit %d outside [0, %d)", o.q0, n);
            QF_RETURN_IF(o.kind == QF_OP_CLOCK && o.param >= nparams, QF_EINVAL, "param %d outside [0, %d)", o.param,
                         nparams);
            break;
        case QF_OP_RX:
        case QF_OP_RY:
            QF_RETURN_IF(!qok(o.q0), QF_EINVAL, "rotation qudit %d outside [0, %d)", o.q0, n);
            QF_RETURN_IF(!(o.j >= 0 && o.j < o.k && o.k < dims[o.q0]), QF_EINVAL,
                         "levels (%d, %d) need 0 <= j < k < %d", o.j, o.k, dims[o.q0]);
            QF_RETURN_IF(o.param < 0 || o.param >= nparams, QF_EINVAL, "param %d outside [0, %d)", o.param, nparams);
            break;
        case QF_OP_RZ:
            QF_RETURN_IF(!qok(o.q0), QF_EINVAL, "rotation qudit %d outside [0, %d)", o.q0, n);
            QF_RETURN_IF(!(o.j >= 1 && o.j < dims[o.q0]), QF_EINVAL, "R_z level j = %d needs 1 <= j < %d", o.j,
                         dims[o.q0]);
            QF_RETURN_IF(o.param < 0 || o.param >= nparams, QF_EINVAL, "param %d outside [0, %d)", o.param, nparams);
            break;
        case QF_OP_CSUM:
        case QF_OP_CSHIFT:
        case QF_OP_CZ:
            QF_RETURN_IF(!qok(o.q0) || !qok(o.q1) || o.q0 == o.q1, QF_EINVAL, "two-qudit gate on (%d, %d)", o.q0,
                         o.q1);
            break;
        case QF_OP_CRX:
        case QF_OP_CRY:
        case QF_OP_CRZ:
            QF_RETURN_IF(!qok(o.q0) || !qok(o.q1) || o.q0 == o.q1, QF_EINVAL, "controlled rotation on (%d, %d)", o.q0,
                         o.q1);
            if (o.kind == QF_OP_CRZ)
                QF_RETURN_IF(!(o.j >= 1 && o.j < dims[o.q1]), QF_EINVAL, "R_z level j = %d needs 1 <= j < %d", o.j,
                             dims[o.q1]);
            else
                QF_RETURN_IF(!(o.j >= 0 && o.j < o.k && o.k < dims[o.q1]), QF_EINVAL,
                             "levels (%d, %d) need 0 <= j < k < %d", o.j, o.k, dims[o.q1]);
            QF_RETURN_IF(o.param < 0 || o.param >= nparams, QF_EINVAL, "param %d outside [0, %d)", o.param, nparams);
            break;
        case QF_OP_SWAP:
            QF_RETURN_IF(!qok(o.q0) || !qok(o.q1) || o.q0 == o.q1, QF_EINVAL, "SWAP of (%d, %d)", o.q0, o.q1);
            QF_RETURN_IF(dims[o.q0] != dims[o.q1], QF_EINVAL, "SWAP of qudits of dimensions %d and %d", dims[o.q0],
                         dims[o.q1]);
            break;
        case QF_OP_MCX:
            QF_RETURN_IF(!qok(o.q1), QF_EINVAL, "MCX target %d outside [0, %d)", o.q1, n);
            QF_RETURN_IF(o.j < 1 || o.j > 8, QF_EINVAL, "MCX with %d controls (1..8)", o.j);
            for (int i = 0; i < o.j; ++i) {
                QF_RETURN_IF(!qok(o.shifts[i]) || o.shifts[i] == o.q1, QF_EINVAL, "MCX control %d", o.shifts[i]);
                for (int m = 0; m < i; ++m)
                    QF_RETURN_IF(o.shifts[m] == o.shifts[i], QF_EINVAL, "MCX control %d listed twice", o.shifts[i]);
            }
            break;
        case QF_OP_U:
            QF_RETURN_IF(o.q1 < 1 || o.q0 < 0 || o.q0 + o.q1 > n, QF_EINVAL, "U on qudits %d..%d", o.q0,
                         o.q0 + o.q1 - 1);
            {
                uint64_t K = 1;
                for (int q = o.q0; q < o.q0 + o.q1; ++q) K *= uint64_t(dims[q]);
                QF_RETURN_IF(K > 1024, QF_ERANGE, "U block of %llu > 1024 levels", (unsigned long long)K);
            }
            QF_RETURN_IF(o.mat == nullptr, QF_EINVAL, "U matrix is NULL");
            break;
        default:
            return set_error(QF_EINVAL, "unknown op kind %d", o.kind);
    }
    return QF_OK;
}

static void to_interleaved(const Mat& m, std::vector<double>& out) {
    out.resize(m.size() * 2);
    for (size_t i = 0; i < m.size(); ++i) {
        out[2 * i] = m[i].real();
        out[2 * i + 1] = m[i].imag();
    }
}

static int shift_of(const qf_op& o, int c, int D) {
    int v = 0;
    if (o.kind == QF_OP_X) v = (c == 0) ? o.j : 0;
    if (o.kind == QF_OP_CSUM) v = c;
    if (o.kind == QF_OP_CSHIFT) v = o.shifts[c];
    return ((v % D) + D) % D;
}

// Controlled phase w_t^(x_c x_t) over (x_c, x_t), w_t = exp(2 pi i / d_t): the
// clock gate of the target raised to the control digit.
static void cz_table(int dc, int dt, bool inverse, Mat& out) {
    const double pi = 3.14159265358979323846;
    out.assign(size_t(dc) * dt, cd(0, 0));
    for (int a = 0; a < dc; ++a)
        for (int b = 0; b < dt; ++b)
            out[size_t(a) * dt + b] = std::polar(1.0, 2 * pi * double((a * b) % dt) / dt * (inverse ? -1.0 : 1.0));
}

// ---- per-gate schedule ----

static void build_steps(qf_plan* p) {
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
    const bool per_gate = p->opts.fuse == 1;
    for (int gi = 0; gi < int(p->gates.size()); ++gi) {
        const qf_op& o = p->gates[gi].op;
        if (is_1q(o.kind)) {
            pending[o.q0].push_back(gi);
            if (per_gate) flush(o.q0);
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
            case QF_OP_CRX:
            case QF_OP_CRY:
            case QF_OP_CRZ:
                flush(o.q0);
                flush(o.q1);
                s.type = ST_CROT;
                s.q = o.q1;
                s.q2 = o.q0;
                break;
            case QF_OP_SWAP:
                flush(o.q0);
                flush(o.q1);
                s.type = ST_PERM;
                s.q = o.q1;
                break;
            case QF_OP_MCX:
                for (int i = 0; i < o.j; ++i) flush(o.shifts[i]);
                flush(o.q1);
                s.type = ST_PERM;
                s.q = o.q1;
                break;
        }
        p->steps.push_back(s);
    }
    for (int q = 0; q < p->n; ++q) flush(q);
    p->nslots = 0;
    p->ncr_steps = 0;
    for (auto& s : p->steps) {
        // a step of one lone rotation runs as a slab sweep: it reads and writes
        // only the levels the rotation moves, and its gradient comes straight
        // from the slab adjoint kernel
        s.slab = s.type == ST_AXIS && s.gates.size() == 1 && is_rot(p->gates[s.gates[0]].op.kind);
        if (s.type == ST_AXIS && s.has_param && !s.slab) s.slot = p->nslots++;
        if (s.type == ST_CROT || s.slab) s.cr_slot = p->ncr_steps++;
    }
}

// Number of control levels of a controlled rotation's table (2 for a lone
// rotation run as a slab: m = 0 unused, m = 1 the rotation).
static int ctrl_levels(const qf_plan* p, const qf_op& o) { return o.q0 >= 0 ? p->dims[o.q0] : 2; }

static Mat step_matrix(const qf_plan* p, const Step& s, const double* theta) {
    const int d = p->dims[s.q];
    Mat U = identity(d);
    for (int gi : s.gates) U = matmul(gate_matrix(p->gates[gi].op, d, theta), U, d);
    return U;
}

static qf_status run_step(const qf_plan* p, const Step& s, const StateView& v, const double* theta, bool inverse,
                          hipStream_t st) {
    switch (s.type) {
        case ST_AXIS: {
            if (s.slab) {
                const qf_op so = slab_op(p->gates[s.gates[0]].op);
                std::vector<double> tab;
                crot_table(so, ctrl_levels(p, so), theta, inverse, tab);
                return launch_crot(v, crot_args(so), nullptr, 0, tab.data(), st);
            }
            Mat U = step_matrix(p, s, theta);
            if (inverse) U = dagger(U, p->dims[s.q]);
            std::vector<double> buf;
            to_interleaved(U, buf);
            return launch_apply_1q(v, s.q, buf.data(), st);
        }
        case ST_CTRL: {
            int32_t sh[kMaxDim] = {};
            const qf_op& o = p->gates[s.gates[0]].op;
            const int dt = p->dims[s.q], nc = s.q2 >= 0 ? p->dims[s.q2] : 1;
            for (int c = 0; c < nc; ++c) {
                const int v0 = shift_of(o, c, dt);
                sh[c] = inverse ? (dt - v0) % dt : v0;
            }
            return launch_ctrl(v, s.q2, s.q, sh, st);
        }
        case ST_DIAG: {
            Mat t;
            cz_table(p->dims[s.q], p->dims[s.q2], inverse, t);
            std::vector<double> buf;
            to_interleaved(t, buf);
            const int32_t qs[2] = {s.q, s.q2};
            return launch_diag(v, 2, qs, buf.data(), st);
        }
        case ST_FUSED: {
            const Gate& g = p->gates[s.gates[0]];
            return launch_fused(v, s.k, s.q, inverse ? g.dmat_adj : g.dmat, st);
        }
        case ST_CROT: {
            const qf_op& o = p->gates[s.gates[0]].op;
            std::vector<double> tab;
            crot_table(o, ctrl_levels(p, o), theta, inverse, tab);
            return launch_crot(v, crot_args(o), nullptr, 0, tab.data(), st);
        }
        case ST_PERM:
            return launch_perm_gate(v, p->gates[s.gates[0]].op, inverse, st);
    }
    return QF_OK;
}

// ---- stage planning ----

struct Touch {
    int q;
    bool diag;  // the gate is block diagonal in this qudit's basis
};

static void touches(const qf_op& o, std::vector<Touch>& t) {
    t.clear();
    switch (o.kind) {
        case QF_OP_H:
        case QF_OP_RX:
        case QF_OP_RY:
        case QF_OP_X:
            t.push_back({o.q0, false});
            break;
        case QF_OP_CLOCK:
        case QF_OP_RZ:
            t.push_back({o.q0, true});
            break;
        case QF_OP_CSUM:
        case QF_OP_CSHIFT:
            t.push_back({o.q0, true});
            t.push_back({o.q1, false});
            break;
        case QF_OP_CZ:
            t.push_back({o.q0, true});
            t.push_back({o.q1, true});
            break;
        case QF_OP_CRX:
        case QF_OP_CRY:
        case QF_OP_CRZ:
            t.push_back({o.q0, true});
            t.push_back({o.q1, o.kind == QF_OP_CRZ});
            break;
        case QF_OP_SWAP:
            t.push_back({o.q0, false});
            t.push_back({o.q1, false});
            break;
        case QF_OP_MCX:
            for (int i = 0; i < o.j; ++i) t.push_back({o.shifts[i], true});
            t.push_back({o.q1, false});
            break;
        case QF_OP_U:
            for (int q = o.q0; q < o.q0 + o.q1; ++q) t.push_back({q, false});
            break;
    }
}

static const qf_op& op_of(const qf_plan* p, const GRef& r) {
    const int ng = int(p->gates.size());
    return r.gi < ng ? p->gates[r.gi].op : p->synth[r.gi - ng].op;
}

// Pair mode: one-qudit runs of qudits (2i, 2i+1) are collected and emitted as
// one dense two-qudit block right before the next gate that touches either
// qudit (the runs commute with every gate in between).  An odd last qudit keeps
// its one-qudit gates.
static void pair_fuse(qf_plan* p, int lo, int hi, std::vector<GRef>& seq) {
    const int n = p->n, ng = int(p->gates.size());
    std::vector<std::vector<int>> pending(n);
    auto flush_pair = [&](int pr) {
        const int a = 2 * pr, b = 2 * pr + 1;
        if (b >= n) {
            for (int gi : pending[a]) seq.push_back({gi, false});
            pending[a].clear();
            return;
        }
        if (pending[a].empty() && pending[b].empty()) return;
        Synth sy;
        sy.op = qf_op{};
        sy.op.kind = QF_OP_U;
        sy.op.q0 = a;
        sy.op.q1 = 2;
        sy.op.param = -1;
        sy.run0 = pending[a];
        sy.run1 = pending[b];
        sy.real = true;
        for (int gi : sy.run0) sy.real = sy.real && p->gates[gi].op.kind == QF_OP_RY;
        for (int gi : sy.run1) sy.real = sy.real && p->gates[gi].op.kind == QF_OP_RY;
        p->synth.push_back(sy);
        seq.push_back({ng + int(p->synth.size()) - 1, false});
        pending[a].clear();
        pending[b].clear();
    };
    std::vector<Touch> tv;
    for (int gi = lo; gi < hi; ++gi) {
        const qf_op& o = p->gates[gi].op;
        if (is_1q(o.kind)) {
            pending[o.q0].push_back(gi);
            continue;
        }
        touches(o, tv);
        for (const Touch& t : tv) flush_pair(t.q / 2);
        seq.push_back({gi, false});
    }
    for (int pr = 0; 2 * pr < n; ++pr) flush_pair(pr);
}

// Qudit that must be inside the tile (-1: none; CZ acts on any digits).
static int local_need(const qf_op& o) {
    if (is_1q(o.kind) || o.kind == QF_OP_X) return o.q0;
    if (o.kind == QF_OP_CSUM || o.kind == QF_OP_CSHIFT) return o.q1;
    return -1;
}

// Default register group size per D (best of a sweep on MI355X, complex64,
// at the default tile size).
static int default_group(int D, int dtype) {
    (void)dtype;
    return std::min(max_group_size(uint32_t(D)), D == 2 ? 4 : D <= 5 ? 2 : 1);
}

static void tile_shape(int D, int n, int dtype, int tile_opt, int low_opt, bool adjoint, int& k, int& r) {
    const size_t esz = dtype == QF_C64 ? 8 : 16;
    // Default tile: at most 32 KB of forward amplitudes (measured best for
    // D = 3, 5 on MI355X: several workgroups per CU overlap their load, compute
    // and store phases); the adjoint holds psi and lam tiles in 40 KB (D = 3:
    // 7 qudits; D = 5: 4 qudits, 2.4x faster per pass than 5 qudits in 50 KB),
    // 64 KB for D = 4 (6 qudits: 15% faster than 5 on batches of 4^8 registers).
    const size_t budget = (adjoint ? (D == 4 ? 64 : 40) * 1024 : 32 * 1024);
    if (tile_opt > 0) {
        k = tile_opt;
    } else {
        k = 1;
        while (size_t(ipow(D, k + 1)) * esz * (adjoint ? 2 : 1) <= budget && k + 1 <= n) ++k;
    }
    if (k >= n) {
        k = n;
        r = n;
        return;
    }
    if (low_opt > 0) {
        r = low_opt;
    } else {
        // the smallest r whose runs fill a 64-byte segment; qf_plan_create may
        // raise it (choose_low)
        r = 1;
        while (size_t(ipow(D, r)) * esz < 64 && r + 1 < k) ++r;
    }
    if (r >= k) r = k - 1;
    while (ipow(D, k - r) > uint32_t(kMaxHi)) ++r;
}

static void make_geom(int D, int n, int k, int r, const std::vector<int>& T, StageGeom& g) {
    g = StageGeom{};
    std::vector<bool> in(n, false);
    for (int q : T) in[q] = true;
    // the tile's HBM runs: the longest stretch of lowest qudits it holds (at
    // least the r it was planned with), shorter than the 256-lane workgroup
    // (longer runs take fewer, fuller memory requests; the LDS layout does not
    // depend on r)
    while (r < k && in[size_t(n - 1 - r)] && ipow(D, r + 1) < 256u) ++r;
    g.k = k;
    g.r = r;
    g.TE = ipow(D, k);
    g.R = ipow(D, r);
    g.nhi = ipow(D, k - r);
    g.ntiles = ipow(D, n - k);
    g.N = ipow(D, n);
    g.nout = n - k;
    g.divR.init(g.R);
    int h = 0;
    for (int q : T)
        if (q < n - r) g.hi_stride[h++] = ipow(D, n - 1 - q);
    int o = 0;
    for (int q = 0; q < n; ++q)
        if (!in[q]) g.out_stride[o++] = ipow(D, n - 1 - q);
}

// Gates a pass over tile inT would take: every remaining gate (from index
// first on) whose target is in the tile and that commutes with every gate left
// behind so far (two gates commute when every qudit they share is one on which
// both act block-diagonally).  Returns the count of multi-qudit gates taken in
// the high 32 bits and the count of all gates taken in the low 32 bits.
static uint64_t pass_take(const qf_plan* p, const std::vector<GRef>& seq, const std::vector<char>& done, int first,
                          const std::vector<char>& inT, std::vector<char>& bFull, std::vector<char>& bDiag,
                          std::vector<Touch>& tv) {
    std::fill(bFull.begin(), bFull.end(), 0);
    std::fill(bDiag.begin(), bDiag.end(), 0);
    uint64_t multi = 0, all = 0;
    int nfull = 0;
    const int n = int(bFull.size());
    for (int i = first; i < int(seq.size()) && nfull < n; ++i) {
        if (done[i]) continue;
        const qf_op& o = op_of(p, seq[i]);
        touches(o, tv);
        bool conflict = false;
        for (const Touch& t : tv) conflict = conflict || bFull[t.q] || (!t.diag && bDiag[t.q]);
        const int need = local_need(o);
        if (!conflict && !pass_gate(o.kind) && (need < 0 || inT[need])) {
            ++all;
            multi += tv.size() > 1 ? 1 : 0;
        } else {
            for (const Touch& t : tv) {
                if (t.diag) {
                    bDiag[t.q] = 1;
                } else if (!bFull[t.q]) {
                    bFull[t.q] = 1;
                    ++nfull;  // once every qudit is blocked no later gate can be taken
                }
            }
        }
    }
    return (multi << 32) | all;
}

// Greedy stage builder over a gate sequence.  Each pass picks a tile of k
// qudits (the low r qudits plus the qudits the earliest remaining gates need),
// then takes the gates pass_take admits, in order.  With climb set, the tile is
// then improved by single swaps of a non-low qudit in for one out (the qudit
// the first remaining gate needs stays), each taken when it raises the number
// of multi-qudit gates the pass takes, then the number of all gates: the
// entangling gates are the chain that orders a circuit's layers, so a tile that
// advances that chain further leaves less for later passes.
// Gate visits the swap climb may spend on one gate sequence; past it the
// remaining passes keep their greedy tiles (bounds the planning time of very
// long circuits on many qudits).
constexpr uint64_t kClimbBudget = uint64_t(1) << 27;

static void plan_passes_one(const qf_plan* p, const std::vector<GRef>& seq, int k, int r, int seg, bool climb,
                            std::vector<Pass>& out) {
    const int n = p->n;
    const int m = int(seq.size());
    std::vector<char> done(m, 0);
    int remaining = m, first = 0;
    std::vector<Touch> tv;
    std::vector<char> tb0(n), tb1(n);
    uint64_t spent = 0;
    while (remaining > 0) {
        while (done[first]) ++first;
        const qf_op& o0 = op_of(p, seq[first]);
        if (pass_gate(o0.kind)) {
            Pass pf;
            pf.tile = false;
            pf.fused = seq[first];
            pf.seg = seg;
            done[first] = 1;
            --remaining;
            out.push_back(pf);
            continue;
        }
        std::vector<char> inT(n, 0);
        int cnt = 0;
        for (int q = n - r; q < n; ++q) inT[q] = 1, ++cnt;
        for (int i = first; i < m && cnt < k; ++i) {
            if (done[i]) continue;
            const int q = local_need(op_of(p, seq[i]));
            if (q >= 0 && !inT[q]) inT[q] = 1, ++cnt;
        }
        for (int q = n - r - 1; q >= 0 && cnt < k; --q)
            if (!inT[q]) inT[q] = 1, ++cnt;
        if (climb && spent < kClimbBudget) {
            const int keep = local_need(o0);
            uint64_t best = pass_take(p, seq, done, first, inT, tb0, tb1, tv);
            for (bool improved = true; improved && spent < kClimbBudget;) {
                improved = false;
                for (int a = 0; a < n - r && !improved; ++a) {
                    if (!inT[a] || a == keep) continue;
                    for (int b = 0; b < n - r && !improved; ++b) {
                        if (inT[b]) continue;
                        inT[a] = 0;
                        inT[b] = 1;
                        spent += uint64_t(m - first);
                        const uint64_t sc = pass_take(p, seq, done, first, inT, tb0, tb1, tv);
                        if (sc > best) {
                            best = sc;
                            improved = true;
                        } else {
                            inT[a] = 1;
                            inT[b] = 0;
                        }
                    }
                }
            }
        }
        Pass ps;
        ps.seg = seg;
        for (int q = 0; q < n; ++q)
            if (inT[q]) ps.T.push_back(q);
        make_geom(p->D, n, k, r, ps.T, ps.geom);
        ps.geom.xcd = p->opts.tile_order == 0 ? 1u : 0u;
        std::vector<char> bFull(n, 0), bDiag(n, 0);
        std::vector<std::vector<GRef>> pending(n);
        auto flush = [&](int q) {
            if (pending[q].empty()) return;
            HOp h;
            h.type = SOP_U;
            h.q = q;
            h.g = pending[q];
            ps.ops.push_back(h);
            pending[q].clear();
        };
        for (int i = first; i < m; ++i) {
            if (done[i]) continue;
            const qf_op& o = op_of(p, seq[i]);
            touches(o, tv);
            bool conflict = false;
            for (const Touch& t : tv) conflict = conflict || bFull[t.q] || (!t.diag && bDiag[t.q]);
            const int need = local_need(o);
            const bool local = !pass_gate(o.kind) && (need < 0 || inT[need]);
            if (!conflict && local) {
                done[i] = 1;
                --remaining;
                if (is_1q(o.kind)) {
                    pending[o.q0].push_back(seq[i]);
                    continue;
                }
                for (const Touch& t : tv) flush(t.q);
                if (o.kind == QF_OP_CZ) {
                    if (!ps.ops.empty() && ps.ops.back().type == SOP_PHASE && int(ps.ops.back().g.size()) < kMaxPairs) {
                        ps.ops.back().g.push_back(seq[i]);
                    } else {
                        HOp h;
                        h.type = SOP_PHASE;
                        h.g = {seq[i]};
                        ps.ops.push_back(h);
                    }
                } else {
                    HOp h;
                    h.type = SOP_SHIFT;
                    h.q = (o.kind == QF_OP_X) ? o.q0 : o.q1;
                    h.ctrl = (o.kind == QF_OP_X) ? -1 : o.q0;
                    h.g = {seq[i]};
                    ps.ops.push_back(h);
                }
            } else {
                for (const Touch& t : tv) (t.diag ? bDiag : bFull)[t.q] = 1;
            }
        }
        for (int q = 0; q < n; ++q) flush(q);
        out.push_back(ps);
    }
}

// Passes of one gate sequence: the greedy plan, and (tile_search 0: for
// states of at least 2^20 amplitudes, where every pass is a full sweep of HBM;
// 2: at any size) also the climbed one; the plan with fewer passes is kept
// (ties: the greedy plan).
static void plan_passes(const qf_plan* p, const std::vector<GRef>& seq, int k, int r, int seg, PassList& out) {
    std::vector<Pass> greedy;
    plan_passes_one(p, seq, k, r, seg, false, greedy);
    double amps = 1;
    for (int i = 0; i < p->n; ++i) amps *= p->D;
    const int search = p->opts.tile_search;
    if (search != 1 && (search == 2 || amps >= double(1 << 20)) && r < p->n && k < p->n) {
        std::vector<Pass> climbed;
        plan_passes_one(p, seq, k, r, seg, true, climbed);
        if (climbed.size() < greedy.size()) greedy.swap(climbed);
    }
    for (Pass& ps : greedy) out.passes.push_back(std::move(ps));
}

// Number of low qudits of the tiles: fewer low qudits leave more tile qudits to
// the gates and so fewer passes, at the price of shorter contiguous runs (the
// XCD-grouped tile order keeps neighbouring tiles' shared cache lines in one
// L2).  Among r0 .. r0 + 3, the r with the fewest passes is taken; ties go to
// the longer runs.
static int choose_low(const qf_plan* p, const std::vector<std::vector<GRef>>& seqs, int k, int r0, bool adjoint) {
    if (r0 >= k) return r0;
    int best = r0;
    size_t best_passes = SIZE_MAX;
    for (int r = r0; r < k && r <= r0 + 3; ++r) {
        PassList trial;
        if (adjoint)
            for (int sgi = int(seqs.size()) - 1; sgi >= 0; --sgi) plan_passes(p, seqs[sgi], k, r, sgi, trial);
        else
            for (size_t sgi = 0; sgi < seqs.size(); ++sgi) plan_passes(p, seqs[sgi], k, r, int(sgi), trial);
        if (trial.passes.size() <= best_passes) {
            best_passes = trial.passes.size();
            best = r;
        }
    }
    return best;
}

static Mat group_matrix(const qf_plan* p, const std::vector<GRef>& g, const double* theta) {
    Mat U = identity(p->D);
    for (const GRef& r : g) {
        Mat G = gate_matrix(p->gates[r.gi].op, p->D, theta);
        if (r.inv) G = dagger(G, p->D);
        U = matmul(G, U, p->D);
    }
    return U;
}

// Register rounds of a tile pass.  A round starts with up to two SHIFT ops
// folded into its loads (pre0: target on group position 0, control outside
// the group or none; pre1: target on position 1, control on position 0; a
// single leading SHIFT whose control is a tile qudit is taken as pre1), takes
// consecutive in-place ops (U, PHASE) while the U targets fit in a group of M
// tile qudits, and may end with one SHIFT folded into its stores (post: target
// on position 0, control on position 1, outside the group or none).  In
// forward lists with groups of 2 and at most 256 sub-tiles, U on a, then
// SHIFT x_t += s(x_c), then U on c (a, c, t different, t outside the group, c
// on group position 1) is taken as one round: U on a commutes with the SHIFT,
// which moves before it and into the loads (pre2), and the two U make a pair.  The group is padded
// with unused tile qudits.  Adjoint lists: a U that owns an M slot
// opens its round (no SHIFT before it in the round).
static void build_rounds(const qf_plan* p, Pass& ps, PassList& L, const std::vector<int>& dim_of, size_t& moff,
                         bool adjoint) {
    const int D = p->D;
    const int k = int(ps.geom.k);
    const int M = adjoint ? adj_group(p) : p->group;
    ps.nrounds = 0;
    ps.round_off = int(L.hrounds.size());
    // rounds address at most 8 other tile qudits (sub_base); larger tiles run op by op
    if (k < M || k - M > 8 || ps.ops.empty()) return;
    const size_t nops = ps.ops.size();
    auto has = [](const std::vector<int>& v, int d) { return std::find(v.begin(), v.end(), d) != v.end(); };
    auto ctrl_dim = [&](const HOp& h) { return h.ctrl >= 0 ? dim_of[h.ctrl] : -1; };  // -1: none or outside
    auto slotted = [&](size_t j) { return adjoint && ps.ops[j].type == SOP_U && L.hops[ps.op_off + j].slot >= 0; };
    // pre2 rounds (forward lists, groups of 2): the kernel keeps one sub-tile
    // per lane of its 256-lane workgroup across a barrier
    const bool pre2_ok = !adjoint && M == 2 && ipow(D, k - M) <= 256;
    size_t i = 0;
    while (i < nops) {
        std::vector<int> front;  // fixed group positions 0, 1, ...
        std::vector<int> rest;   // other group qudits (U targets)
        int pre0 = -1, pre1 = -1, pre2 = -1, post = -1;
        size_t j = i;
        if (ps.ops[j].type == SOP_SHIFT) {
            const int t = dim_of[ps.ops[j].q], c = ctrl_dim(ps.ops[j]);
            if (M >= 2 && c >= 0) {
                front = {c, t};
                pre1 = int(j);
                ++j;
            } else {
                front = {t};
                pre0 = int(j);
                ++j;
                if (M >= 2 && j < nops && ps.ops[j].type == SOP_SHIFT && ctrl_dim(ps.ops[j]) == t &&
                    dim_of[ps.ops[j].q] != t) {
                    front.push_back(dim_of[ps.ops[j].q]);
                    pre1 = int(j);
                    ++j;
                }
            }
        }
        const size_t ip0 = j;
        size_t ipe = j;
        auto members = [&]() {
            std::vector<int> m = front;
            m.insert(m.end(), rest.begin(), rest.end());
            return m;
        };
        // groups of at most 2 qudits take only the dispatch-free shapes: one U,
        // one PHASE, or two complex U on different qudits (the kernels compile
        // the generic interpreter for larger groups only)
        const bool small = M <= 2;
        auto is_real_u = [&](size_t x) { return L.hops[ps.op_off + x].real != 0; };
        for (; j < nops; ++j) {
            const HOp& h = ps.ops[j];
            if (j > i && slotted(j)) break;
            const size_t nin = j - ip0;  // in-place ops taken so far
            if (h.type == SOP_PHASE) {
                if (small && nin > 0) break;
                ipe = j + 1;
                continue;
            }
            if (h.type == SOP_U) {
                if (small && nin > 0) {
                    const HOp& f = ps.ops[ip0];
                    const bool pair_ok = M == 2 && nin == 1 && f.type == SOP_U && f.q != h.q && !is_real_u(ip0) &&
                                         !is_real_u(j);
                    if (!pair_ok) break;
                }
                const int d = dim_of[h.q];
                const std::vector<int> m = members();
                if (!has(m, d)) {
                    if (int(m.size()) == M) break;
                    rest.push_back(d);
                }
                ipe = j + 1;
                continue;
            }
            const int t = dim_of[h.q], c = ctrl_dim(h);
            // U on a, SHIFT c -> t, U on c: the SHIFT becomes pre2 and the U a pair
            if (pre2_ok && nin == 1 && pre2 < 0 && c >= 0 && j + 1 < nops && ps.ops[ip0].type == SOP_U) {
                const HOp& nx = ps.ops[j + 1];
                const int a = dim_of[ps.ops[ip0].q];
                const std::vector<int> m = members();
                const bool pair = nx.type == SOP_U && dim_of[nx.q] == c && !slotted(j + 1) && !is_real_u(ip0) &&
                                  !is_real_u(j + 1);
                // the control lands on group position 1 (the kernel reads it there)
                const int cpos = has(m, c) ? int(std::find(m.begin(), m.end(), c) - m.begin()) : int(m.size());
                const bool fits = cpos == 1;
                const int lane_ctrl = pre0 >= 0 ? ctrl_dim(ps.ops[size_t(pre0)]) : -2;
                if (pair && fits && a != c && a != t && c != t && !has(m, t) && lane_ctrl != t && lane_ctrl != c) {
                    if (!has(m, c)) rest.push_back(c);
                    pre2 = int(j);
                    ++j;         // the loop's ++j passes the second U
                    ipe = j + 1;
                    continue;
                }
            }
            // a SHIFT after the in-place ops: post if it fits
            if (front.empty()) {
                std::vector<int> r2, r1;
                for (int d : rest) {
                    if (d != t && d != c) r2.push_back(d);
                    if (d != t) r1.push_back(d);
                }
                if (c >= 0 && M >= 2 && int(r2.size()) + 2 <= M) {
                    front = {t, c};
                    rest = r2;
                } else if (int(r1.size()) + 1 <= M && !has(r1, c)) {
                    front = {t};
                    rest = r1;
                } else {
                    break;
                }
            } else {
                // positions are fixed: the target must be position 0 and the
                // control position 1 or outside the group
                const std::vector<int> m = members();
                if (front[0] != t) break;
                const bool c_at1 = m.size() >= 2 && c >= 0 && m[1] == c;
                if (!c_at1 && c >= 0 && has(m, c)) break;
                if (!c_at1 && c >= 0 && int(m.size()) < M) break;  // padding could place it in the group
            }
            post = int(j);
            ++j;
            break;
        }
        std::vector<int> grp = members();
        auto pad = [&](int d) { return !has(grp, d); };
        for (int d = 0; int(grp.size()) < M && d < k; ++d) {
            // never pad with the control of a per-lane permutation (its digit must stay outside)
            bool lane_ctrl = false;
            for (int pi : {pre0, post})
                if (pi >= 0 && ctrl_dim(ps.ops[size_t(pi)]) == d) lane_ctrl = true;
            if (pad(d) && !lane_ctrl) grp.push_back(d);
        }
        RoundDesc rd{};
        rd.op0 = int(ip0);
        rd.nops = int(ipe - ip0);
        rd.pre0 = pre0;
        rd.pre1 = pre1;
        rd.post = post;
        const uint32_t esz = p->dtype == QF_C64 ? 8u : 16u;
        for (int g = 0; g < M; ++g) {
            rd.gls[g] = ipow(D, k - 1 - grp[g]);
            rd.glsb[g] = rd.gls[g] * esz;
        }
        rd.nother = k - M;
        int o = 0;
        for (int d = 0; d < k; ++d)
            if (!has(grp, d)) rd.ols[o++] = ipow(D, k - 1 - d);
        for (int i = 0; i < 8 && i < rd.nother; ++i)  // strides < 2^16 (tiles hold < 2^16 amplitudes per LDS budget)
            rd.spair[i / 2] |= (rd.ols[rd.nother - 1 - i] & 0xffffu) << (16 * (i % 2));
        auto gpos_of_qudit = [&](int q) -> int {
            if (q < 0 || dim_of[q] < 0) return -1;
            auto it = std::find(grp.begin(), grp.end(), dim_of[q]);
            return it == grp.end() ? -1 : int(it - grp.begin());
        };
        bool need = false;
        for (size_t oi = ip0; oi < ipe; ++oi) {
            const HOp& h = ps.ops[oi];
            StageOp& so = L.hops[ps.op_off + oi];
            so.gpos = h.type == SOP_PHASE ? -1 : gpos_of_qudit(h.q);
            so.ctrl_gpos = -1;
            if (h.type == SOP_PHASE) {
                for (size_t pi = 0; pi < h.g.size(); ++pi) {
                    const qf_op& g = p->gates[h.g[pi].gi].op;
                    so.agpos[pi] = gpos_of_qudit(g.q0);
                    so.bgpos[pi] = gpos_of_qudit(g.q1);
                    need = need || so.agpos[pi] < 0 || so.bgpos[pi] < 0;
                }
                so.wtab = int(moff);
                moff += size_t(D);
            }
        }
        for (int pi : {pre0, pre1, post}) {
            if (pi < 0) continue;
            const HOp& h = ps.ops[size_t(pi)];
            StageOp& so = L.hops[ps.op_off + pi];
            so.gpos = gpos_of_qudit(h.q);
            so.ctrl_gpos = gpos_of_qudit(h.ctrl);
            need = need || (so.has_ctrl && so.ctrl_gpos < 0);
        }
        rd.need_gidx = need ? 1 : 0;
        rd.kind = RK_GENERIC;
        if (rd.nops == 0) {
            rd.kind = RK_NONE;
        } else if (rd.nops <= 2) {
            bool allu = true, anyreal = false;
            int posmask = 0;
            for (size_t oi = ip0; oi < ipe; ++oi) {
                const StageOp& so = L.hops[ps.op_off + oi];
                allu = allu && so.type == SOP_U;
                anyreal = anyreal || so.real;
                if (so.type == SOP_U && so.gpos >= 0 && so.gpos < 2) posmask |= 1 << so.gpos;
            }
            if (allu && rd.nops == 1 && posmask == 1) rd.kind = anyreal ? RK_U0_REAL : RK_U0;
            if (allu && rd.nops == 1 && posmask == 2 && M >= 2) rd.kind = anyreal ? RK_U1_REAL : RK_U1;
            if (rd.nops == 1 && L.hops[ps.op_off + ip0].type == SOP_PHASE) rd.kind = RK_PHASE;
            if (allu && rd.nops == 2 && posmask == 3 && !anyreal && M >= 2) rd.kind = RK_U01;
        }
        rd.pre2 = pre2;
        if (pre2 >= 0) {
            // ops: U, the pre2 SHIFT, U
            const StageOp& ua = L.hops[ps.op_off + ip0];
            const StageOp& ub = L.hops[ps.op_off + ip0 + 2];
            const StageOp& sh = L.hops[ps.op_off + size_t(pre2)];
            const HOp& h = ps.ops[size_t(pre2)];
            rd.kind = RK_U01;
            rd.mat0 = ua.gpos == 0 ? ua.mat : ub.mat;
            rd.mat1 = ua.gpos == 0 ? ub.mat : ua.mat;
            const int t = dim_of[h.q];
            int ot = 0;  // t's index among the other tile qudits (ols order)
            for (int d = 0; d < t; ++d)
                if (!has(grp, d)) ++ot;
            rd.pre2_byte = rd.nother - 1 - ot;
            rd.pre2_lsb = ipow(D, k - 1 - t) * esz;
            for (int c = 0; c < 16; ++c) rd.pre2_shifts[c] = sh.shifts[c];
        }
        if (pre2 < 0 && (rd.kind == RK_U0 || rd.kind == RK_U0_REAL || rd.kind == RK_U1 || rd.kind == RK_U1_REAL ||
                         rd.kind == RK_U01)) {
            const StageOp& a = L.hops[ps.op_off + ip0];
            rd.mat0 = rd.mat1 = a.mat;
            if (rd.kind == RK_U01) {
                const StageOp& b = L.hops[ps.op_off + ip0 + 1];
                // the two U act on different qudits and commute: mat0 is position 0's
                if (a.gpos == 0) {
                    rd.mat1 = b.mat;
                } else {
                    rd.mat0 = b.mat;
                    rd.mat1 = a.mat;
                }
            }
        }
        rd.mslot = rd.mpos = -1;
        if (rd.nops > 0 && pre0 < 0 && pre1 < 0) {
            const StageOp& so = L.hops[ps.op_off + ip0];
            if (so.type == SOP_U && so.slot >= 0) {
                rd.mslot = so.slot;
                rd.mpos = so.gpos;
            }
        }
        {
            const int perm_ops[3] = {pre0, pre1, post};
            for (int j = 0; j < 3; ++j) {
                if (perm_ops[j] < 0) continue;
                const StageOp& so = L.hops[ps.op_off + size_t(perm_ops[j])];
                PermDesc& pd = rd.perm[j];
                pd.has_ctrl = so.has_ctrl;
                pd.ctrl_gpos = so.ctrl_gpos;
                pd.shift_mul = so.shift_mul;
                pd.ctrl_stride = so.ctrl_stride;
                for (int c = 0; c < 16; ++c) pd.shifts[c] = so.shifts[c];
            }
        }
        if (M <= 2 && rd.kind == RK_GENERIC) {
            // the shape rules above exclude this; should it happen, the pass
            // runs op by op (the round kernels for M <= 2 have no interpreter)
            L.hrounds.resize(size_t(ps.round_off));
            ps.nrounds = 0;
            return;
        }
        L.hrounds.push_back(rd);
        ++ps.nrounds;
        i = j;
    }
}

// Moves every U of a stage up to right after the last earlier op that touches
// its qudit (it commutes with the ops it passes, which act on other qudits), so
// that it meets the SHIFT ops around its qudit in the same register round.
static void hoist_u(const qf_plan* p, std::vector<HOp>& ops) {
    auto touches_q = [&](const HOp& h, int q) {
        if (h.type == SOP_U) return h.q == q;
        if (h.type == SOP_SHIFT) return h.q == q || h.ctrl == q;
        for (const GRef& r : h.g) {
            const qf_op& g = p->gates[r.gi].op;
            if (g.q0 == q || g.q1 == q) return true;
        }
        return false;
    };
    for (size_t idx = 1; idx < ops.size(); ++idx) {
        if (ops[idx].type != SOP_U) continue;
        const int q = ops[idx].q;
        for (size_t j = idx; j > 0 && !touches_q(ops[j - 1], q); --j) std::swap(ops[j - 1], ops[j]);
    }
}

// Static part of the stage ops; matrix offsets; M slots (for adjoint lists).
static void finalize_passes(const qf_plan* p, PassList& L, bool adjoint) {
    const int D = p->D, n = p->n;
    L.hops.clear();
    L.hrounds.clear();
    L.nmats = 0;
    L.nslots = 0;
    L.ncr = 0;
    const int ng = int(p->gates.size());
    for (Pass& ps : L.passes) {
        if (!ps.tile) {
            if (ps.fused.gi >= ng) {  // synthetic pair block: its D^2 x D^2 matrix lives in the pass mats
                ps.mat_off = L.nmats;
                ps.nmat = size_t(D) * D * D * D;
                L.nmats += ps.nmat;
            } else if (is_crot(p->gates[ps.fused.gi].op.kind)) {  // controlled rotation: its 2 D table
                ps.mat_off = L.nmats;
                ps.nmat = size_t(2) * D;
                L.nmats += ps.nmat;
                ps.cr_slot = L.ncr++;
            }
            continue;
        }
        hoist_u(p, ps.ops);
        ps.op_off = int(L.hops.size());
        ps.mat_off = L.nmats;
        ps.nslots = 0;
        ps.slot0 = L.nslots;
        size_t moff = 0;
        std::vector<int> dim_of(n, -1);
        for (size_t i = 0; i < ps.T.size(); ++i) dim_of[ps.T[i]] = int(i);
        const int k = int(ps.geom.k);
        for (HOp& h : ps.ops) {
            StageOp so{};
            so.type = h.type;
            so.slot = -1;
            if (h.type == SOP_U || h.type == SOP_SHIFT) {
                so.dim = dim_of[h.q];
                so.ls = ipow(D, k - 1 - so.dim);
                so.divls.init(so.ls);
            }
            if (h.type == SOP_U) {
                so.mat = int(moff);
                moff += size_t(D) * D;
                bool real = true, rot = false;
                for (const GRef& r : h.g) {
                    const int kind = p->gates[r.gi].op.kind;
                    real = real && kind == QF_OP_RY;
                    rot = rot || is_rot(kind);
                }
                so.real = real;
                if (adjoint && rot) {
                    h.slot = ps.nslots++;
                    h.gslot = L.nslots++;
                    so.slot = h.slot;
                }
            } else if (h.type == SOP_SHIFT) {
                const GRef& r = h.g[0];
                const qf_op& o = p->gates[r.gi].op;
                so.has_ctrl = h.ctrl >= 0;
                so.ctrl_stride.init(h.ctrl >= 0 ? ipow(D, n - 1 - h.ctrl) : 1u);
                for (int c = 0; c < D; ++c) {
                    const int v = shift_of(o, c, D);
                    so.shifts[c] = r.inv ? (D - v) % D : v;
                }
                so.shift_mul = -1;
                for (int a = 0; a < D && so.shift_mul < 0; ++a) {
                    bool ok = true;
                    for (int c = 0; c < D; ++c) ok = ok && so.shifts[c] == (a * c + so.shifts[0]) % D;
                    if (ok) so.shift_mul = a;
                }
            } else {
                so.npairs = int(h.g.size());
                for (size_t j = 0; j < h.g.size(); ++j) {
                    const qf_op& o = p->gates[h.g[j].gi].op;
                    so.pa[j].init(ipow(D, n - 1 - o.q0));
                    so.pb[j].init(ipow(D, n - 1 - o.q1));
                    so.ptab[j] = int(moff);
                    moff += size_t(D) * D;
                }
            }
            L.hops.push_back(so);
        }
        ps.nops = int(ps.ops.size());
        build_rounds(p, ps, L, dim_of, moff, adjoint);
        ps.nmat = moff;
        L.nmats += moff;
    }
}

static qf_status upload_ops(const qf_plan* p, PassList& L) {
    const size_t esz = p->dtype == QF_C64 ? 8 : 16;
    if (!L.hops.empty()) {
        QF_CHECK(dev_malloc(reinterpret_cast<void**>(&L.dops), L.hops.size() * sizeof(StageOp), "stage ops"));
        QF_HIP_CHECK(hipMemcpy(L.dops, L.hops.data(), L.hops.size() * sizeof(StageOp), hipMemcpyHostToDevice));
    }
    if (!L.hrounds.empty()) {
        QF_CHECK(dev_malloc(reinterpret_cast<void**>(&L.drounds), L.hrounds.size() * sizeof(RoundDesc), "rounds"));
        QF_HIP_CHECK(hipMemcpy(L.drounds, L.hrounds.data(), L.hrounds.size() * sizeof(RoundDesc),
                               hipMemcpyHostToDevice));
    }
    const size_t mb = std::max<size_t>(L.nmats, 1) * esz;
    QF_CHECK(dev_malloc(&L.dmats, mb, "stage matrices"));
    QF_CHECK(host_malloc_pinned(&L.hmats, mb, "stage matrix staging"));
    QF_HIP_CHECK(hipEventCreateWithFlags(&L.copied, hipEventDisableTiming));
    QF_HIP_CHECK(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
    return QF_OK;
}

template <typename T>
static void put_mat(void* base, size_t off, const Mat& m) {
    cplx<T>* d = reinterpret_cast<cplx<T>*>(base) + off;
    for (size_t i = 0; i < m.size(); ++i) d[i] = cmake<T>(T(m[i].real()), T(m[i].imag()));
}

// Build every stage matrix from theta into the pinned staging buffer and copy it
// to the device on `st`.
static qf_status upload_mats(const qf_plan* p, PassList& L, const double* theta, hipStream_t st) {
    if (L.dmats == nullptr) QF_CHECK(upload_ops(p, L));
    if (L.copied_valid) QF_HIP_CHECK(hipEventSynchronize(L.copied));
    const int D = p->D;
    const int ng = int(p->gates.size());
    for (const Pass& ps : L.passes) {
        if (!ps.tile) {
            if (ps.fused.gi >= ng) {
                const Synth& sy = p->synth[ps.fused.gi - ng];
                Mat A = identity(D), B = identity(D);
                for (int gi : sy.run0) A = matmul(gate_matrix(p->gates[gi].op, D, theta), A, D);
                for (int gi : sy.run1) B = matmul(gate_matrix(p->gates[gi].op, D, theta), B, D);
                const int K = D * D;
                Mat Kr(size_t(K) * K);
                for (int a0 = 0; a0 < D; ++a0)
                    for (int b0 = 0; b0 < D; ++b0)
                        for (int a1 = 0; a1 < D; ++a1)
                            for (int b1 = 0; b1 < D; ++b1)
                                Kr[size_t(a0 * D + b0) * K + (a1 * D + b1)] = A[a0 * D + a1] * B[b0 * D + b1];
                if (p->dtype == QF_C64)
                    put_mat<float>(L.hmats, ps.mat_off, Kr);
                else
                    put_mat<double>(L.hmats, ps.mat_off, Kr);
            } else if (ps.cr_slot >= 0) {
                std::vector<double> tab;
                crot_table(p->gates[ps.fused.gi].op, D, theta, ps.fused.inv, tab);
                Mat t(size_t(2) * D);
                for (size_t i = 0; i < t.size(); ++i) t[i] = cd(tab[2 * i], tab[2 * i + 1]);
                if (p->dtype == QF_C64)
                    put_mat<float>(L.hmats, ps.mat_off, t);
                else
                    put_mat<double>(L.hmats, ps.mat_off, t);
            }
            continue;
        }
        for (size_t i = 0; i < ps.ops.size(); ++i) {
            const HOp& h = ps.ops[i];
            const StageOp& so = L.hops[ps.op_off + i];
            if (h.type == SOP_U) {
                const Mat U = group_matrix(p, h.g, theta);
                if (p->dtype == QF_C64)
                    put_mat<float>(L.hmats, ps.mat_off + so.mat, U);
                else
                    put_mat<double>(L.hmats, ps.mat_off + so.mat, U);
            } else if (h.type == SOP_PHASE) {
                for (size_t j = 0; j < h.g.size(); ++j) {
                    Mat t;
                    cz_table(D, D, h.g[j].inv, t);
                    if (p->dtype == QF_C64)
                        put_mat<float>(L.hmats, ps.mat_off + so.ptab[j], t);
                    else
                        put_mat<double>(L.hmats, ps.mat_off + so.ptab[j], t);
                }
                if (ps.nrounds > 0) {
                    // w^e for the summed exponent e of the op's CZ factors (all of one direction)
                    const double pi = 3.14159265358979323846;
                    const double sgn = h.g[0].inv ? -1.0 : 1.0;
                    Mat w(static_cast<size_t>(D));
                    for (int e = 0; e < D; ++e) w[e] = std::polar(1.0, sgn * 2 * pi * e / D);
                    if (p->dtype == QF_C64)
                        put_mat<float>(L.hmats, ps.mat_off + so.wtab, w);
                    else
                        put_mat<double>(L.hmats, ps.mat_off + so.wtab, w);
                }
            }
        }
    }
    if (L.done_valid) QF_HIP_CHECK(hipStreamWaitEvent(st, L.done, 0));
    const size_t esz = p->dtype == QF_C64 ? 8 : 16;
    if (L.nmats) QF_HIP_CHECK(hipMemcpyAsync(L.dmats, L.hmats, L.nmats * esz, hipMemcpyHostToDevice, st));
    QF_HIP_CHECK(hipEventRecord(L.copied, st));
    L.copied_valid = true;
    return QF_OK;
}

// ---- profiling ----

static qf_status prof_begin(qf_plan* p, hipStream_t st, hipEvent_t* a) {
    *a = nullptr;
    if (!p->profiling) return QF_OK;
    if (p->ev_used + 2 > p->ev_pool.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            QF_HIP_CHECK(hipEventCreate(&e));
            p->ev_pool.push_back(e);
        }
    }
    *a = p->ev_pool[p->ev_used++];
    QF_HIP_CHECK(hipEventRecord(*a, st));
    return QF_OK;
}

static qf_status prof_end(qf_plan* p, hipStream_t st, hipEvent_t a, int family, double bytes) {
    if (!p->profiling || a == nullptr) return QF_OK;
    hipEvent_t b = p->ev_pool[p->ev_used++];
    QF_HIP_CHECK(hipEventRecord(b, st));
    p->prof.push_back({family, bytes, a, b});
    return QF_OK;
}

// ---- checkpoints ----

static size_t state_bytes(const StateView& v) { return size_t(v.total) * (v.dtype == QF_C64 ? 8 : 16); }

static qf_status ensure_ckpt(qf_plan* p, const StateView& v) {
    const size_t nsave = p->seg_end.size() > 1 ? p->seg_end.size() - 1 : 0;
    const size_t need = nsave * state_bytes(v);
    if (need <= p->ckpt_bytes) return QF_OK;
    if (p->ckpt) QF_HIP_CHECK(hipFree(p->ckpt));
    p->ckpt = nullptr;
    p->ckpt_bytes = 0;
    p->ckpt_amps = nullptr;
    p->ckpt_batch = 0;
    QF_CHECK(dev_malloc(&p->ckpt, need, "checkpoints"));
    p->ckpt_bytes = need;
    return QF_OK;
}

// A checkpointed reverse walk re-anchors psi from the checkpoints of the last
// forward pass, so they must come from a forward pass of this very state
// buffer at this batch size.
static qf_status check_ckpt_source(const qf_plan* p, const StateView& v) {
    if (p->seg_end.size() <= 1) return QF_OK;
    QF_RETURN_IF(p->ckpt == nullptr || p->ckpt_amps == nullptr, QF_EINVAL,
                 "checkpointed plan: run the forward pass on this state first");
    QF_RETURN_IF(p->ckpt_amps != v.amps || p->ckpt_batch != v.batch, QF_EINVAL,
                 "checkpointed plan: the checkpoints hold the forward pass of another state buffer or batch size; "
                 "run the forward pass on this state first");
    QF_RETURN_IF((p->seg_end.size() - 1) * state_bytes(v) > p->ckpt_bytes, QF_EINVAL,
                 "checkpointed plan: checkpoint buffer smaller than this state");
    return QF_OK;
}

// One forward tile pass with the kernel the options select (register rounds,
// pipelined rounds or one sweep per op).
static qf_status launch_forward_pass(const qf_plan* p, const PassList& L, const Pass& ps, const StateView& v,
                                     const void* mats, size_t mat_stride, hipStream_t st) {
    const int kern = p->opts.stage_kernel;
    if (ps.nrounds > 0 && kern == 2 && p->group <= 3 && v.dtype == QF_C64 && p->D <= 12 && stage_pipe_ok(ps.geom))
        return launch_stage_pipe(v, p->group, ps.geom, L.drounds + ps.round_off, ps.nrounds, L.dops + ps.op_off, mats,
                                 p->opts.pipe_wgs > 0 ? p->opts.pipe_wgs : 4, st, mat_stride);
    if (ps.nrounds > 0 && kern != 1)
        return launch_stage_rounds(v, p->group, ps.geom, L.drounds + ps.round_off, ps.nrounds, L.dops + ps.op_off,
                                   mats, st, mat_stride);
    return launch_stage(v, ps.geom, L.dops + ps.op_off, ps.nops, mats, st, mat_stride);
}

static qf_status run_tile_pass(qf_plan* p, const PassList& L, const Pass& ps, const StateView& v, void* lam,
                               double* partial, hipStream_t st) {
    const size_t esz = p->dtype == QF_C64 ? 8 : 16;
    const void* mats = reinterpret_cast<const unsigned char*>(L.dmats) + ps.mat_off * esz;
    hipEvent_t a;
    QF_CHECK(prof_begin(p, st, &a));
    if (lam == nullptr) {
        QF_CHECK(launch_forward_pass(p, L, ps, v, mats, 0, st));
        QF_CHECK(prof_end(p, st, a, F_STAGE, 2.0 * state_bytes(v)));
    } else {
        if (ps.nrounds > 0 && p->opts.stage_kernel != 1)
            QF_CHECK(launch_stage_adj_rounds(v, lam, adj_group(p), ps.geom, L.drounds + ps.round_off,
                                             ps.nrounds, L.dops + ps.op_off, mats, partial, st));
        else
            QF_CHECK(launch_stage_adj(v, lam, ps.geom, L.dops + ps.op_off, ps.nops, mats, partial, st));
        QF_CHECK(prof_end(p, st, a, F_STAGE_ADJ, 4.0 * state_bytes(v)));
    }
    return QF_OK;
}

static qf_status run_fused_pass(qf_plan* p, const PassList& L, const Pass& ps, const StateView& v, hipStream_t st) {
    const int ng = int(p->gates.size());
    hipEvent_t a;
    QF_CHECK(prof_begin(p, st, &a));
    if (ps.fused.gi >= ng) {
        const Synth& sy = p->synth[ps.fused.gi - ng];
        const size_t esz = p->dtype == QF_C64 ? 8 : 16;
        const void* m = reinterpret_cast<const unsigned char*>(L.dmats) + ps.mat_off * esz;
        QF_CHECK(launch_fused(v, 2, sy.op.q0, m, st, sy.real));
    } else if (ps.cr_slot >= 0) {
        const size_t esz = p->dtype == QF_C64 ? 8 : 16;
        const void* tab = reinterpret_cast<const unsigned char*>(L.dmats) + ps.mat_off * esz;
        QF_CHECK(launch_crot(v, crot_args(p->gates[ps.fused.gi].op), tab, 0, nullptr, st));
        return prof_end(p, st, a, F_CROT, 2.0 * state_bytes(v) * 2.0 / p->D);
    } else if (p->gates[ps.fused.gi].op.kind == QF_OP_SWAP || p->gates[ps.fused.gi].op.kind == QF_OP_MCX) {
        QF_CHECK(launch_perm_gate(v, p->gates[ps.fused.gi].op, ps.fused.inv, st));
        return prof_end(p, st, a, F_CTRL, 2.0 * state_bytes(v));
    } else {
        const Gate& g = p->gates[ps.fused.gi];
        QF_CHECK(launch_fused(v, g.op.q1, g.op.q0, ps.fused.inv ? g.dmat_adj : g.dmat, st, g.real));
    }
    return prof_end(p, st, a, F_FUSED, 2.0 * state_bytes(v));
}

static qf_status check_plan_state(const qf_plan* p, const qf_state* s, StateView& v) {
    QF_RETURN_IF(p == nullptr, QF_EINVAL, "plan is NULL");
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(int(v.D) != p->D || int(v.n) != p->n || v.dtype != p->dtype, QF_EINVAL,
                 "state (dim %u, n %u, dtype %d) does not match the plan (dim %d, n %d, dtype %d)", v.D, v.n, v.dtype,
                 p->D, p->n, p->dtype);
    for (int q = 0; q < p->n; ++q)
        QF_RETURN_IF(int(v.dims[q]) != p->dims[q], QF_EINVAL, "qudit %d has dimension %u in the state, %d in the plan",
                     q, v.dims[q], p->dims[q]);
    return QF_OK;
}

// Gradient contributions of one fused run of one-qudit gates from its M:
// dL/dtheta_i += Im Tr(V_i S_i V_i^dagger M), V_i = product of the run's gates
// after gate i (forward order), M = sum_f psi_f lam_f^dagger after the run.
static void add_group_grad(const qf_plan* p, const std::vector<int>& fwd_gates, const double* theta,
                           const double* M, double* grad) {
    const int D = p->dims[p->gates[fwd_gates[0]].op.q0];
    const int m = int(fwd_gates.size());
    std::vector<Mat> suffix(m + 1);
    suffix[m] = identity(D);
    for (int i = m - 1; i >= 0; --i)
        suffix[i] = matmul(suffix[i + 1], gate_matrix(p->gates[fwd_gates[i]].op, D, theta), D);
    for (int i = 0; i < m; ++i) {
        const qf_op& o = p->gates[fwd_gates[i]].op;
        if (!is_rot(o.kind)) continue;
        const Mat& V = suffix[i + 1];
        const Mat A = matmul(matmul(V, generator(o, D), D), dagger(V, D), D);
        cd tr(0, 0);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) tr += A[size_t(r) * D + c] * cd(M[2 * (c * D + r)], M[2 * (c * D + r) + 1]);
        grad[o.param] += tr.imag();
    }
}

// QF_CHECK_NORM=<tol>: after a forward pass, synchronise and check every
// register's norm (sum of |psi_x|^2 in FP64 by the expectation kernel with the
// constant observable 1).
static qf_status check_norm_env(const StateView& v, hipStream_t st) {
    const char* e = std::getenv("QF_CHECK_NORM");
    if (e == nullptr || e[0] == '\0') return QF_OK;
    const double tol = std::atof(e);
    if (!(tol > 0.0)) return QF_OK;
    std::vector<int> active{0};
    std::vector<double> table(2 * v.dims[0], 0.0);
    for (uint32_t d = 0; d < v.dims[0]; ++d) table[2 * d] = 1.0;
    double* out = nullptr;
    QF_CHECK(dev_malloc_async(reinterpret_cast<void**>(&out), size_t(v.batch) * 2 * sizeof(double), st, "norm check"));
    qf_status rs = launch_expect(v, active, table, out, st);
    std::vector<double> h(size_t(v.batch) * 2);
    if (rs == QF_OK && hipMemcpyAsync(h.data(), out, h.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
        rs = set_error(QF_EHIP, "norm check copy failed");
    (void)hipFreeAsync(out, st);
    if (hipStreamSynchronize(st) != hipSuccess && rs == QF_OK) rs = set_error(QF_EHIP, "norm check sync failed");
    if (rs != QF_OK) return rs;
    for (uint32_t b = 0; b < v.batch; ++b) {
        const double nrm = std::sqrt(h[2 * b]);
        QF_RETURN_IF(!(std::fabs(nrm - 1.0) <= tol), QF_ERANGE,
                     "QF_CHECK_NORM: register %u has norm %.9g after the forward pass (tolerance %g)", b, nrm, tol);
    }
    return QF_OK;
}

}  // namespace qf

using namespace qf;

extern "C" {

}  // extern "C"

// Plan creation for per-qudit dimensions; dim = the common dimension, or 0
// when they differ (then only the per-gate schedules exist).
static qf_status create_plan(const std::vector<int>& dims, int32_t dtype, const qf_op* ops, int32_t nops,
                             int32_t nparams, const qf_plan_opts* opts, qf_plan** out) {
    QF_RETURN_IF(out == nullptr, QF_EINVAL, "out is NULL");
    *out = nullptr;
    const int n = int(dims.size());
    QF_RETURN_IF(n < 1 || n > 32, QF_EINVAL, "n = %d outside 1..32", n);
    int dim = dims[0];
    for (int d : dims) {
        QF_RETURN_IF(d < 2 || d > kMaxDim, QF_ERANGE, "dim %d outside 2..%d", d, kMaxDim);
        if (d != dim) dim = 0;
    }
    const bool mixed = dim == 0;
    QF_RETURN_IF(dtype != QF_C64 && dtype != QF_C128, QF_EDTYPE, "unknown dtype %d", dtype);
    QF_RETURN_IF(nops < 0 || (nops > 0 && ops == nullptr), QF_EINVAL, "bad op list");
    QF_RETURN_IF(nparams < 0, QF_EINVAL, "nparams < 0");
    {
        uint64_t N = 1;
        for (int d : dims) N *= uint64_t(d);
        QF_RETURN_IF(N >= (1ull << 32), QF_ERANGE, "the register exceeds 2^32 amplitudes");
    }
    for (int i = 0; i < nops; ++i) {
        qf_status st = validate_op(ops[i], dims, nparams);
        if (st != QF_OK) return set_error(st, "op %d: %s", i, qf_last_error());
    }
    std::unique_ptr<qf_plan> p(new (std::nothrow) qf_plan);
    QF_RETURN_IF(!p, QF_ENOMEM, "plan allocation failed");
    p->D = dim;
    p->dims = dims;
    p->n = n;
    p->dtype = dtype;
    p->nparams = nparams;
    if (opts) p->opts = *opts;
    QF_RETURN_IF(p->opts.fuse < 0 || p->opts.fuse > 3, QF_EINVAL, "fuse = %d outside 0..3", p->opts.fuse);
    if (mixed) {
        // mixed dimensions: the per-gate schedules only
        if (p->opts.fuse == 0) p->opts.fuse = 2;
        QF_RETURN_IF(p->opts.fuse == 3, QF_EUNSUPPORTED, "fuse = 3 needs qudits of one dimension");
        QF_RETURN_IF(p->opts.ckpt_every != 0, QF_EUNSUPPORTED, "checkpoints need qudits of one dimension");
    }
    const int gdim = mixed ? 2 : dim;  // register-round group sizes are a stage option
    QF_RETURN_IF(p->opts.group_digits < 0 || p->opts.group_digits > max_group_size(uint32_t(gdim)), QF_EINVAL,
                 "group_digits = %d outside 0..%d for dim %d", p->opts.group_digits, max_group_size(uint32_t(gdim)),
                 gdim);
    p->group = p->opts.group_digits > 0 ? p->opts.group_digits : default_group(gdim, dtype);
    QF_RETURN_IF(p->opts.tile_digits < 0 || p->opts.tile_digits > kMaxTileDims || p->opts.adj_tile_digits < 0 ||
                     p->opts.adj_tile_digits > kMaxTileDims || p->opts.low_digits < 0 || p->opts.ckpt_every < 0 ||
                     p->opts.stage_kernel < 0 || p->opts.stage_kernel > 2 || p->opts.pipe_wgs < 0 ||
                     p->opts.pipe_wgs > 16 || p->opts.tile_order < 0 || p->opts.tile_order > 1 ||
                     p->opts.tile_search < 0 || p->opts.tile_search > 2,
                 QF_EINVAL, "bad tile / checkpoint options");
    p->gates.resize(nops);
    for (int i = 0; i < nops; ++i) {
        Gate& g = p->gates[i];
        g.op = ops[i];
        g.op.mat = nullptr;
        if (ops[i].kind == QF_OP_U) {
            size_t K = 1;
            for (int q = ops[i].q0; q < ops[i].q0 + ops[i].q1; ++q) K *= size_t(dims[q]);
            g.mat.resize(K * K);
            g.real = true;
            for (size_t e = 0; e < K * K; ++e) {
                g.mat[e] = cd(ops[i].mat[2 * e], ops[i].mat[2 * e + 1]);
                g.real = g.real && ops[i].mat[2 * e + 1] == 0.0;
            }
            const size_t esz = dtype == QF_C64 ? 8 : 16;
            std::vector<unsigned char> a(K * K * esz), b(K * K * esz);
            for (size_t r = 0; r < K; ++r)
                for (size_t c = 0; c < K; ++c) {
                    const cd x = g.mat[r * K + c];
                    const cd y = std::conj(g.mat[c * K + r]);
                    if (dtype == QF_C64) {
                        float* fa = reinterpret_cast<float*>(a.data()) + 2 * (r * K + c);
                        float* fb = reinterpret_cast<float*>(b.data()) + 2 * (r * K + c);
                        fa[0] = float(x.real());
                        fa[1] = float(x.imag());
                        fb[0] = float(y.real());
                        fb[1] = float(y.imag());
                    } else {
                        double* da = reinterpret_cast<double*>(a.data()) + 2 * (r * K + c);
                        double* db = reinterpret_cast<double*>(b.data()) + 2 * (r * K + c);
                        da[0] = x.real();
                        da[1] = x.imag();
                        db[0] = y.real();
                        db[1] = y.imag();
                    }
                }
            QF_CHECK(dev_malloc(&g.dmat, a.size(), "custom gate matrix"));
            QF_CHECK(dev_malloc(&g.dmat_adj, b.size(), "custom gate matrix"));
            QF_HIP_CHECK(hipMemcpy(g.dmat, a.data(), a.size(), hipMemcpyHostToDevice));
            QF_HIP_CHECK(hipMemcpy(g.dmat_adj, b.data(), b.size(), hipMemcpyHostToDevice));
        }
    }
    // checkpoint segments: [0, e0), [e0, e1), ...
    const int every = p->opts.ckpt_every;
    for (int e = every; every > 0 && e < nops; e += every) p->seg_end.push_back(e);
    p->seg_end.push_back(nops);
    if (!staged(p.get())) {
        build_steps(p.get());
        log_msg("plan D=%d n=%d: %d gates, per-gate schedule (fuse %d): %zu steps", dim, n, nops, p->opts.fuse,
                p->steps.size());
    } else if (nops > 0) {
        int k, r, ka, ra;
        tile_shape(dim, n, dtype, p->opts.tile_digits, p->opts.low_digits, false, k, r);
        tile_shape(dim, n, dtype, p->opts.adj_tile_digits, p->opts.low_digits, true, ka, ra);
        const size_t esz = dtype == QF_C64 ? 8 : 16;
        // gfx950 has 160 KB of LDS per workgroup
        QF_RETURN_IF(size_t(ipow(dim, k)) * esz + 4096 > 160 * 1024 ||
                         2 * size_t(ipow(dim, ka)) * esz + 8192 > 160 * 1024,
                     QF_ERANGE, "tile of %d (adjoint %d) qudits exceeds the 160 KB LDS of a workgroup", k, ka);
        std::vector<std::vector<GRef>> fseq(p->seg_end.size()), rseq(p->seg_end.size());
        int start = 0;
        for (size_t sgi = 0; sgi < p->seg_end.size(); ++sgi) {
            if (p->opts.fuse == 3)
                pair_fuse(p.get(), start, p->seg_end[sgi], fseq[sgi]);
            else
                for (int i = start; i < p->seg_end[sgi]; ++i) fseq[sgi].push_back({i, false});
            start = p->seg_end[sgi];
        }
        for (int sgi = int(p->seg_end.size()) - 1; sgi >= 0; --sgi) {
            const int lo = sgi == 0 ? 0 : p->seg_end[sgi - 1];
            for (int i = p->seg_end[sgi] - 1; i >= lo; --i) rseq[sgi].push_back({i, true});
        }
        if (p->opts.low_digits == 0) {
            r = choose_low(p.get(), fseq, k, r, false);
            ra = choose_low(p.get(), rseq, ka, ra, true);
        }
        for (size_t sgi = 0; sgi < fseq.size(); ++sgi) plan_passes(p.get(), fseq[sgi], k, r, int(sgi), p->fwd);
        for (int sgi = int(rseq.size()) - 1; sgi >= 0; --sgi) plan_passes(p.get(), rseq[sgi], ka, ra, sgi, p->rev);
        finalize_passes(p.get(), p->fwd, false);
        finalize_passes(p.get(), p->rev, true);
        log_msg("plan D=%d n=%d %s: %d gates, tile %d qudits (%d low), group %d: %zu forward passes; adjoint tile %d "
                "(%d low): %zu passes, %d M slots", dim, n, dtype == QF_C64 ? "c64" : "c128", nops, k, r, p->group,
                p->fwd.passes.size(), ka, ra, p->rev.passes.size(), p->rev.nslots);
        // forward register rounds by shape and the permutations folded into their addresses
        int kinds[8] = {0, 0, 0, 0, 0, 0, 0, 0}, nperm = 0;
        for (const RoundDesc& rd : p->fwd.hrounds) {
            if (rd.kind >= 0 && rd.kind < 8) ++kinds[rd.kind];
            nperm += (rd.pre0 >= 0) + (rd.pre1 >= 0) + (rd.pre2 >= 0) + (rd.post >= 0);
        }
        log_msg("plan rounds (forward): %zu (generic %d, none %d, U0 %d, U0 real %d, U01 %d, U1 %d, U1 real %d, "
                "phase %d), %d folded permutations", p->fwd.hrounds.size(), kinds[0], kinds[1], kinds[2], kinds[3],
                kinds[4], kinds[5], kinds[6], kinds[7], nperm);
    }
    *out = p.release();
    return QF_OK;
}

extern "C" {

qf_status qf_plan_create(int32_t dim, int32_t n, int32_t dtype, const qf_op* ops, int32_t nops, int32_t nparams,
                         const qf_plan_opts* opts, qf_plan** out) {
    if (out) *out = nullptr;
    QF_RETURN_IF(n < 1 || n > 32, QF_EINVAL, "n = %d outside 1..32", n);
    return create_plan(std::vector<int>(size_t(n), dim), dtype, ops, nops, nparams, opts, out);
}

qf_status qf_plan_create_dims(const int32_t* dims, int32_t n, int32_t dtype, const qf_op* ops, int32_t nops,
                              int32_t nparams, const qf_plan_opts* opts, qf_plan** out) {
    if (out) *out = nullptr;
    QF_RETURN_IF(dims == nullptr, QF_EINVAL, "dims is NULL");
    QF_RETURN_IF(n < 1 || n > 32, QF_EINVAL, "n = %d outside 1..32", n);
    return create_plan(std::vector<int>(dims, dims + n), dtype, ops, nops, nparams, opts, out);
}

int32_t qf_plan_num_stages(const qf_plan* plan) {
    if (!plan) return -1;
    return !staged(plan) ? int32_t(plan->steps.size()) : int32_t(plan->fwd.passes.size());
}

int32_t qf_plan_num_adjoint_stages(const qf_plan* plan) {
    if (!plan) return -1;
    return !staged(plan) ? int32_t(plan->steps.size()) : int32_t(plan->rev.passes.size());
}

qf_status qf_plan_forward(qf_plan* plan, const qf_state* s, const double* theta, void* stream) {
    StateView v;
    QF_CHECK(check_plan_state(plan, s, v));
    QF_RETURN_IF(plan->nparams > 0 && theta == nullptr, QF_EINVAL, "theta is NULL");
    QF_CHECK(check_finite_theta(theta, plan->nparams));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!staged(plan)) {
        for (const Step& step : plan->steps) {
            hipEvent_t a;
            QF_CHECK(prof_begin(plan, st, &a));
            QF_CHECK(run_step(plan, step, v, theta, false, st));
            const int fam = step.type == ST_AXIS ? F_AXIS
                            : step.type == ST_CTRL ? F_CTRL
                            : step.type == ST_DIAG ? F_DIAG
                            : step.type == ST_CROT ? F_CROT
                            : step.type == ST_PERM ? F_CTRL
                                                   : F_FUSED;
            QF_CHECK(prof_end(plan, st, a, fam, 2.0 * state_bytes(v)));
        }
        return check_norm_env(v, st);
    }
    if (plan->fwd.passes.empty()) return QF_OK;
    const bool save = plan->seg_end.size() > 1;
    if (save) QF_CHECK(ensure_ckpt(plan, v));
    QF_CHECK(upload_mats(plan, plan->fwd, theta, st));
    const size_t sb = state_bytes(v);
    for (size_t i = 0; i < plan->fwd.passes.size(); ++i) {
        const Pass& ps = plan->fwd.passes[i];
        if (ps.tile)
            QF_CHECK(run_tile_pass(plan, plan->fwd, ps, v, nullptr, nullptr, st));
        else
            QF_CHECK(run_fused_pass(plan, plan->fwd, ps, v, st));
        const bool seg_end = i + 1 == plan->fwd.passes.size() || plan->fwd.passes[i + 1].seg != ps.seg;
        if (save && seg_end && size_t(ps.seg) + 1 < plan->seg_end.size()) {
            hipEvent_t a;
            QF_CHECK(prof_begin(plan, st, &a));
            QF_HIP_CHECK(hipMemcpyAsync(reinterpret_cast<unsigned char*>(plan->ckpt) + size_t(ps.seg) * sb, v.amps,
                                        sb, hipMemcpyDeviceToDevice, st));
            QF_CHECK(prof_end(plan, st, a, F_CKPT, 2.0 * sb));
        }
    }
    QF_HIP_CHECK(hipEventRecord(plan->fwd.done, st));
    plan->fwd.done_valid = true;
    if (save) {
        plan->ckpt_amps = v.amps;
        plan->ckpt_batch = v.batch;
    }
    return check_norm_env(v, st);
}

qf_status qf_adjoint_grad(qf_plan* plan, const qf_state* psi, const qf_state* lam, const double* theta,
                          int32_t nterms, const int32_t* term_qudit, const double* term_diag, double* grad,
                          uint32_t flags, void* stream) {
    StateView v, vl;
    QF_CHECK(check_plan_state(plan, psi, v));
    QF_CHECK(check_plan_state(plan, lam, vl));
    QF_RETURN_IF((flags & ~uint32_t(QF_SEED)) != 0, QF_EINVAL, "unknown flags 0x%x", flags);
    const bool seed = (flags & QF_SEED) != 0;
    QF_RETURN_IF(vl.batch != v.batch, QF_EINVAL, "psi and lam batch differ");
    QF_RETURN_IF(psi->amps == lam->amps, QF_EINVAL, "psi and lam must not alias");
    QF_RETURN_IF(grad == nullptr, QF_EINVAL, "grad is NULL");
    QF_RETURN_IF(plan->nparams > 0 && theta == nullptr, QF_EINVAL, "theta is NULL");
    QF_CHECK(check_finite_theta(theta, plan->nparams));
    std::vector<int> active;
    std::vector<double> table;
    if (!seed) QF_CHECK(combine_terms(v, nterms, term_qudit, term_diag, active, table));
    std::vector<double> table_re(table.size() / 2);
    for (size_t i = 0; i < table_re.size(); ++i) table_re[i] = table[2 * i];
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int D = plan->D;
    const size_t E = size_t(v.dmax) * v.dmax;  // M entries per slot (the largest qudit's D x D)
    const bool stg = staged(plan);
    const int nslots = stg ? plan->rev.nslots : plan->nslots;
    if (stg) QF_CHECK(check_ckpt_source(plan, v));

    size_t pdoubles = 1;
    if (stg) {
        for (const Pass& ps : plan->rev.passes)
            if (ps.tile) pdoubles = std::max(pdoubles, size_t(ps.nslots) * ps.geom.ntiles * v.batch * E * 2);
    } else {
        pdoubles = std::max<size_t>(adj_axis_partial_doubles(v), 1);
    }
    const int ncr = stg ? plan->rev.ncr : plan->ncr_steps;
    if (ncr > 0) pdoubles = std::max(pdoubles, crot_partial_doubles(v));
    double* partial = nullptr;
    double* mdev = nullptr;
    double* crout = nullptr;
    const size_t mcount = size_t(v.batch) * std::max(nslots, 1) * E * 2;
    const size_t crcount = size_t(v.batch) * std::max(ncr, 1);
    qf_status rs = dev_malloc_async(reinterpret_cast<void**>(&partial), pdoubles * sizeof(double), st,
                                    "adjoint partial sums");
    if (rs == QF_OK) rs = dev_malloc_async(reinterpret_cast<void**>(&mdev), mcount * sizeof(double), st, "adjoint M");
    if (rs == QF_OK && ncr > 0)
        rs = dev_malloc_async(reinterpret_cast<void**>(&crout), crcount * sizeof(double), st,
                              "controlled-rotation gradients");
    // lam = H_O psi with H_O the Hermitian part of O (seed mode: lam already holds the seed)
    if (rs == QF_OK && !seed) rs = launch_diag_observable(v, lam->amps, active, table_re, st);
    if (rs == QF_OK && stg) {
        rs = upload_mats(plan, plan->rev, theta, st);
        const size_t sb = state_bytes(v);
        for (size_t i = 0; i < plan->rev.passes.size() && rs == QF_OK; ++i) {
            const Pass& ps = plan->rev.passes[i];
            // re-anchor psi at the start of each reverse segment but the last one
            const bool seg_start = i == 0 || plan->rev.passes[i - 1].seg != ps.seg;
            if (seg_start && size_t(ps.seg) + 1 < plan->seg_end.size()) {
                hipError_t e = hipMemcpyAsync(v.amps, reinterpret_cast<unsigned char*>(plan->ckpt) + size_t(ps.seg) * sb,
                                              sb, hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) rs = set_error(QF_EHIP, "checkpoint restore failed: %s", hipGetErrorString(e));
            }
            if (rs != QF_OK) break;
            if (ps.tile) {
                rs = run_tile_pass(plan, plan->rev, ps, v, lam->amps, partial, st);
                if (rs == QF_OK)
                    rs = launch_stage_mreduce(partial, ps.nslots, ps.geom.ntiles, v.batch, uint32_t(E), mdev,
                                              uint32_t(plan->rev.nslots), uint32_t(ps.slot0), st);
            } else if (ps.cr_slot >= 0) {
                const size_t esz = plan->dtype == QF_C64 ? 8 : 16;
                const void* tab = reinterpret_cast<const unsigned char*>(plan->rev.dmats) + ps.mat_off * esz;
                hipEvent_t a;
                rs = prof_begin(plan, st, &a);
                if (rs == QF_OK)
                    rs = launch_crot_adj(v, lam->amps, crot_args(plan->gates[ps.fused.gi].op), tab, 0, nullptr,
                                         partial, crout + ps.cr_slot, uint32_t(ncr), st);
                if (rs == QF_OK) rs = prof_end(plan, st, a, F_CROT_ADJ, 4.0 * state_bytes(v) * 2.0 / D);
            } else {
                rs = run_fused_pass(plan, plan->rev, ps, v, st);
                if (rs == QF_OK) rs = run_fused_pass(plan, plan->rev, ps, vl, st);
            }
        }
        if (rs == QF_OK) {
            hipError_t e = hipEventRecord(plan->rev.done, st);
            if (e == hipSuccess) plan->rev.done_valid = true;
        }
    } else if (rs == QF_OK) {
        for (int si = int(plan->steps.size()) - 1; si >= 0 && rs == QF_OK; --si) {
            const Step& s = plan->steps[si];
            if (s.type == ST_AXIS && s.slab) {
                const qf_op so = slab_op(plan->gates[s.gates[0]].op);
                std::vector<double> tab;
                crot_table(so, ctrl_levels(plan, so), theta, true, tab);
                rs = launch_crot_adj(v, lam->amps, crot_args(so), nullptr, 0, tab.data(), partial, crout + s.cr_slot,
                                     uint32_t(ncr), st);
            } else if (s.type == ST_AXIS && s.has_param) {
                Mat W = dagger(step_matrix(plan, s, theta), plan->dims[s.q]);
                std::vector<double> buf;
                to_interleaved(W, buf);
                hipEvent_t a;
                rs = prof_begin(plan, st, &a);
                if (rs == QF_OK)
                    rs = launch_adj_axis(v, lam->amps, s.q, buf.data(), partial, mdev, plan->nslots, s.slot,
                                         uint32_t(E), st);
                if (rs == QF_OK) rs = prof_end(plan, st, a, F_ADJ_AXIS, 4.0 * state_bytes(v));
            } else if (s.type == ST_CROT) {
                const qf_op& o = plan->gates[s.gates[0]].op;
                std::vector<double> tab;
                crot_table(o, ctrl_levels(plan, o), theta, true, tab);
                rs = launch_crot_adj(v, lam->amps, crot_args(o), nullptr, 0, tab.data(), partial, crout + s.cr_slot,
                                     uint32_t(ncr), st);
            } else {
                rs = run_step(plan, s, v, theta, true, st);
                if (rs == QF_OK) rs = run_step(plan, s, vl, theta, true, st);
            }
        }
    }
    std::vector<double> mhost(mcount), crhost(crcount, 0.0);
    if (rs == QF_OK && nslots > 0) {
        hipError_t e = hipMemcpyAsync(mhost.data(), mdev, mcount * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) rs = set_error(QF_EHIP, "copy of M matrices failed: %s", hipGetErrorString(e));
    }
    if (rs == QF_OK && ncr > 0) {
        hipError_t e = hipMemcpyAsync(crhost.data(), crout, crcount * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) rs = set_error(QF_EHIP, "copy of controlled-rotation gradients failed: %s",
                                            hipGetErrorString(e));
    }
    if (partial) (void)hipFreeAsync(partial, st);
    if (mdev) (void)hipFreeAsync(mdev, st);
    if (crout) (void)hipFreeAsync(crout, st);
    hipError_t e = hipStreamSynchronize(st);
    if (rs != QF_OK) return rs;
    QF_RETURN_IF(e != hipSuccess, QF_EHIP, "stream synchronisation failed: %s", hipGetErrorString(e));

    std::memset(grad, 0, sizeof(double) * size_t(v.batch) * plan->nparams);
    for (uint32_t b = 0; b < v.batch; ++b) {
        double* gb = grad + size_t(b) * plan->nparams;
        if (stg) {
            for (const Pass& ps : plan->rev.passes)
                for (const HOp& h : ps.ops) {
                    if (h.gslot < 0) continue;
                    std::vector<int> fwd_gates;
                    for (auto it = h.g.rbegin(); it != h.g.rend(); ++it) fwd_gates.push_back(it->gi);
                    add_group_grad(plan, fwd_gates, theta, mhost.data() + ((size_t(b) * nslots + h.gslot) * E) * 2,
                                   gb);
                }
            for (const Pass& ps : plan->rev.passes)
                if (ps.cr_slot >= 0) gb[plan->gates[ps.fused.gi].op.param] += crhost[size_t(b) * ncr + ps.cr_slot];
        } else {
            for (const Step& s : plan->steps) {
                if (s.type == ST_AXIS && s.has_param && !s.slab)
                    add_group_grad(plan, s.gates, theta, mhost.data() + ((size_t(b) * nslots + s.slot) * E) * 2, gb);
                if (s.cr_slot >= 0) gb[plan->gates[s.gates[0]].op.param] += crhost[size_t(b) * ncr + s.cr_slot];
            }
        }
    }
    // seed mode: lam held torch's gradient g = 2 dL/d(conj psi), the adjoint needs dL/d(conj psi)
    if (seed)
        for (size_t i = 0; i < size_t(v.batch) * plan->nparams; ++i) grad[i] *= 0.5;
    return QF_OK;
}

qf_status qf_plan_set_profiling(qf_plan* plan, int32_t enable) {
    QF_RETURN_IF(plan == nullptr, QF_EINVAL, "plan is NULL");
    plan->profiling = enable != 0;
    plan->prof.clear();
    plan->ev_used = 0;
    return QF_OK;
}

qf_status qf_plan_read_profile(qf_plan* plan, qf_kernel_stat* out, int32_t cap, int32_t* count) {
    QF_RETURN_IF(plan == nullptr || count == nullptr, QF_EINVAL, "plan or count is NULL");
    double ms[F_COUNT] = {0}, bytes[F_COUNT] = {0};
    int64_t launches[F_COUNT] = {0};
    for (const ProfRec& r : plan->prof) {
        QF_HIP_CHECK(hipEventSynchronize(r.b));
        float t = 0.f;
        QF_HIP_CHECK(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.family] += t;
        bytes[r.family] += r.bytes;
        launches[r.family] += 1;
    }
    int c = 0;
    for (int f = 0; f < F_COUNT; ++f) {
        if (launches[f] == 0) continue;
        if (out && c < cap) {
            std::memset(out[c].name, 0, sizeof(out[c].name));
            std::strncpy(out[c].name, kFamilies[f], sizeof(out[c].name) - 1);
            out[c].launches = launches[f];
            out[c].total_ms = ms[f];
            out[c].bytes = bytes[f];
        }
        ++c;
    }
    *count = c;
    plan->prof.clear();
    plan->ev_used = 0;
    return QF_OK;
}

void qf_plan_destroy(qf_plan* plan) { delete plan; }

}  // extern "C"

namespace qf {

// Reconstructs the op list a plan was created from (matrices of custom gates
// as interleaved FP64).
static void plan_ops(const qf_plan* p, std::vector<qf_op>& ops, std::vector<std::vector<double>>& mats) {
    ops.clear();
    mats.clear();
    mats.reserve(p->gates.size());
    for (const Gate& g : p->gates) {
        qf_op o = g.op;
        if (o.kind == QF_OP_U) {
            mats.emplace_back();
            to_interleaved(g.mat, mats.back());
            o.mat = mats.back().data();
        }
        ops.push_back(o);
    }
}

static uint64_t plan_key(const qf_plan* p, uint32_t batch) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix(uint64_t(p->D));
    mix(uint64_t(p->n));
    mix(uint64_t(p->dtype));
    mix(uint64_t(batch));
    mix(uint64_t(p->opts.ckpt_every));
    for (const Gate& g : p->gates) {
        mix(uint64_t(g.op.kind));
        mix(uint64_t(uint32_t(g.op.q0)) | (uint64_t(uint32_t(g.op.q1)) << 32));
        mix(uint64_t(uint32_t(g.op.j)) | (uint64_t(uint32_t(g.op.k)) << 32));
        if (g.op.kind == QF_OP_MCX || g.op.kind == QF_OP_CSHIFT)
            for (int i = 0; i < 16; ++i) mix(uint64_t(uint32_t(g.op.shifts[i])));
    }
    return h;
}

// Chosen options per (device architecture, circuit structure, batch, flags):
// kept for the life of the process and, when QF_TUNE_CACHE names a file,
// read from it once and appended to after every new choice.
struct TuneCache {
    std::vector<std::pair<uint64_t, qf_plan_opts>> entries;
    bool loaded = false;
};
static TuneCache g_tune;
static std::mutex g_tune_mu;

static constexpr int kOptFields = 10;

static void opts_to_array(const qf_plan_opts& o, int32_t* a) {
    const int32_t v[kOptFields] = {o.fuse, o.tile_digits, o.low_digits, o.ckpt_every, o.adj_tile_digits,
                                   o.stage_kernel, o.group_digits, o.pipe_wgs, o.tile_order, o.tile_search};
    std::memcpy(a, v, sizeof(v));
}

static qf_plan_opts opts_from_array(const int32_t* a) {
    qf_plan_opts o{};
    o.fuse = a[0];
    o.tile_digits = a[1];
    o.low_digits = a[2];
    o.ckpt_every = a[3];
    o.adj_tile_digits = a[4];
    o.stage_kernel = a[5];
    o.group_digits = a[6];
    o.pipe_wgs = a[7];
    o.tile_order = a[8];
    o.tile_search = a[9];
    return o;
}

// File format: one choice per line, "<key as 16 hex digits> <10 option values>".
static void tune_cache_load() {
    if (g_tune.loaded) return;
    g_tune.loaded = true;
    const char* path = std::getenv("QF_TUNE_CACHE");
    if (path == nullptr || path[0] == '\0') return;
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return;
    char line[512];
    size_t n = 0;
    while (std::fgets(line, sizeof(line), f)) {
        unsigned long long key = 0;
        int32_t a[kOptFields];
        if (std::sscanf(line, "%llx %d %d %d %d %d %d %d %d %d %d", &key, &a[0], &a[1], &a[2], &a[3], &a[4], &a[5],
                        &a[6], &a[7], &a[8], &a[9]) == 1 + kOptFields) {
            g_tune.entries.push_back({uint64_t(key), opts_from_array(a)});
            ++n;
        }
    }
    std::fclose(f);
    log_msg("autotune cache %s: %zu entries", path, n);
}

static void tune_cache_store(uint64_t key, const qf_plan_opts& o) {
    g_tune.entries.push_back({key, o});
    const char* path = std::getenv("QF_TUNE_CACHE");
    if (path == nullptr || path[0] == '\0') return;
    FILE* f = std::fopen(path, "a");
    if (f == nullptr) {
        log_msg("autotune cache %s: cannot append", path);
        return;
    }
    int32_t a[kOptFields];
    opts_to_array(o, a);
    std::fprintf(f, "%016llx %d %d %d %d %d %d %d %d %d %d\n", (unsigned long long)key, a[0], a[1], a[2], a[3], a[4],
                 a[5], a[6], a[7], a[8], a[9]);
    std::fclose(f);
}

// FNV-1a of the current device's architecture name (e.g. "gfx950:sramecc+:xnack-").
static qf_status arch_hash(uint64_t* out) {
    int dev = 0;
    QF_HIP_CHECK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QF_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    uint64_t h = 1469598103934665603ull;
    for (const char* c = prop.gcnArchName; *c; ++c) {
        h ^= uint64_t(uint8_t(*c));
        h *= 1099511628211ull;
    }
    *out = h;
    return QF_OK;
}

// Device buffers and observable used to time candidates.
struct TuneBench {
    const qf_state* s = nullptr;
    qf_state sl{};                  // adjoint state (scratch of the state's size)
    const double* theta = nullptr;  // host
    double* theta_dev = nullptr;    // bound mode: shared by every register (stride 0)
    double* grad_dev = nullptr;
    double* loss_dev = nullptr;
    std::vector<double> grad_host;
    int32_t term_q = 0;
    std::vector<double> term_tab;   // Z on qudit 0
    uint32_t flags = 0;
    hipStream_t st = nullptr;
};

static qf_status tune_step(qf_plan* tp, TuneBench& b) {
    const bool bound = (b.flags & QF_TUNE_BOUND) != 0, adj = (b.flags & QF_TUNE_ADJOINT) != 0;
    void* stream = reinterpret_cast<void*>(b.st);
    if (bound) {
        QF_CHECK(qf_plan_forward_dev(tp, b.s, b.theta_dev, 0, stream));
        if (adj)
            QF_CHECK(qf_adjoint_grad_dev(tp, b.s, &b.sl, b.theta_dev, 0, 1, &b.term_q, b.term_tab.data(), b.grad_dev,
                                         b.loss_dev, 0, stream));
        return QF_OK;
    }
    QF_CHECK(qf_plan_forward(tp, b.s, b.theta, stream));
    if (adj)
        QF_CHECK(qf_adjoint_grad(tp, b.s, &b.sl, b.theta, 1, &b.term_q, b.term_tab.data(), b.grad_host.data(), 0,
                                 stream));
    return QF_OK;
}

}  // namespace qf

extern "C" void qf_shutdown(void) {
    std::lock_guard<std::mutex> lock(qf::g_tune_mu);
    std::vector<std::pair<uint64_t, qf_plan_opts>>().swap(qf::g_tune.entries);
    qf::g_tune.loaded = false;
    qf::trim_pools();
}

extern "C" {

qf_status qf_plan_autotune(qf_plan* plan, const qf_state* s, const double* theta, uint32_t flags,
                           qf_plan_opts* chosen, void* stream) {
    StateView v;
    QF_CHECK(check_plan_state(plan, s, v));
    QF_RETURN_IF(plan->nparams > 0 && theta == nullptr, QF_EINVAL, "theta is NULL");
    QF_RETURN_IF((flags & ~uint32_t(QF_TUNE_ADJOINT | QF_TUNE_BOUND)) != 0, QF_EINVAL, "unknown flags 0x%x", flags);
    QF_RETURN_IF(plan->D == 0, QF_EUNSUPPORTED, "autotuning needs qudits of one dimension");
    QF_CHECK(check_finite_theta(theta, plan->nparams));
    const bool bound = (flags & QF_TUNE_BOUND) != 0;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint64_t key = plan_key(plan, v.batch), ah = 0;
    QF_CHECK(arch_hash(&ah));
    key = (key ^ ah) * 1099511628211ull;
    key = (key ^ uint64_t(flags)) * 1099511628211ull;
    std::vector<qf_op> ops;
    std::vector<std::vector<double>> mats;
    plan_ops(plan, ops, mats);
    qf_plan_opts best = plan->opts;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_cache_load();
    bool cached = false;
    for (const auto& e : g_tune.entries)
        if (e.first == key) {
            best = e.second;
            cached = true;
        }
    if (!cached) {
        // candidates: stage plans over tile sizes and register-group sizes (group
        // 1 applies each qudit's run as a D x D matrix, group 2 the runs of two
        // qudits as one D^2 x D^2 block), the one-sweep-per-op and pipelined
        // stage kernels; without QF_TUNE_BOUND also the two-qudit dense blocks
        // (fuse 3) and the per-qudit-run sweeps (fuse 2)
        std::vector<qf_plan_opts> cand;
        int k0, r0;
        tile_shape(plan->D, plan->n, plan->dtype, 0, 0, false, k0, r0);
        const int gmax = max_group_size(uint32_t(plan->D));
        for (int dk = -1; dk <= 1; ++dk) {
            const int k = k0 + dk;
            if (k < 1 || k > plan->n) continue;
            for (int g = 1; g <= gmax; ++g) {
                qf_plan_opts o = plan->opts;
                o.fuse = 0;
                o.tile_digits = k;
                o.group_digits = g;
                o.stage_kernel = 0;
                cand.push_back(o);
            }
            qf_plan_opts o = plan->opts;
            o.fuse = 0;
            o.tile_digits = k;
            o.stage_kernel = 1;
            cand.push_back(o);
            for (int g = 1; g <= std::min(gmax, 3); ++g)
                for (int w : {2, 4, 8}) {
                    qf_plan_opts q = plan->opts;
                    q.fuse = 0;
                    q.tile_digits = k;
                    q.group_digits = g;
                    q.stage_kernel = 2;
                    q.pipe_wgs = w;
                    cand.push_back(q);
                }
        }
        if (!bound && plan->D * plan->D >= 16) {
            qf_plan_opts o = plan->opts;
            o.fuse = 3;
            o.tile_digits = 0;
            o.group_digits = 0;
            cand.push_back(o);
        }
        if (!bound) {
            qf_plan_opts o = plan->opts;
            o.fuse = 2;
            cand.push_back(o);
        }
        TuneBench b;
        b.s = s;
        b.theta = theta;
        b.flags = flags;
        b.st = st;
        b.term_tab.assign(2 * size_t(plan->D), 0.0);
        for (int d = 0; d < plan->D; ++d) {
            b.term_tab[2 * d] = std::cos(2 * 3.14159265358979323846 * d / plan->D);
            b.term_tab[2 * d + 1] = std::sin(2 * 3.14159265358979323846 * d / plan->D);
        }
        b.grad_host.assign(size_t(v.batch) * std::max(plan->nparams, 1), 0.0);
        b.sl = *s;
        b.sl.amps = nullptr;
        qf_status rs = QF_OK;
        if (flags & QF_TUNE_ADJOINT) rs = dev_malloc(&b.sl.amps, state_bytes(v), "autotune adjoint state");
        if (rs == QF_OK && bound) {
            rs = dev_malloc(reinterpret_cast<void**>(&b.theta_dev), sizeof(double) * std::max(plan->nparams, 1),
                            "autotune angles");
            if (rs == QF_OK)
                rs = dev_malloc(reinterpret_cast<void**>(&b.grad_dev),
                                sizeof(double) * v.batch * std::max(plan->nparams, 1), "autotune gradients");
            if (rs == QF_OK)
                rs = dev_malloc(reinterpret_cast<void**>(&b.loss_dev), sizeof(double) * 2 * v.batch, "autotune loss");
            if (rs == QF_OK && plan->nparams > 0 &&
                hipMemcpy(b.theta_dev, theta, sizeof(double) * plan->nparams, hipMemcpyHostToDevice) != hipSuccess)
                rs = set_error(QF_EHIP, "autotune: copy of the angles failed");
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (rs == QF_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
            rs = set_error(QF_EHIP, "autotune: event creation failed");
        float best_ms = 1e30f;
        size_t timed = 0, ntried = 0;
        // times one candidate (two steps after a warm-up step); < 0: it did not run
        auto time_opts = [&](const qf_plan_opts& o) -> float {
            ++ntried;
            qf_plan* tp = nullptr;
            if (qf_plan_create(plan->D, plan->n, plan->dtype, ops.data(), int32_t(ops.size()), plan->nparams, &o,
                               &tp) != QF_OK)
                return -1.f;  // e.g. a tile beyond the LDS size
            qf_status cs = bound ? qf_plan_bind(tp, v.batch) : QF_OK;
            if (cs == QF_OK) cs = tune_step(tp, b);  // warm-up
            if (cs == QF_OK) cs = hipEventRecord(e0, st) == hipSuccess ? QF_OK : QF_EHIP;
            for (int rep = 0; rep < 2 && cs == QF_OK; ++rep) cs = tune_step(tp, b);
            if (cs == QF_OK) cs = hipEventRecord(e1, st) == hipSuccess ? QF_OK : QF_EHIP;
            float ms = -1.f;
            if (cs == QF_OK && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                ++timed;
            else
                ms = -1.f;
            qf_plan_destroy(tp);
            if (cs == QF_EHIP) rs = cs;  // a failing HIP call ends the search
            return ms;
        };
        for (size_t ci = 0; ci < cand.size() && rs == QF_OK; ++ci) {
            const float ms = time_opts(cand[ci]);
            if (ms >= 0.f && ms < best_ms) {
                best_ms = ms;
                best = cand[ci];
            }
        }
        // second phase when the adjoint is timed: the adjoint tile of the best
        // stage plan, from one qudit below its default up to the whole register
        if (rs == QF_OK && (flags & QF_TUNE_ADJOINT) && best.fuse == 0 && best_ms < 1e30f) {
            int ka, ra;
            tile_shape(plan->D, plan->n, plan->dtype, best.adj_tile_digits, best.low_digits, true, ka, ra);
            const qf_plan_opts base = best;
            for (int k = std::max(1, ka - 1); k <= plan->n && rs == QF_OK; ++k) {
                if (k == ka) continue;
                qf_plan_opts o = base;
                o.adj_tile_digits = k;
                const float ms = time_opts(o);
                if (ms >= 0.f && ms < best_ms) {
                    best_ms = ms;
                    best = o;
                }
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(st);
        for (void* q : {b.sl.amps, static_cast<void*>(b.theta_dev), static_cast<void*>(b.grad_dev),
                        static_cast<void*>(b.loss_dev)})
            if (q) (void)hipFree(q);
        if (rs != QF_OK) return rs;
        QF_RETURN_IF(timed == 0, QF_EHIP, "no autotuning candidate ran");
        log_msg("autotune D=%d n=%d batch %u flags %u: %zu of %zu candidates timed, chose fuse %d tile %d group %d "
                "kernel %d pipe %d adjoint tile %d (%.3f ms for two steps)", plan->D, plan->n, v.batch, flags, timed,
                ntried, best.fuse, best.tile_digits, best.group_digits, best.stage_kernel, best.pipe_wgs,
                best.adj_tile_digits, double(best_ms));
        tune_cache_store(key, best);
    }
    // rebuild this plan with the chosen options (unbound)
    qf_plan* np = nullptr;
    QF_CHECK(qf_plan_create(plan->D, plan->n, plan->dtype, ops.data(), int32_t(ops.size()), plan->nparams, &best, &np));
    plan->swap_with(*np);
    qf_plan_destroy(np);
    if (chosen) *chosen = best;
    return QF_OK;
}

}  // extern "C"

namespace qf {

static DevGate dev_gate(const qf_op& o) { return DevGate{o.kind, o.j, o.k, o.param}; }

static void bound_groups(qf_plan* p, PassList& L) {
    L.hgroups.clear();
    for (const Pass& ps : L.passes) {
        if (!ps.tile && ps.cr_slot >= 0) {
            L.hgroups.push_back(DevGroup{DG_CR, uint32_t(ps.mat_off), int32_t(p->hgates.size()), 1,
                                         ps.fused.inv ? 1 : 0});
            p->hgates.push_back(dev_gate(p->gates[ps.fused.gi].op));
        }
        if (!ps.tile) continue;
        for (size_t i = 0; i < ps.ops.size(); ++i) {
            const HOp& h = ps.ops[i];
            const StageOp& so = L.hops[ps.op_off + i];
            if (h.type == SOP_U) {
                DevGroup g{DG_U, uint32_t(ps.mat_off + so.mat), int32_t(p->hgates.size()), int32_t(h.g.size()),
                           h.g[0].inv ? 1 : 0};
                for (const GRef& r : h.g) p->hgates.push_back(dev_gate(op_of(p, r)));
                L.hgroups.push_back(g);
            } else if (h.type == SOP_PHASE) {
                for (size_t j = 0; j < h.g.size(); ++j)
                    L.hgroups.push_back(DevGroup{DG_CZ, uint32_t(ps.mat_off + so.ptab[j]), 0, 0, h.g[j].inv ? 1 : 0});
                if (ps.nrounds > 0)
                    L.hgroups.push_back(DevGroup{DG_W, uint32_t(ps.mat_off + so.wtab), 0, 0, h.g[0].inv ? 1 : 0});
            }
        }
    }
}

template <typename X>
static qf_status dev_upload(X** dst, const std::vector<X>& src) {
    if (src.empty()) return QF_OK;
    QF_CHECK(dev_malloc(reinterpret_cast<void**>(dst), src.size() * sizeof(X), "bound-mode tables"));
    QF_HIP_CHECK(hipMemcpy(*dst, src.data(), src.size() * sizeof(X), hipMemcpyHostToDevice));
    return QF_OK;
}

static qf_status dev_alloc(void** dst, size_t bytes) {
    return dev_malloc(dst, bytes, "bound-mode workspace");
}

static qf_status check_bound(const qf_plan* p, const StateView& v, int64_t theta_stride) {
    QF_RETURN_IF(p->bound == 0, QF_EINVAL, "plan is not bound: call qf_plan_bind first");
    QF_RETURN_IF(v.batch > p->bound, QF_ERANGE, "state batch %u exceeds the bound batch %u", v.batch, p->bound);
    QF_RETURN_IF(theta_stride != 0 && theta_stride < p->nparams, QF_EINVAL,
                 "theta_stride %lld must be 0 or >= nparams %d", (long long)theta_stride, p->nparams);
    return QF_OK;
}

}  // namespace qf

extern "C" {

qf_status qf_plan_bind(qf_plan* plan, int64_t batch) {
    QF_RETURN_IF(plan == nullptr, QF_EINVAL, "plan is NULL");
    QF_RETURN_IF(batch < 1 || batch >= (int64_t(1) << 31), QF_EINVAL, "batch %lld out of range", (long long)batch);
    QF_RETURN_IF(plan->opts.fuse != 0, QF_EUNSUPPORTED, "device-parameter mode needs a stage plan (fuse = 0)");
    plan->release_bound();
    const uint64_t N = ipow(plan->D, plan->n);
    QF_RETURN_IF(N * uint64_t(batch) >= (1ull << 32), QF_ERANGE, "batch * D^n exceeds 2^32 amplitudes");
    const int D = plan->D;
    const size_t E = size_t(D) * D;
    const size_t esz = plan->dtype == QF_C64 ? 8 : 16;
    plan->hgates.clear();
    bound_groups(plan, plan->fwd);
    bound_groups(plan, plan->rev);
    // gradient runs and contribution slots
    plan->hgg.clear();
    std::vector<std::pair<int, int>> contrib;  // (param, slot)
    int nc = 0;
    for (const Pass& ps : plan->rev.passes)
        for (const HOp& h : ps.ops) {
            if (h.gslot < 0) continue;
            DevGradGroup g{h.gslot, int32_t(plan->hgates.size()), int32_t(h.g.size()), nc};
            for (auto it = h.g.rbegin(); it != h.g.rend(); ++it) plan->hgates.push_back(dev_gate(op_of(plan, *it)));
            for (int i = int(h.g.size()) - 1; i >= 0; --i) {  // the kernel walks the run backwards
                const qf_op& o = op_of(plan, h.g[h.g.size() - 1 - i]);
                if (is_rot(o.kind)) contrib.push_back({o.param, nc++});
            }
            plan->hgg.push_back(g);
        }
    plan->cr_contrib.assign(size_t(plan->rev.ncr), -1);
    for (const Pass& ps : plan->rev.passes)
        if (ps.cr_slot >= 0) {
            contrib.push_back({plan->gates[ps.fused.gi].op.param, nc});
            plan->cr_contrib[size_t(ps.cr_slot)] = nc++;
        }
    plan->ncontrib = nc;
    std::vector<int32_t> poff(plan->nparams + 1, 0), plist(nc);
    for (auto& c : contrib) poff[c.first + 1]++;
    for (int i = 0; i < plan->nparams; ++i) poff[i + 1] += poff[i];
    {
        std::vector<int32_t> fill(poff.begin(), poff.end() - 1);
        for (auto& c : contrib) plist[fill[c.first]++] = c.second;
    }
    qf_status rs = QF_OK;
    auto step = [&](qf_status r) {
        if (rs == QF_OK) rs = r;
    };
    step(dev_upload(&plan->dgates, plan->hgates));
    step(dev_upload(&plan->fwd.dgroups, plan->fwd.hgroups));
    step(dev_upload(&plan->rev.dgroups, plan->rev.hgroups));
    step(dev_upload(&plan->dgg, plan->hgg));
    step(dev_upload(&plan->d_poff, poff));
    if (nc > 0) step(dev_upload(&plan->d_plist, plist));
    if (rs == QF_OK && plan->fwd.dmats == nullptr) step(upload_ops(plan, plan->fwd));
    if (rs == QF_OK && plan->rev.dmats == nullptr) step(upload_ops(plan, plan->rev));
    step(dev_alloc(&plan->fwd.dmats_b, std::max<size_t>(plan->fwd.nmats, 1) * esz * size_t(batch)));
    step(dev_alloc(&plan->rev.dmats_b, std::max<size_t>(plan->rev.nmats, 1) * esz * size_t(batch)));
    size_t pd = 1;
    for (const Pass& ps : plan->rev.passes)
        if (ps.tile) pd = std::max(pd, size_t(ps.nslots) * ps.geom.ntiles * size_t(batch) * E * 2);
    if (plan->rev.ncr > 0) pd = std::max(pd, crot_partial_doubles(uniform_view(D, plan->n, batch, plan->dtype)));
    step(dev_alloc(reinterpret_cast<void**>(&plan->w_partial), pd * sizeof(double)));
    step(dev_alloc(reinterpret_cast<void**>(&plan->w_m),
                   size_t(batch) * std::max(plan->rev.nslots, 1) * E * 2 * sizeof(double)));
    step(dev_alloc(reinterpret_cast<void**>(&plan->w_contrib), size_t(batch) * std::max(nc, 1) * sizeof(double)));
    StateView v = uniform_view(D, plan->n, batch, plan->dtype);
    step(dev_alloc(reinterpret_cast<void**>(&plan->w_expect), expect_ws_doubles(v) * sizeof(double)));
    if (rs == QF_OK && plan->seg_end.size() > 1) step(ensure_ckpt(plan, v));
    if (rs != QF_OK) {
        plan->release_bound();
        return rs;
    }
    plan->bound = uint32_t(batch);
    return QF_OK;
}

qf_status qf_plan_forward_dev(qf_plan* plan, const qf_state* s, const double* theta, int64_t theta_stride,
                              void* stream) {
    StateView v;
    QF_CHECK(check_plan_state(plan, s, v));
    QF_CHECK(check_bound(plan, v, theta_stride));
    QF_RETURN_IF(plan->nparams > 0 && theta == nullptr, QF_EINVAL, "theta is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PassList& L = plan->fwd;
    const size_t esz = plan->dtype == QF_C64 ? 8 : 16;
    QF_CHECK(launch_build_mats(plan->D, plan->dtype, L.dgroups, int(L.hgroups.size()), plan->dgates, theta,
                               theta_stride, v.batch, L.dmats_b, L.nmats, st));
    const size_t sb = state_bytes(v);
    for (size_t i = 0; i < L.passes.size(); ++i) {
        const Pass& ps = L.passes[i];
        if (ps.tile) {
            const void* mats = reinterpret_cast<const unsigned char*>(L.dmats_b) + ps.mat_off * esz;
            QF_CHECK(launch_forward_pass(plan, L, ps, v, mats, L.nmats, st));
        } else if (ps.cr_slot >= 0) {
            const void* tab = reinterpret_cast<const unsigned char*>(L.dmats_b) + ps.mat_off * esz;
            QF_CHECK(launch_crot(v, crot_args(plan->gates[ps.fused.gi].op), tab, L.nmats, nullptr, st));
        } else if (plan->gates[ps.fused.gi].op.kind == QF_OP_SWAP || plan->gates[ps.fused.gi].op.kind == QF_OP_MCX) {
            QF_CHECK(launch_perm_gate(v, plan->gates[ps.fused.gi].op, false, st));
        } else {
            const Gate& g = plan->gates[ps.fused.gi];
            QF_CHECK(launch_fused(v, g.op.q1, g.op.q0, g.dmat, st, g.real));
        }
        const bool seg_end = i + 1 == L.passes.size() || L.passes[i + 1].seg != ps.seg;
        if (plan->seg_end.size() > 1 && seg_end && size_t(ps.seg) + 1 < plan->seg_end.size())
            QF_HIP_CHECK(hipMemcpyAsync(reinterpret_cast<unsigned char*>(plan->ckpt) + size_t(ps.seg) * sb, v.amps,
                                        sb, hipMemcpyDeviceToDevice, st));
    }
    if (plan->seg_end.size() > 1) {
        plan->ckpt_amps = v.amps;
        plan->ckpt_batch = v.batch;
    }
    return QF_OK;
}

qf_status qf_adjoint_grad_dev(qf_plan* plan, const qf_state* psi, const qf_state* lam, const double* theta,
                              int64_t theta_stride, int32_t nterms, const int32_t* term_qudit,
                              const double* term_diag, double* grad, double* loss, uint32_t flags, void* stream) {
    StateView v, vl;
    QF_CHECK(check_plan_state(plan, psi, v));
    QF_CHECK(check_plan_state(plan, lam, vl));
    QF_CHECK(check_bound(plan, v, theta_stride));
    QF_RETURN_IF((flags & ~uint32_t(QF_SEED)) != 0, QF_EINVAL, "unknown flags 0x%x", flags);
    const bool seed = (flags & QF_SEED) != 0;
    QF_RETURN_IF(seed && loss != nullptr, QF_EINVAL, "seed mode has no observable: loss must be NULL");
    QF_RETURN_IF(vl.batch != v.batch, QF_EINVAL, "psi and lam batch differ");
    QF_RETURN_IF(psi->amps == lam->amps, QF_EINVAL, "psi and lam must not alias");
    QF_RETURN_IF(grad == nullptr && plan->nparams > 0, QF_EINVAL, "grad is NULL");
    QF_RETURN_IF(plan->nparams > 0 && theta == nullptr, QF_EINVAL, "theta is NULL");
    QF_CHECK(check_ckpt_source(plan, v));
    std::vector<int> active;
    std::vector<double> table;
    if (!seed) QF_CHECK(combine_terms(v, nterms, term_qudit, term_diag, active, table));
    std::vector<double> table_re(active.size() * v.D);
    for (size_t i = 0; i < table_re.size(); ++i) table_re[i] = table[2 * i];
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int D = plan->D;
    const size_t E = size_t(D) * D;
    const size_t esz = plan->dtype == QF_C64 ? 8 : 16;
    if (loss) QF_CHECK(launch_expect_ws(v, active, table, loss, plan->w_expect, st));
    if (!seed) QF_CHECK(launch_diag_observable(v, lam->amps, active, table_re, st));
    PassList& L = plan->rev;
    QF_CHECK(launch_build_mats(plan->D, plan->dtype, L.dgroups, int(L.hgroups.size()), plan->dgates, theta,
                               theta_stride, v.batch, L.dmats_b, L.nmats, st));
    const size_t sb = state_bytes(v);
    for (size_t i = 0; i < L.passes.size(); ++i) {
        const Pass& ps = L.passes[i];
        const bool seg_start = i == 0 || L.passes[i - 1].seg != ps.seg;
        if (seg_start && size_t(ps.seg) + 1 < plan->seg_end.size())
            QF_HIP_CHECK(hipMemcpyAsync(v.amps, reinterpret_cast<unsigned char*>(plan->ckpt) + size_t(ps.seg) * sb, sb,
                                        hipMemcpyDeviceToDevice, st));
        if (ps.tile) {
            const void* mats = reinterpret_cast<const unsigned char*>(L.dmats_b) + ps.mat_off * esz;
            if (ps.nrounds > 0 && plan->opts.stage_kernel != 1)
                QF_CHECK(launch_stage_adj_rounds(v, lam->amps, adj_group(plan), ps.geom,
                                                 L.drounds + ps.round_off, ps.nrounds, L.dops + ps.op_off, mats,
                                                 plan->w_partial, st, L.nmats));
            else
                QF_CHECK(launch_stage_adj(v, lam->amps, ps.geom, L.dops + ps.op_off, ps.nops, mats, plan->w_partial,
                                          st, L.nmats));
            QF_CHECK(launch_stage_mreduce(plan->w_partial, ps.nslots, ps.geom.ntiles, v.batch, uint32_t(E), plan->w_m,
                                          uint32_t(L.nslots), uint32_t(ps.slot0), st));
        } else if (ps.cr_slot >= 0) {
            const void* tab = reinterpret_cast<const unsigned char*>(L.dmats_b) + ps.mat_off * esz;
            QF_CHECK(launch_crot_adj(v, lam->amps, crot_args(plan->gates[ps.fused.gi].op), tab, L.nmats, nullptr,
                                     plan->w_partial, plan->w_contrib + plan->cr_contrib[size_t(ps.cr_slot)],
                                     uint32_t(plan->ncontrib), st));
        } else if (plan->gates[ps.fused.gi].op.kind == QF_OP_SWAP || plan->gates[ps.fused.gi].op.kind == QF_OP_MCX) {
            QF_CHECK(launch_perm_gate(v, plan->gates[ps.fused.gi].op, true, st));
            QF_CHECK(launch_perm_gate(vl, plan->gates[ps.fused.gi].op, true, st));
        } else {
            const Gate& g = plan->gates[ps.fused.gi];
            QF_CHECK(launch_fused(v, g.op.q1, g.op.q0, g.dmat_adj, st, g.real));
            QF_CHECK(launch_fused(vl, g.op.q1, g.op.q0, g.dmat_adj, st, g.real));
        }
    }
    // seed mode: lam held torch's gradient g = 2 dL/d(conj psi), the adjoint needs dL/d(conj psi)
    return launch_grad(D, plan->dgg, int(plan->hgg.size()), plan->dgates, theta, theta_stride, plan->w_m, L.nslots,
                       v.batch, plan->w_contrib, plan->ncontrib, plan->d_poff, plan->d_plist, plan->nparams,
                       seed ? 0.5 : 1.0, grad, st);
}

}  // extern "C"
