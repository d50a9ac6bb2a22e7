// C ABI of the per-gate entry points: argument validation (synchronous, before
// any HIP call) and dispatch to the kernel launchers.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "qf_internal.h"

namespace qf {

static thread_local char g_err[512] = "";

qf_status set_error(qf_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

qf_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(QF_EHIP, "%s: launch failed: %s", what, hipGetErrorString(e));
    return QF_OK;
}

static bool env_on(const char* name) {
    const char* e = std::getenv(name);
    return e != nullptr && e[0] != '\0' && !(e[0] == '0' && e[1] == '\0');
}

qf_status dev_malloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (env_on("QF_TEST_FAIL_ALLOC")) return set_error(QF_ENOMEM, "%s: allocation of %zu bytes refused "
                                                       "(QF_TEST_FAIL_ALLOC)", what, bytes);
    if (hipMalloc(p, bytes < 16 ? 16 : bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(QF_ENOMEM, "%s: device allocation of %zu bytes failed", what, bytes);
    }
    return QF_OK;
}

// The temporaries are stream-ordered allocations from each device's default
// pool.  With the pool's default release threshold (0) every synchronisation
// hands freed memory back to the driver, so the next call maps its pages again
// (hundreds of microseconds for the FP64 prefix sums of a large register).
// Freed memory up to kPoolKeepBytes per device stays in the pool instead;
// qf_shutdown trims it.
constexpr uint64_t kPoolKeepBytes = uint64_t(4) << 30;
static std::mutex g_pool_mu;
static std::vector<char> g_pool_set;

static void keep_pool_memory() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (size_t(dev) < g_pool_set.size() && g_pool_set[size_t(dev)]) return;
    if (size_t(dev) >= g_pool_set.size()) g_pool_set.resize(size_t(dev) + 1, 0);
    hipMemPool_t pool = nullptr;
    uint64_t keep = kPoolKeepBytes;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess ||
        hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
        (void)hipGetLastError();  // the pool keeps its default: correct, only slower
    }
    g_pool_set[size_t(dev)] = 1;
}

void trim_pools() {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    for (size_t dev = 0; dev < g_pool_set.size(); ++dev) {
        if (!g_pool_set[dev]) continue;
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, int(dev)) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
        (void)hipGetLastError();
    }
}

qf_status dev_malloc_async(void** p, size_t bytes, hipStream_t st, const char* what) {
    *p = nullptr;
    if (env_on("QF_TEST_FAIL_ALLOC")) return set_error(QF_ENOMEM, "%s: allocation of %zu bytes refused "
                                                       "(QF_TEST_FAIL_ALLOC)", what, bytes);
    keep_pool_memory();
    if (hipMallocAsync(p, bytes < 16 ? 16 : bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(QF_ENOMEM, "%s: stream-ordered allocation of %zu bytes failed", what, bytes);
    }
    return QF_OK;
}

qf_status host_malloc_pinned(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (env_on("QF_TEST_FAIL_ALLOC")) return set_error(QF_ENOMEM, "%s: allocation of %zu bytes refused "
                                                       "(QF_TEST_FAIL_ALLOC)", what, bytes);
    if (hipHostMalloc(p, bytes < 16 ? 16 : bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(QF_ENOMEM, "%s: pinned host allocation of %zu bytes failed", what, bytes);
    }
    return QF_OK;
}

bool log_enabled() { return env_on("QF_LOG"); }

void log_msg(const char* fmt, ...) {
    if (!log_enabled()) return;
    va_list ap;
    va_start(ap, fmt);
    std::fputs("[qf] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    va_end(ap);
}

qf_status make_view(const qf_state* s, StateView& v) {
    QF_RETURN_IF(s == nullptr, QF_EINVAL, "state is NULL");
    QF_RETURN_IF(s->amps == nullptr, QF_EINVAL, "state amplitudes pointer is NULL");
    QF_RETURN_IF(s->dtype != QF_C64 && s->dtype != QF_C128, QF_EDTYPE, "unknown dtype %d", s->dtype);
    if (s->dims == nullptr) {
        QF_RETURN_IF(s->dim < 2 || s->dim > kMaxDim, QF_ERANGE, "dim %d outside 2..%d", s->dim, kMaxDim);
    } else {
        QF_RETURN_IF(s->dim != 0, QF_EINVAL, "dim = %d must be 0 when dims is given", s->dim);
    }
    QF_RETURN_IF(s->n < 1 || s->n > kMaxQudits, QF_EINVAL, "n = %d outside 1..%d", s->n, kMaxQudits);
    QF_RETURN_IF(s->batch < 1, QF_EINVAL, "batch = %lld < 1", (long long)s->batch);
    uint64_t N = 1;
    for (int i = 0; i < s->n; ++i) {
        const int32_t d = s->dims ? s->dims[i] : s->dim;
        QF_RETURN_IF(d < 2 || d > kMaxDim, QF_ERANGE, "dimension %d of qudit %d outside 2..%d", d, i, kMaxDim);
        v.dims[i] = uint32_t(d);
        N *= uint64_t(d);
        QF_RETURN_IF(N >= (1ull << 32), QF_ERANGE, "the register exceeds 2^32 amplitudes");
    }
    const uint64_t total = N * uint64_t(s->batch);
    QF_RETURN_IF(total >= (1ull << 32), QF_ERANGE, "batch * amplitudes = %llu exceeds 2^32 - 1",
                 (unsigned long long)total);
    v.amps = s->amps;
    v.n = uint32_t(s->n);
    v.N = uint32_t(N);
    v.batch = uint32_t(s->batch);
    v.total = uint32_t(total);
    v.dtype = s->dtype;
    v.dmin = v.dmax = v.dims[0];
    uint32_t stride = 1;
    for (int i = int(v.n) - 1; i >= 0; --i) {
        v.strides[i] = stride;
        stride *= v.dims[i];
        v.dmin = std::min(v.dmin, v.dims[i]);
        v.dmax = std::max(v.dmax, v.dims[i]);
    }
    v.D = v.dmin == v.dmax ? v.dmin : 0u;
    return QF_OK;
}

static qf_status check_qudit(const StateView& v, int q, const char* what) {
    QF_RETURN_IF(q < 0 || uint32_t(q) >= v.n, QF_EINVAL, "%s qudit %d outside [0, %u)", what, q, v.n);
    return QF_OK;
}

static qf_status check_finite(const double* a, size_t cnt, const char* what) {
    for (size_t i = 0; i < cnt; ++i)
        QF_RETURN_IF(!std::isfinite(a[i]), QF_EINVAL, "%s contains a non-finite value at %zu", what, i);
    return QF_OK;
}

// Combine one-qudit diagonal terms into per-qudit tables (terms on the same
// qudit add up).  Returns the active qudits and their complex tables back to
// back (d_q values for qudit q, in the order of active).
qf_status combine_terms(const StateView& v, int32_t nterms, const int32_t* term_qudit, const double* term_diag,
                        std::vector<int>& active, std::vector<double>& table) {
    QF_RETURN_IF(nterms < 1, QF_EINVAL, "nterms = %d < 1", nterms);
    QF_RETURN_IF(term_qudit == nullptr || term_diag == nullptr, QF_EINVAL, "term arrays are NULL");
    size_t len = 0;
    for (int t = 0; t < nterms; ++t) {
        QF_CHECK(check_qudit(v, term_qudit[t], "term"));
        len += v.dims[term_qudit[t]];
    }
    QF_CHECK(check_finite(term_diag, len * 2, "term_diag"));
    std::vector<int> off(v.n, -1);
    active.clear();
    table.clear();
    size_t src = 0;
    for (int t = 0; t < nterms; ++t) {
        const int q = term_qudit[t];
        const uint32_t d = v.dims[q];
        if (off[q] < 0) {
            off[q] = int(table.size() / 2);
            active.push_back(q);
            table.resize(table.size() + 2 * d, 0.0);
        }
        for (uint32_t l = 0; l < d; ++l) {
            table[2 * (off[q] + l)] += term_diag[2 * (src + l)];
            table[2 * (off[q] + l) + 1] += term_diag[2 * (src + l) + 1];
        }
        src += d;
    }
    QF_RETURN_IF(table.size() / 2 > 128 || active.size() > 32, QF_ERANGE,
                 "observable tables hold %zu values over %zu qudits (limit 128)", table.size() / 2, active.size());
    return QF_OK;
}

}  // namespace qf

using namespace qf;

extern "C" {

const char* qf_last_error(void) { return g_err; }

int32_t qf_version(void) { return 200; }

qf_status qf_state_init(const qf_state* s, const int32_t* digits, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    std::vector<uint32_t> idx;
    if (digits == nullptr) {
        idx.push_back(0);
    } else {
        bool same = true;
        for (uint32_t b = 0; b < v.batch; ++b) {
            uint32_t x = 0;
            for (uint32_t k = 0; k < v.n; ++k) {
                const int32_t d = digits[size_t(b) * v.n + k];
                QF_RETURN_IF(d < 0 || uint32_t(d) >= v.dims[k], QF_EINVAL,
                             "digit %d of qudit %u of register %u outside [0, %u)", d, k, b, v.dims[k]);
                x = x * v.dims[k] + uint32_t(d);
            }
            if (!idx.empty() && idx[0] != x) same = false;
            idx.push_back(x);
        }
        if (same) idx.resize(1);
    }
    return launch_init(v, idx, reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_apply_1q(const qf_state* s, int32_t q, const double* U, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_CHECK(check_qudit(v, q, "target"));
    QF_RETURN_IF(U == nullptr, QF_EINVAL, "U is NULL");
    QF_CHECK(check_finite(U, size_t(v.dims[q]) * v.dims[q] * 2, "U"));
    return launch_apply_1q(v, q, U, reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_apply_ctrl(const qf_state* s, int32_t ctrl, int32_t tgt, const int32_t* shift, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_CHECK(check_qudit(v, tgt, "target"));
    QF_RETURN_IF(ctrl != -1 && (ctrl < 0 || uint32_t(ctrl) >= v.n), QF_EINVAL, "control qudit %d outside [-1, %u)",
                 ctrl, v.n);
    QF_RETURN_IF(ctrl == tgt, QF_EINVAL, "control and target are both %d", ctrl);
    QF_RETURN_IF(shift == nullptr, QF_EINVAL, "shift is NULL");
    return launch_ctrl(v, ctrl, tgt, shift, reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_apply_diag(const qf_state* s, int32_t k, const int32_t* qudits, const double* phases, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(k < 1 || k > 8 || uint32_t(k) > v.n, QF_EINVAL, "k = %d outside [1, min(8, n)]", k);
    QF_RETURN_IF(qudits == nullptr || phases == nullptr, QF_EINVAL, "qudits or phases is NULL");
    for (int i = 0; i < k; ++i) {
        QF_CHECK(check_qudit(v, qudits[i], "diagonal"));
        for (int j = 0; j < i; ++j)
            QF_RETURN_IF(qudits[i] == qudits[j], QF_EINVAL, "qudit %d listed twice", qudits[i]);
    }
    size_t ntab = 1;
    for (int i = 0; i < k; ++i) ntab *= v.dims[qudits[i]];
    QF_CHECK(check_finite(phases, ntab * 2, "phases"));
    return launch_diag(v, k, qudits, phases, reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_apply_crot(const qf_state* s, int32_t kind, int32_t ctrl, int32_t tgt, int32_t j, int32_t k,
                        double theta, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(kind != QF_OP_CRX && kind != QF_OP_CRY && kind != QF_OP_CRZ, QF_EINVAL,
                 "kind %d is not a controlled rotation", kind);
    QF_CHECK(check_qudit(v, ctrl, "control"));
    QF_CHECK(check_qudit(v, tgt, "target"));
    QF_RETURN_IF(ctrl == tgt, QF_EINVAL, "control and target are both %d", ctrl);
    const uint32_t dt = v.dims[tgt], dc = v.dims[ctrl];
    if (kind == QF_OP_CRZ)
        QF_RETURN_IF(j < 1 || uint32_t(j) >= dt, QF_EINVAL, "R_z level j = %d needs 1 <= j < %u", j, dt);
    else
        QF_RETURN_IF(!(j >= 0 && j < k && uint32_t(k) < dt), QF_EINVAL, "levels (%d, %d) need 0 <= j < k < %u", j, k,
                     dt);
    QF_RETURN_IF(!std::isfinite(theta), QF_EINVAL, "theta is not finite");
    // table for control levels m = 0..d_c-1 (layout in k_crot.hip)
    std::vector<double> tab(size_t(4) * dc, 0.0);
    for (uint32_t m = 0; m < dc; ++m) {
        if (kind == QF_OP_CRZ) {
            const double a = std::sqrt(2.0 / (double(j) * (j + 1)));
            tab[4 * m] = std::cos(-0.5 * m * theta * a);
            tab[4 * m + 1] = std::sin(-0.5 * m * theta * a);
            tab[4 * m + 2] = std::cos(0.5 * m * theta * a * j);
            tab[4 * m + 3] = std::sin(0.5 * m * theta * a * j);
        } else {
            tab[4 * m] = std::cos(0.5 * m * theta);
            tab[4 * m + 1] = std::sin(0.5 * m * theta);
        }
    }
    return launch_crot(v, CrotArgs{kind - QF_OP_CRX, ctrl, tgt, j, k}, nullptr, 0, tab.data(),
                       reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_apply_swap(const qf_state* s, int32_t a, int32_t b, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_CHECK(check_qudit(v, a, "first"));
    QF_CHECK(check_qudit(v, b, "second"));
    QF_RETURN_IF(a == b, QF_EINVAL, "SWAP of qudit %d with itself", a);
    QF_RETURN_IF(v.dims[a] != v.dims[b], QF_EINVAL, "SWAP of qudits of dimensions %u and %u", v.dims[a], v.dims[b]);
    return launch_swap(v, a, b, reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_apply_mcx(const qf_state* s, int32_t nctrl, const int32_t* ctrls, int32_t tgt, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(nctrl < 1 || nctrl > 8, QF_EINVAL, "nctrl = %d outside 1..8", nctrl);
    QF_RETURN_IF(ctrls == nullptr, QF_EINVAL, "ctrls is NULL");
    QF_CHECK(check_qudit(v, tgt, "target"));
    for (int i = 0; i < nctrl; ++i) {
        QF_CHECK(check_qudit(v, ctrls[i], "control"));
        QF_RETURN_IF(ctrls[i] == tgt, QF_EINVAL, "control %d is the target", ctrls[i]);
        for (int j = 0; j < i; ++j) QF_RETURN_IF(ctrls[i] == ctrls[j], QF_EINVAL, "control %d listed twice", ctrls[i]);
    }
    return launch_mcx(v, nctrl, ctrls, tgt, false, reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_apply_rot(const qf_state* s, int32_t kind, int32_t q, int32_t j, int32_t k, double theta,
                       void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(kind != QF_OP_RX && kind != QF_OP_RY && kind != QF_OP_RZ, QF_EINVAL, "kind %d is not a rotation",
                 kind);
    QF_CHECK(check_qudit(v, q, "target"));
    const uint32_t dq = v.dims[q];
    if (kind == QF_OP_RZ)
        QF_RETURN_IF(j < 1 || uint32_t(j) >= dq, QF_EINVAL, "R_z level j = %d needs 1 <= j < %u", j, dq);
    else
        QF_RETURN_IF(!(j >= 0 && j < k && uint32_t(k) < dq), QF_EINVAL, "levels (%d, %d) need 0 <= j < k < %u", j, k,
                     dq);
    QF_RETURN_IF(!std::isfinite(theta), QF_EINVAL, "theta is not finite");
    // the slab kernel's table at control level m = 1 (layout in k_crot.hip)
    std::vector<double> tab(8, 0.0);
    if (kind == QF_OP_RZ) {
        const double a = std::sqrt(2.0 / (double(j) * (j + 1)));
        tab[4] = std::cos(-0.5 * theta * a);
        tab[5] = std::sin(-0.5 * theta * a);
        tab[6] = std::cos(0.5 * theta * a * j);
        tab[7] = std::sin(0.5 * theta * a * j);
    } else {
        tab[4] = std::cos(0.5 * theta);
        tab[5] = std::sin(0.5 * theta);
    }
    return launch_crot(v, CrotArgs{kind - QF_OP_RX, -1, q, j, k}, nullptr, 0, tab.data(),
                       reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_apply_fused(const qf_state* s, int32_t k, int32_t q0, const void* B, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(k < 1 || uint32_t(k) > v.n, QF_EINVAL, "k = %d outside [1, n]", k);
    QF_RETURN_IF(q0 < 0 || uint32_t(q0 + k) > v.n, QF_EINVAL, "qudits %d..%d outside [0, %u)", q0, q0 + k - 1, v.n);
    uint64_t K = 1;
    for (int i = 0; i < k; ++i) K *= v.dims[q0 + i];
    QF_RETURN_IF(K > 1024, QF_ERANGE, "block size D^k = %llu > 1024", (unsigned long long)K);
    QF_RETURN_IF(B == nullptr, QF_EINVAL, "B is NULL");
    return launch_fused(v, k, q0, B, reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_probs(const qf_state* s, int32_t m, const int32_t* qudits, void* out, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(out == nullptr, QF_EINVAL, "out is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (m == 0) {
        QF_RETURN_IF(qudits != nullptr, QF_EINVAL, "m = 0 requires qudits = NULL");
        return launch_probs_full(v, out, false, st);
    }
    QF_RETURN_IF(m < 0 || uint32_t(m) > v.n || m > 32, QF_EINVAL, "m = %d outside [0, min(n, 32)]", m);
    QF_RETURN_IF(qudits == nullptr, QF_EINVAL, "qudits is NULL");
    bool identity = uint32_t(m) == v.n;
    for (int i = 0; i < m; ++i) {
        QF_CHECK(check_qudit(v, qudits[i], "measured"));
        for (int j = 0; j < i; ++j)
            QF_RETURN_IF(qudits[i] == qudits[j], QF_EINVAL, "qudit %d listed twice", qudits[i]);
        identity = identity && qudits[i] == i;
    }
    if (identity) return launch_probs_full(v, out, false, st);
    return launch_probs_marginal(v, m, qudits, out, false, st);
}

qf_status qf_sample(const qf_state* s, int32_t m, const int32_t* qudits, int64_t shots, const double* u,
                    int64_t* counts, int32_t* samples, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(counts == nullptr, QF_EINVAL, "counts is NULL");
    QF_RETURN_IF(shots < 0, QF_EINVAL, "shots = %lld < 0", (long long)shots);
    QF_RETURN_IF(shots > 0 && u == nullptr, QF_EINVAL, "u is NULL");
    QF_RETURN_IF(uint64_t(shots) * v.batch >= (1ull << 32), QF_ERANGE, "batch * shots >= 2^32");
    if (m == 0) {
        QF_RETURN_IF(qudits != nullptr, QF_EINVAL, "m = 0 requires qudits = NULL");
    } else {
        QF_RETURN_IF(m < 0 || uint32_t(m) > v.n || m > 32, QF_EINVAL, "m = %d outside [0, min(n, 32)]", m);
        QF_RETURN_IF(qudits == nullptr, QF_EINVAL, "qudits is NULL");
        bool identity = uint32_t(m) == v.n;
        for (int i = 0; i < m; ++i) {
            QF_CHECK(check_qudit(v, qudits[i], "measured"));
            for (int j = 0; j < i; ++j)
                QF_RETURN_IF(qudits[i] == qudits[j], QF_EINVAL, "qudit %d listed twice", qudits[i]);
            identity = identity && qudits[i] == i;
        }
        if (identity) m = 0;
    }
    uint64_t K = v.N;
    if (m > 0) {
        K = 1;
        for (int i = 0; i < m; ++i) K *= v.dims[qudits[i]];
    }
    QF_RETURN_IF(samples != nullptr && K > (1ull << 31), QF_ERANGE, "%llu outcomes do not fit int32 samples",
                 (unsigned long long)K);
    return launch_sample(v, m, m == 0 ? nullptr : qudits, uint64_t(shots), u, counts, samples,
                         reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_expect(const qf_state* s, int32_t nterms, const int32_t* term_qudit, const double* term_diag,
                    double* out, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(out == nullptr, QF_EINVAL, "out is NULL");
    std::vector<int> active;
    std::vector<double> table;
    QF_CHECK(combine_terms(v, nterms, term_qudit, term_diag, active, table));
    return launch_expect(v, active, table, out, reinterpret_cast<hipStream_t>(stream));
}

qf_status qf_expect_noalloc(const qf_state* s, int32_t nterms, const int32_t* term_qudit, const double* term_diag,
                            double* out, void* stream) {
    StateView v;
    QF_CHECK(make_view(s, v));
    QF_RETURN_IF(out == nullptr, QF_EINVAL, "out is NULL");
    std::vector<int> active;
    std::vector<double> table;
    QF_CHECK(combine_terms(v, nterms, term_qudit, term_diag, active, table));
    return launch_expect_noalloc(v, active, table, out, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
