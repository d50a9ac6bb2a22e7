// Interfaces between the C-ABI layer (abi.cpp, plan.cpp) and the kernel
// launchers (*.hip).  Everything here is host code; arguments are validated by
// the caller.
#pragma once

#include <vector>

#include "qf_common.h"

namespace qf {

constexpr int kMaxDim = 16;
constexpr int kMaxQudits = 32;

// A validated view of a qf_state.  Per-qudit dimensions and strides are
// filled for every register; D is the common dimension, or 0 when the qudits'
// dimensions differ (launchers that need one D then fail with an error).
struct StateView {
    void* amps;
    uint32_t n;
    uint32_t D;
    uint32_t N;       // prod of the dimensions
    uint32_t batch;
    uint32_t total;   // batch * N  (< 2^32)
    int dtype;        // QF_C64 / QF_C128
    uint32_t dims[kMaxQudits];     // d_q
    uint32_t strides[kMaxQudits];  // S_q = d_{q+1} ... d_{n-1}
    uint32_t dmin, dmax;
};

inline uint32_t ipow(uint32_t b, uint32_t e) {
    uint32_t r = 1;
    while (e--) r *= b;
    return r;
}

// A view of a uniform register of batch registers with no amplitudes, for
// sizing work arrays (D^n * batch < 2^32 is the caller's to check).
inline StateView uniform_view(uint32_t D, uint32_t n, uint32_t batch, int dtype) {
    StateView v{};
    v.n = n;
    v.D = v.dmin = v.dmax = D;
    v.N = ipow(D, n);
    v.batch = batch;
    v.total = v.N * batch;
    v.dtype = dtype;
    uint32_t stride = 1;
    for (int i = int(n) - 1; i >= 0; --i) {
        v.dims[i] = D;
        v.strides[i] = stride;
        stride *= D;
    }
    return v;
}

// d_q0 * ... * d_{q0+k-1}
inline uint32_t span(const StateView& s, int q0, int k) {
    uint32_t r = 1;
    for (int i = q0; i < q0 + k; ++i) r *= s.dims[i];
    return r;
}

// ---- per-gate launchers (k_basic.hip) ----
qf_status launch_init(const StateView& s, const std::vector<uint32_t>& index, hipStream_t st);
qf_status launch_apply_1q(const StateView& s, int q, const double* U, hipStream_t st);
qf_status launch_ctrl(const StateView& s, int ctrl, int tgt, const int32_t* shift, hipStream_t st);
qf_status launch_diag(const StateView& s, int k, const int32_t* qudits, const double* phases,
                      hipStream_t st);
// x_tgt -> x_tgt +/- prod_i x_{ctrls[i]} mod D (1 <= nctrl <= 8); inverse subtracts.
qf_status launch_mcx(const StateView& s, int nctrl, const int32_t* ctrls, int tgt, bool inverse, hipStream_t st);
// Exchange the digits of qudits a and b (a != b).
qf_status launch_swap(const StateView& s, int a, int b, hipStream_t st);
// Probabilities in the state's precision, or in FP64 when f64 is set.
qf_status launch_probs_full(const StateView& s, void* out, bool f64, hipStream_t st);
qf_status launch_probs_marginal(const StateView& s, int m, const int32_t* qudits, void* out, bool f64,
                                hipStream_t st);
// Measurement shots (k_sample.hip): m = 0 samples the full register, else the
// marginal of the m listed qudits; u holds batch * shots uniforms in [0, 1),
// counts batch * D^m (or D^n) bins, samples (NULL or batch * shots) the drawn
// bin of each shot.
qf_status launch_sample(const StateView& s, int m, const int32_t* qudits, uint64_t shots, const double* u,
                        int64_t* counts, int32_t* samples, hipStream_t st);
// table: per active qudit D complex values (combined terms), active: qudit list
qf_status launch_expect(const StateView& s, const std::vector<int>& active,
                        const std::vector<double>& table, double* out, hipStream_t st);
// Same with a caller workspace of expect_ws_doubles(s) doubles (no allocation).
size_t expect_ws_doubles(const StateView& s);
qf_status launch_expect_ws(const StateView& s, const std::vector<int>& active, const std::vector<double>& table,
                           double* out, double* ws, hipStream_t st);
// Same with the library's static scratch array (no allocation; QF_ERANGE past its size).
qf_status launch_expect_noalloc(const StateView& s, const std::vector<int>& active, const std::vector<double>& table,
                                double* out, hipStream_t st);
// Elementwise lam = f(x) * psi with f(x) = sum over active qudits of the real
// table value (the Hermitian part of a diagonal observable).
qf_status launch_diag_observable(const StateView& psi, void* lam_amps, const std::vector<int>& active,
                                 const std::vector<double>& table_re, hipStream_t st);

// ---- controlled rotation (k_crot.hip) ----
// sum_m |m><m|_ctrl (x) R(m theta)_tgt; kind 0 = x, 1 = y, 2 = z type; with
// ctrl = -1 the plain rotation R(theta) (table entry m = 1 for every fibre:
// the two-level slab kernel, which reads and writes only the levels the
// rotation moves).  The
// table holds 2*D complex entries per register (see k_crot.hip), from the
// device (dtab, register stride tab_stride) or, when dtab is NULL, from htab
// (host, 2*D complex FP64, shared by every register).
struct CrotArgs {
    int kind;
    int ctrl, tgt;
    int j, k;
};
qf_status launch_crot(const StateView& s, const CrotArgs& a, const void* dtab, size_t tab_stride, const double* htab,
                      hipStream_t st);
// Un-applies the gate (inverse table) on psi and lam and writes, per register b,
// sum over fibres of m * Im <lam_f| S |psi_f> to out[b * ostride].  partial:
// crot_partial_doubles(s) doubles of scratch.
qf_status launch_crot_adj(const StateView& s, void* lam, const CrotArgs& a, const void* dtab, size_t tab_stride,
                          const double* htab, double* partial, double* out, uint32_t ostride, hipStream_t st);
size_t crot_partial_doubles(const StateView& s);

// ---- fused dense blocks (k_fused.hip) ----
// real: every imaginary part of B is zero (halves the matrix-core products).
qf_status launch_fused(const StateView& s, int k, int q0, const void* B, hipStream_t st, bool real = false);

}  // namespace qf

namespace qf {

// ---- fused LDS stages (k_stage.hip) ----
//
// A stage keeps a tile of k qudits of one register in LDS: the r least
// significant qudits (a contiguous run of R = D^r amplitudes in HBM) plus k - r
// further qudits.  The other n - k qudits are fixed per tile.  The tile's local
// index e has the tile qudits in increasing qudit order (most significant
// first); the global index of local element e is
//   base(tile) + offhi[e / R] + e % R.
constexpr int kMaxTileDims = 16;
constexpr int kMaxOuter = 32;
constexpr int kMaxHi = 1024;  // D^(k-r) entries of the offhi table
constexpr int kMaxPairs = 8;

struct StageGeom {
    uint32_t k, r;       // tile qudits, low (contiguous) qudits
    uint32_t TE;         // D^k tile elements
    uint32_t R;          // D^r
    uint32_t nhi;        // D^(k-r)
    uint32_t ntiles;     // D^(n-k) tiles per register
    uint32_t N;          // D^n
    uint32_t nout;       // n - k
    FastDiv divR;
    uint32_t xcd;        // 1: tiles grouped per XCD (tile_of_block), 0: dispatch order
    uint32_t hi_stride[kMaxTileDims];  // global strides of the high tile qudits, most significant first
    uint32_t out_stride[kMaxOuter];    // global strides of the outer qudits, most significant first
};

enum StageOpType : int32_t { SOP_U = 0, SOP_SHIFT = 1, SOP_PHASE = 2 };

// Register rounds of a stage: each lane holds a sub-tile of D^M amplitudes
// (every combination of the M group qudits) in registers and applies the
// round's in-place ops [op0, op0 + nops) (U, PHASE) to it; the group position
// of each op's qudits is stored in the op (gpos, agpos/bgpos).  Permutation
// ops (SHIFT) are folded into the LDS addresses: pre0 (target position 0,
// control position 1, outside the group or none) and then pre1 (target
// position 1, control position 0) before the in-place ops, post (like pre0)
// after them.
constexpr int kMaxGroup = 5;
// Round shapes with a dispatch-free kernel path (RK_GENERIC: anything else).
enum RoundKind : int32_t {
    RK_GENERIC = 0,
    RK_NONE = 1,     // no in-place op (a permutation only)
    RK_U0 = 2,       // one complex U on group position 0
    RK_U0_REAL = 3,  // one real U on group position 0
    RK_U01 = 4,      // two complex U on group positions 0 and 1
    RK_U1 = 5,       // one complex U on group position 1
    RK_U1_REAL = 6,  // one real U on group position 1
    RK_PHASE = 7,    // one PHASE op
};
// A permutation op folded into a round's loads or stores (a copy of its op's
// fields, so that the round reads them with its own descriptor).
struct PermDesc {
    int32_t has_ctrl;       // 1 if controlled
    int32_t ctrl_gpos;      // group position of the control, -1 = not in the group
    int32_t shift_mul;      // shifts[c] = (shift_mul * c + shifts[0]) mod D, or -1 if not affine
    FastDiv ctrl_stride;    // global stride of the control qudit
    int32_t shifts[16];     // x_t -> x_t + shifts[x_c]
};

struct RoundDesc {
    int32_t kind;
    int32_t op0, nops;
    int32_t pre0, pre1, post;       // permutation ops, -1 = none
    int32_t need_gidx;              // some op reads a digit from the global index
    uint32_t gls[kMaxGroup];        // LDS strides of the group qudits, register digit 0 first
    uint32_t glsb[kMaxGroup];       // the same in bytes (amplitudes of the plan's dtype)
    int32_t nother;                 // k - M
    uint32_t ols[kMaxTileDims];     // LDS strides of the other tile qudits, most significant first
    uint32_t spair[4];              // the last 8 of ols, least significant first, two 16-bit halves per word
    // copies of op fields the round's common shapes read, so that a round needs
    // no op lookup before its matrix loads or its addresses
    int32_t mat0, mat1;             // U shapes: matrix offset of the U on position 0 (or the one U), position 1
    PermDesc perm[3];               // the pre0, pre1 and post permutations (where present)
    // pre2 (groups of 2): a permutation after pre0 and pre1 whose target t is a
    // tile qudit outside the group and whose control is group position 1; the
    // lane's digit x_t loads from x_t - pre2_shifts[d_1]
    int32_t pre2;                   // its op, -1 = none
    int32_t pre2_byte;              // byte of the sub-tile digits (sub_digits) that holds x_t
    uint32_t pre2_lsb;              // LDS stride of t in bytes
    int32_t pre2_shifts[16];
    int32_t mslot, mpos;            // adjoint: M slot and group position of the U that opens the round, -1 = none
};

struct StageOp {
    int32_t type;
    int32_t dim;          // local tile dimension (U, SHIFT)
    uint32_t ls;          // LDS stride of dim, D^(k-1-dim)
    FastDiv divls;
    int32_t has_ctrl;     // SHIFT: 1 if controlled
    FastDiv ctrl_stride;  // SHIFT: global stride of the control qudit
    int32_t shifts[16];   // SHIFT: x_t -> x_t + shifts[x_c] (already in [0, D))
    int32_t shift_mul;    // SHIFT: shifts[c] = (shift_mul * c + shifts[0]) mod D, or -1 if not affine
    int32_t mat;          // U: offset (complex elements) of the D x D matrix
    int32_t real;         // U: all imaginary parts are zero
    int32_t slot;         // adjoint: M slot of this U inside the stage, -1 = none
    int32_t npairs;       // PHASE: number of two-qudit diagonal factors
    FastDiv pa[kMaxPairs], pb[kMaxPairs];  // PHASE: global strides of the two qudits
    int32_t ptab[kMaxPairs];               // PHASE: offset of each D x D table (complex)
    // register-round form (forward stages)
    int32_t gpos;         // U, SHIFT: group position of the target
    int32_t ctrl_gpos;    // SHIFT: group position of the control, -1 = not in the group
    int32_t agpos[kMaxPairs], bgpos[kMaxPairs];  // PHASE: group positions, -1 = not in the group
    int32_t wtab;         // PHASE: offset of the D-entry table w^e (e = sum of x_a x_b mod D)
};

// mat_stride: complex elements between the matrices of consecutive registers
// (0: every register uses the same matrices).
qf_status launch_stage(const StateView& s, const StageGeom& g, const StageOp* dops, int nops, const void* dmats,
                       hipStream_t st, size_t mat_stride = 0);
// Register-round form with groups of M qudits (1 <= M <= max_group_size(D)).
int max_group_size(uint32_t D);
qf_status launch_stage_rounds(const StateView& s, int M, const StageGeom& g, const RoundDesc* drounds, int nrounds,
                              const StageOp* dops, const void* dmats, hipStream_t st, size_t mat_stride = 0);
// Reverse stage: applies the (already inverted) ops to psi and lam; before each
// U with slot >= 0 it accumulates M = sum_f psi_f lam_f^dagger over the tile
// into partial[(slot * nblocks + block) * D*D] (complex FP64).
qf_status launch_stage_adj(const StateView& s, void* lam, const StageGeom& g, const StageOp* dops, int nops,
                           const void* dmats, double* partial, hipStream_t st, size_t mat_stride = 0);
// Pipelined persistent forward stage (register rounds, M <= 3, D <= 12, complex64): grid of at most
// 256 * wgs_per_cu workgroups; needs stage_pipe_ok(g) (runs shorter than a
// workgroup, at most 32 runs per lane).
bool stage_pipe_ok(const StageGeom& g);
qf_status launch_stage_pipe(const StateView& s, int M, const StageGeom& g, const RoundDesc* drounds, int nrounds,
                            const StageOp* dops, const void* dmats, int wgs_per_cu, hipStream_t st,
                            size_t mat_stride = 0);
// Reverse stage in register rounds (M in {1, 2}); a U owning an M slot opens its round.
qf_status launch_stage_adj_rounds(const StateView& s, void* lam, int M, const StageGeom& g, const RoundDesc* drounds,
                                  int nrounds, const StageOp* dops, const void* dmats, double* partial, hipStream_t st,
                                  size_t mat_stride = 0);
// mout[(b * nslots_total + slot0 + j) * E] = sum over the tiles of register b of
// partial[j], for j < nslots (fixed order).
qf_status launch_stage_mreduce(const double* partial, uint32_t nslots, uint32_t ntiles, uint32_t batch, uint32_t E,
                               double* mout, uint32_t nslots_total, uint32_t slot0, hipStream_t st);
size_t stage_lds_bytes(const StageGeom& g, int dtype, bool adjoint);

}  // namespace qf

namespace qf {

// ---- device-side parameters (k_params.hip) ----
// A forward-order gate of a fused run (kinds: QF_OP_H, CLOCK, RX, RY, RZ).
struct DevGate {
    int32_t kind, j, k, param;
};
// One matrix a register needs: a fused run product, a CZ table or a w^e table.
enum DevGroupType : int32_t { DG_U = 0, DG_CZ = 1, DG_W = 2, DG_CR = 3 };
struct DevGroup {
    int32_t type;
    uint32_t mat_off;  // complex elements from the start of a register's matrices
    int32_t g0, ng;    // DG_U: gates [g0, g0 + ng) of the gate list, application order; DG_CR: gate g0
    int32_t inv;       // DG_U: every gate is applied as its inverse; DG_CZ / DG_W: conjugated
};
// A fused run that owns an adjoint M slot; its gates in forward order.
struct DevGradGroup {
    int32_t gslot;
    int32_t g0, ng;    // forward-order gates in the gate list
    int32_t c0;        // first contribution slot (one per rotation of the run)
};

qf_status launch_build_mats(int D, int dtype, const DevGroup* groups, int ngroups, const DevGate* gates,
                            const double* theta, int64_t theta_stride, uint32_t batch, void* mats, size_t mat_stride,
                            hipStream_t st);
qf_status launch_grad(int D, const DevGradGroup* gg, int ngg, const DevGate* gates, const double* theta,
                      int64_t theta_stride, const double* M, int nslots, uint32_t batch, double* contrib, int ncontrib,
                      const int32_t* p_off, const int32_t* p_list, int nparams, double scale, double* grad,
                      hipStream_t st);

}  // namespace qf
