/*
 * qf.h - C ABI of the MI355X (gfx950) qudit state-vector library.
 *
 * The library applies qudit gates to a dense complex state vector of D^n
 * amplitudes, then computes measurement probabilities, diagonal expectation
 * values and adjoint-method gradients.  The gate set and conventions follow
 * Friedrich & Maziero, "QuForge: A Library for Qudits Simulation"
 * (arXiv:2409.17716), Appendix "Matrix form of the quantum gates".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Basis index (decimal representation, subsection "Generalized CNOT gate"):
 *    for digits (x_0, ..., x_{n-1}), x = sum_k x_k D^(n-1-k).  Qudit 0 is the
 *    most significant digit; the stride of qudit q is D^(n-1-q).
 *  - Levels are 0-indexed (the paper programs {|j>}_{j=0}^{D-1}).
 *  - Amplitudes are interleaved (re, im): complex64 = 2 x float, complex128 =
 *    2 x double, exactly torch.complex64 / torch.complex128 memory.
 *  - A state holds `batch` registers of D^n amplitudes back to back.
 *  - Host matrices and tables are always complex FP64 (interleaved doubles);
 *    the library casts them to the state's precision.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *    only enqueues work on it, except those documented as synchronising.
 *
 * Ownership: the caller owns every state, output and device matrix buffer.
 * Host arrays are read before the call returns and may be freed right after.
 * The library owns plan objects (freed by qf_plan_destroy) and stream-ordered
 * temporary reduction buffers (allocated and freed on `stream`, from the
 * device's default pool, which keeps up to 4 GiB of freed memory for reuse
 * until qf_shutdown).
 *
 * Errors: argument validation is synchronous and enqueues nothing on failure.
 * A failed HIP launch returns QF_EHIP.  Faults inside a kernel surface at the
 * caller's next synchronisation.  No C++ exception crosses this ABI.
 * qf_last_error() returns a thread-local message describing the last non-OK
 * status of the calling thread.
 *
 * Limits: 2 <= dim <= 16; n >= 1; batch * dim^n < 2^32 amplitudes per call.
 * Host D x D matrices of the per-gate calls travel as kernel arguments, so
 * complex128 states accept dim <= 11 in qf_apply_1q.
 */
#ifndef QF_H
#define QF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QF_OK = 0,
    QF_EINVAL = -1,        /* bad argument: index out of range, NULL pointer, ...   */
    QF_EDTYPE = -2,        /* unknown dtype or dtype mismatch                       */
    QF_ERANGE = -3,        /* size beyond the documented limits                     */
    QF_ENOMEM = -4,        /* device or host allocation failed                      */
    QF_EHIP = -5,          /* a HIP runtime call failed                             */
    QF_EUNSUPPORTED = -6   /* valid request this build does not implement           */
} qf_status;

typedef enum { QF_C64 = 0, QF_C128 = 1 } qf_dtype;

/* A register (or a batch of registers) in device memory.
 *
 * Uniform registers (dims = NULL): every qudit has dim levels (D).  Mixed
 * registers (the paper's multidimensional circuits, section "Related work",
 * Table 1, and the dim=[2,3,4] example of section "Code style"): dims lists
 * the levels d_q of every qudit (2..16) and dim must be 0; an array whose
 * entries are all equal describes a uniform register.  In both the basis index
 * is x = sum_q x_q S_q with S_q = d_{q+1} ... d_{n-1} (qudit 0 most
 * significant).  Below, d_q is the dimension of qudit q (D for a uniform
 * register) and "outcomes" / table sizes are the products of the d_q involved.
 * Across dimensions the two-qudit gates act as: controlled shift / CSUM
 * x_t -> (x_t + shift[x_c]) mod d_t; controlled phase w_{d_t}^(x_c x_t);
 * controlled rotation over the d_c control levels in the target's dimension;
 * multi-controlled shift x_t -> (x_t + prod x_c) mod d_t; SWAP only between
 * qudits of equal dimension.  Plans on mixed registers run the per-gate
 * schedules (qf_plan_create_dims). */
typedef struct qf_state {
    void*   amps;    /* device pointer, batch * prod(d_q) complex elements          */
    int32_t n;       /* qudits per register                                          */
    int32_t dim;     /* levels per qudit (D); 0 when dims is set                    */
    int64_t batch;   /* registers stored back to back                                */
    int32_t dtype;   /* qf_dtype                                                     */
    const int32_t* dims; /* host, n per-qudit dimensions, or NULL (uniform)          */
} qf_state;

/* ------------------------------------------------------------------------- */
/* Per-gate entry points                                                     */
/* ------------------------------------------------------------------------- */

/* psi = |j_0 j_1 ... j_{n-1}> in every register (the paper's State('j0-j1-..'),
 * section "Code style").  digits: host, batch*n values, digit k in [0, d_k)
 * (register b uses digits[b*n .. b*n+n-1]); NULL means |0...0> everywhere. */
qf_status qf_state_init(const qf_state* s, const int32_t* digits, void* stream);

/* One-qudit gate: psi[h, :, l] <- U psi[h, :, l] with the register viewed as
 * [D^q][D][D^(n-1-q)] (a D x D matrix acting on qudit q, identity elsewhere;
 * subsections "Fourier gate", "Generalized rotation gate", "Generalized
 * phase-shift gate"); on a mixed register [S_q-blocks][d_q][S_q] with a
 * d_q x d_q matrix.  U: host, d_q*d_q complex FP64, row-major (U[a*d_q+b] is
 * <a|U|b>).  q in [0, n).  The matrix need not be unitary. */
qf_status qf_apply_1q(const qf_state* s, int32_t q, const double* U, void* stream);

/* Controlled shift, a pure index permutation (subsections "Generalized NOT
 * gate" and "Generalized CNOT gate"): |.. x_c .. x_t ..> ->
 * |.. x_c .. (x_t + shift[x_c]) mod D ..>.  The generalized CNOT (CSUM) is
 * shift[c] = c; the shift gate X_s is ctrl = -1 with shift[0] = s.
 * shift: host, d_ctrl entries (only shift[0] is read when ctrl = -1), any
 * integers (reduced mod d_tgt).  ctrl != tgt, both in [0, n) (ctrl may be -1).
 * Bit-exact: amplitudes are moved, never recomputed. */
qf_status qf_apply_ctrl(const qf_state* s, int32_t ctrl, int32_t tgt,
                        const int32_t* shift, void* stream);

/* Diagonal gate on k qudits: psi_x <- phases[y] psi_x with
 * y = sum_i x_{qudits[i]} D^(k-1-i) (mixed: the mixed-radix number of those
 * digits over their dimensions, first listed most significant).  Covers the
 * phase-shift (clock) gate and
 * its powers (subsection "Generalized phase-shift gate"), R_z (subsection
 * "Generalized rotation gate", diagonal generator) and a controlled phase
 * w^(x_c x_t) built from the same phase rule.
 * qudits: host, k distinct indices in [0, n); phases: host, D^k (prod of the
 * listed d_q) complex FP64.  Limit: D^k <= 256 (complex64) or 128 (complex128). */
qf_status qf_apply_diag(const qf_state* s, int32_t k, const int32_t* qudits,
                        const double* phases, void* stream);

/* The paper's differentiable controlled rotation (Appendix, subsection
 * "Controlled Rotation Gate"): sum_m |m><m|_ctrl (x) R(m theta)_tgt with
 * R = exp(-i theta S / 2) and S = S_x^{jk} (kind QF_OP_CRX), S_y^{jk}
 * (QF_OP_CRY, j < k) or the diagonal S_z^{j} (QF_OP_CRZ, 1 <= j < D, k ignored);
 * m runs over the control's d_ctrl levels, the levels over the target's d_tgt.
 * ctrl != tgt, both in [0, n); theta in radians.  The x and y types read and
 * write only target levels j and k; the control's level-0 slab is untouched. */
qf_status qf_apply_crot(const qf_state* s, int32_t kind, int32_t ctrl, int32_t tgt,
                        int32_t j, int32_t k, double theta, void* stream);

/* A single rotation exp(-i theta S / 2) (subsection "Generalized rotation
 * gate"; kind QF_OP_RX / QF_OP_RY with levels j < k, or QF_OP_RZ with
 * 1 <= j < D) as a slab sweep: only the levels it moves are read and written
 * (2 of D for R_x, R_y; j + 1 for R_z), the memory form of the paper's sparse
 * rotation.  Same result as qf_apply_1q with the rotation's matrix. */
qf_status qf_apply_rot(const qf_state* s, int32_t kind, int32_t q, int32_t j, int32_t k,
                       double theta, void* stream);

/* SWAP of qudits a and b (subsection "Generalized SWAP Gate"): the digits of
 * a and b are exchanged, |.. x_a .. x_b ..> -> |.. x_b .. x_a ..>.  a != b, both
 * in [0, n), d_a = d_b.  Bit-exact: amplitudes are moved, never recomputed. */
qf_status qf_apply_swap(const qf_state* s, int32_t a, int32_t b, void* stream);

/* Multi-controlled shift (the Toffoli and multi-controlled NOT gates the paper
 * names in section "Quantum Gates", generalized like its CNOT index rule):
 * |.. x_t ..> -> |.. (x_t + prod_i x_{ctrls[i]}) mod d_t ..>.  For qubits this is
 * the Toffoli (2 controls) / multi-controlled NOT; with one control it is CSUM.
 * ctrls: host, nctrl (1..8) distinct qudits, none equal to tgt.  Bit-exact. */
qf_status qf_apply_mcx(const qf_state* s, int32_t nctrl, const int32_t* ctrls, int32_t tgt,
                       void* stream);

/* Custom dense gate on the k adjacent qudits q0..q0+k-1 (the paper's
 * U(matrix, index), section "Grover's algorithm"): psi[h, :, l] <- B psi[h, :, l]
 * with the register viewed as [D^q0][D^k][D^(n-q0-k)] (mixed: K = d_q0 ... d_{q0+k-1}
 * in place of D^k).
 * B: DEVICE pointer, D^k x D^k row-major in the state's precision (complex64
 * or complex128), caller-owned, read during the kernel.  complex64 blocks with
 * D^k >= 32 run on FP32 matrix cores; others on vector ALUs.  D^k <= 1024. */
qf_status qf_apply_fused(const qf_state* s, int32_t k, int32_t q0, const void* B,
                         void* stream);

/* Measurement probabilities (section "Code style": measure returns p).
 * m = 0 and qudits = NULL: full distribution p_x = |psi_x|^2, out holds
 * batch*D^n reals.  Otherwise the marginal of the listed qudits in the listed
 * order, p(y) = sum_{x : x_qudits = y} |psi_x|^2 with y = sum_i y_i D^(m-1-i)
 * (mixed: the mixed-radix number of the y_i over the listed qudits' dimensions);
 * out holds batch*D^m reals (batch * prod of the listed d_q).  out: DEVICE, float for complex64 states, double
 * for complex128.  Marginals accumulate in FP64 in a fixed order (bitwise
 * reproducible run to run). */
qf_status qf_probs(const qf_state* s, int32_t m, const int32_t* qudits, void* out,
                   void* stream);

/* Measurement shots (section "Code style": measure with a shot count returns
 * the histogram of outcomes).  Draw i of register b takes the uniform
 * u[b*shots + i] and returns the first outcome y whose cumulative
 * probability (prefix sum of the distribution qf_probs defines, taken in FP64
 * in a fixed order) exceeds u * total, total being the register's summed
 * probability (the state need not be normalised); a product that reaches the
 * total (u >= 1 after rounding) gives the last outcome of non-zero
 * probability, and a register of zero norm gives outcome 0.
 * m, qudits: as qf_probs (m = 0 with qudits = NULL: the full register, D^n
 * outcomes; else D^m outcomes of the listed qudits, first listed most
 * significant).  shots >= 0 per register.
 * u: DEVICE, batch*shots doubles in [0, 1), caller-drawn (NULL when shots = 0).
 * counts: DEVICE, batch*(outcomes) int64, overwritten with the histogram.
 * samples: DEVICE, batch*shots int32 outcomes, or NULL.
 * All caller-owned.  Errors: QF_EINVAL (bad pointers or qudits), QF_ERANGE
 * when batch*outcomes or batch*shots reaches 2^32, or samples are asked for
 * with more than 2^31 outcomes; QF_ENOMEM when the FP64 work array
 * (about 8 bytes per outcome and register) cannot be allocated. */
qf_status qf_sample(const qf_state* s, int32_t m, const int32_t* qudits, int64_t shots,
                    const double* u, int64_t* counts, int32_t* samples, void* stream);

/* Expectation of a diagonal observable that is a sum of one-qudit terms,
 * <O> = sum_x |psi_x|^2 sum_t term_diag[t][x_{term_qudit[t]}]
 * (e.g. Z_0 with Z = diag(w^k), or sum_i Z_i).  term_qudit: host, nterms
 * indices in [0, n); term_diag: host, nterms*D complex FP64 (mixed: the terms'
 * tables back to back, d_q values for a term on qudit q).
 * out: DEVICE, batch complex128 values (2 doubles each), accumulated in FP64
 * in a fixed order.  Limit: the distinct qudits' tables hold <= 128 values. */
qf_status qf_expect(const qf_state* s, int32_t nterms, const int32_t* term_qudit,
                    const double* term_diag, double* out, void* stream);

/* qf_expect for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and summation order (bitwise the same result), with the
 * partial sums in a library-owned device array of 4 MiB per GPU, held until
 * the process ends, instead of a stream-ordered allocation.  Calls no
 * allocating routine.  Limit: batch * (chunks per register) <= 262144 partial
 * sums, a register splitting into chunks of its smallest qudit stride of at
 * least 4096 amplitudes (one chunk if it has none); so batch * ceil(N / 4096)
 * <= 262144 always fits (one register of up to 2^30 amplitudes).  Beyond the
 * limit QF_ERANGE.  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * threads) race, so the caller must order them. */
qf_status qf_expect_noalloc(const qf_state* s, int32_t nterms, const int32_t* term_qudit,
                            const double* term_diag, double* out, void* stream);

/* ------------------------------------------------------------------------- */
/* Circuit programs (plans): fused forward and adjoint gradient              */
/* ------------------------------------------------------------------------- */

typedef enum {
    QF_OP_H = 0,       /* Fourier gate on q0                                      */
    QF_OP_X = 1,       /* shift x_q0 -> x_q0 + a mod D                             */
    QF_OP_CLOCK = 2,   /* Z^a = diag(w^(a k)) on q0                                */
    QF_OP_RX = 3,      /* exp(-i theta S_x^{jk} / 2) on q0                         */
    QF_OP_RY = 4,      /* exp(-i theta S_y^{jk} / 2) on q0                         */
    QF_OP_RZ = 5,      /* exp(-i theta S_z^{j} / 2) on q0, 1 <= j < D              */
    QF_OP_CSUM = 6,    /* x_q1 -> x_q1 + x_q0 mod D  (q0 control, q1 target)       */
    QF_OP_CSHIFT = 7,  /* x_q1 -> x_q1 + shifts[x_q0] mod D                        */
    QF_OP_CZ = 8,      /* phase w^(x_q0 x_q1)                                      */
    QF_OP_U = 9,       /* dense D^k x D^k matrix `mat` on qudits q0..q0+k-1        */
    QF_OP_CRX = 10,    /* controlled rotation sum_m |m><m|_q0 (x) R_x^{jk}(m theta)_q1 */
    QF_OP_CRY = 11,    /* the same with R_y^{jk}                                   */
    QF_OP_CRZ = 12,    /* the same with R_z^{j}, 1 <= j < D                        */
    QF_OP_SWAP = 13,   /* exchange the digits of q0 and q1                         */
    QF_OP_MCX = 14     /* x_q1 -> x_q1 + prod_i x_{shifts[i]} mod D, i < j (1..8   */
                       /* controls listed in shifts[0 .. j-1])                     */
} qf_op_kind;

typedef struct qf_op {
    int32_t kind;        /* qf_op_kind                                              */
    int32_t q0;          /* target of one-qudit gates; control of CSUM/CSHIFT/CZ;    */
                         /* first qudit of U                                         */
    int32_t q1;          /* target of CSUM/CSHIFT/CZ/CR*; k (qudit count) of U       */
    int32_t j, k;        /* levels: RX/RY use j < k; RZ uses j; X and CLOCK use j as */
                         /* the shift / exponent a                                   */
    int32_t param;       /* rotation angle slot in theta, -1 for fixed gates; a     */
                         /* CLOCK with param >= 0 takes its exponent a from theta    */
    int32_t shifts[16];  /* CSHIFT table (first D entries used)                      */
    const double* mat;   /* U: host D^k x D^k complex FP64, copied at plan creation  */
} qf_op;

typedef struct qf_plan qf_plan;

/* Plan options.  Zero-initialised options select the defaults. */
typedef struct qf_plan_opts {
    int32_t fuse;         /* 0 = fused LDS stages (default); 1 = one kernel per gate; */
                          /* 2 = one kernel per run of one-qudit gates on a qudit;    */
                          /* 3 = stages, with the one-qudit runs of qudit pairs       */
                          /* (2i, 2i+1) applied as dense D^2 x D^2 blocks (matrix    */
                          /* cores for complex64 when D^2 >= 32)                      */
    int32_t tile_digits;  /* qudits per LDS tile of the forward stages; 0 = chosen    */
                          /* from D and the LDS budget                                */
    int32_t low_digits;   /* least significant qudits always in the tile (contiguous */
                          /* HBM runs); 0 = chosen from D                             */
    int32_t ckpt_every;   /* keep a state checkpoint every this many gates of the    */
                          /* circuit for the adjoint; 0 = none                        */
    int32_t adj_tile_digits; /* qudits per tile of the adjoint stages; 0 = chosen     */
    int32_t stage_kernel; /* forward stages: 0 = register rounds (default), 1 = one   */
                          /* LDS sweep per op, 2 = register rounds in a pipelined     */
                          /* persistent kernel (next tile's loads overlap compute;    */
                          /* complex64 and D <= 12 only, otherwise runs as 0)         */
    int32_t group_digits; /* register rounds: qudits per lane group; 0 = chosen from D */
    int32_t pipe_wgs;     /* stage_kernel 2: workgroups per compute unit; 0 = 4        */
    int32_t tile_order;   /* 0 = each XCD (own L2) walks a contiguous range of tiles  */
                          /* (default); 1 = tiles in plain dispatch order            */
    int32_t tile_search;  /* stage tiles: 0 = the greedy choice, and for states of   */
                          /* at least 2^20 amplitudes also the greedy choice improved */
                          /* by single-qudit swaps, keeping the plan with fewer      */
                          /* passes (default); 1 = greedy only; 2 = as 0 at any size */
} qf_plan_opts;

/* Compile a circuit (ops applied in order) for registers of n qudits of
 * dimension dim in precision dtype.  Fixed gates are built here; rotation
 * matrices are rebuilt from theta on each qf_plan_forward / qf_adjoint_grad.
 * Consecutive gates are grouped into stages that each make one pass over HBM.
 * nparams: length of theta.  *out receives the plan. */
qf_status qf_plan_create(int32_t dim, int32_t n, int32_t dtype, const qf_op* ops,
                         int32_t nops, int32_t nparams, const qf_plan_opts* opts,
                         qf_plan** out);

/* qf_plan_create for a register of per-qudit dimensions dims[0..n-1] (each
 * 2..16; host, read during the call).  Levels, shifts, exponents and U blocks
 * of every op are taken in the dimensions of the qudits they act on (a U on
 * q0..q0+k-1 is (d_q0 ... d_{q0+k-1})^2 entries; a CSHIFT table has d_c
 * entries; SWAP needs equal dimensions).  Equal entries give the uniform plan
 * of qf_plan_create.  Mixed dimensions run the per-gate schedules: opts.fuse
 * 1 or 2 (0 selects 2); fuse 3, checkpoints, qf_plan_bind and
 * qf_plan_autotune return QF_EUNSUPPORTED.  States used with the plan must
 * carry the same dims. */
qf_status qf_plan_create_dims(const int32_t* dims, int32_t n, int32_t dtype, const qf_op* ops,
                              int32_t nops, int32_t nparams, const qf_plan_opts* opts,
                              qf_plan** out);

/* Number of kernel passes over the state in the plan's forward schedule. */
int32_t qf_plan_num_stages(const qf_plan* plan);

/* Number of kernel passes of the plan's adjoint (reverse) schedule. */
int32_t qf_plan_num_adjoint_stages(const qf_plan* plan);

/* Per-kernel timing of a plan's launches, measured with HIP events recorded
 * around every pass on the launch stream while profiling is enabled. */
typedef struct qf_kernel_stat {
    char    name[32];     /* kernel family: "stage", "stage_adj", "fused", ...     */
    int64_t launches;
    double  total_ms;     /* summed event-to-event durations                       */
    double  bytes;        /* summed algorithmic HBM bytes (each pass reads and     */
                          /* writes its state(s) once)                             */
} qf_kernel_stat;

/* enable != 0 starts recording (and clears earlier records). */
qf_status qf_plan_set_profiling(qf_plan* plan, int32_t enable);

/* Waits for the recorded events, writes up to cap per-family sums to out and
 * the number of families to *count, then clears the records. */
qf_status qf_plan_read_profile(qf_plan* plan, qf_kernel_stat* out, int32_t cap, int32_t* count);

/* Apply the planned circuit in place to every register of s (shape must match
 * the plan).  theta: host, nparams angles in radians. */
qf_status qf_plan_forward(qf_plan* plan, const qf_state* s, const double* theta,
                          void* stream);

/* Flags of the adjoint entry points. */
#define QF_SEED 1u  /* lam holds the seed on input (see qf_adjoint_grad) */

/* Adjoint-method gradient of a real loss L(psi) of the final state
 * psi = circuit(theta) psi0 (Jones & Gacon, arXiv:2009.02823; rotations
 * R = exp(-i theta S / 2), subsection "Generalized rotation gate", give
 * dL/dtheta = Im <lam|S|psi> with lam = dL/d(conj psi) carried back through the
 * circuit together with psi).
 *  - flags = 0: L = Re <psi| O |psi> for O a sum of one-qudit diagonal terms
 *    (as in qf_expect); lam is scratch, the library sets lam = H_O psi with
 *    H_O = (O + O^dagger) / 2.
 *  - flags = QF_SEED: L is any real function of psi (the paper's training
 *    losses, section "Code style"); on input lam holds g = 2 dL/d(conj psi),
 *    the gradient torch's complex autograd delivers for psi.  nterms,
 *    term_qudit and term_diag are ignored.
 * psi: in = the final state produced by qf_plan_forward; out = clobbered
 * (un-applied back towards psi0).  lam: same shape, clobbered.  A plan with
 * checkpoints (ckpt_every > 0) re-anchors psi from the checkpoints of the last
 * qf_plan_forward, which must have run on this same psi buffer and batch
 * (QF_EINVAL otherwise).
 * grad: host, batch*nparams doubles (register b writes grad[b*nparams ..]).
 * Synchronises `stream` before returning. */
qf_status qf_adjoint_grad(qf_plan* plan, const qf_state* psi, const qf_state* lam,
                          const double* theta, int32_t nterms,
                          const int32_t* term_qudit, const double* term_diag,
                          double* grad, uint32_t flags, void* stream);

/* ---- device-parameter (bound) mode: graph-capturable steps ----
 * qf_plan_bind allocates, once, everything a forward + adjoint step needs for
 * states of up to `batch` registers: per-register gate matrices, reduction
 * scratch, gradient work buffers and checkpoints.  Afterwards
 * qf_plan_forward_dev and qf_adjoint_grad_dev build every matrix on the device
 * from a DEVICE array of angles and neither allocate, copy from the host nor
 * synchronise, so a whole training step can be captured in a HIP graph and
 * replayed with new angles written into the same device array.  Needs a stage
 * plan (fuse = 0).  Synchronous; re-binding frees the previous workspaces. */
qf_status qf_plan_bind(qf_plan* plan, int64_t batch);

/* Forward pass with angles theta (DEVICE, FP64): register b uses
 * theta[b * theta_stride .. + nparams]; theta_stride = 0 shares one set. */
qf_status qf_plan_forward_dev(qf_plan* plan, const qf_state* s, const double* theta,
                              int64_t theta_stride, void* stream);

/* Adjoint gradient as qf_adjoint_grad (same flags), all on the device: grad
 * (DEVICE, batch*nparams doubles), and, if loss is not NULL (flags = 0 only),
 * <O> per register (DEVICE, batch complex values, 2 doubles each) taken before
 * the reverse walk.  Per-parameter sums run in a fixed order (bitwise
 * reproducible). */
qf_status qf_adjoint_grad_dev(qf_plan* plan, const qf_state* psi, const qf_state* lam,
                              const double* theta, int64_t theta_stride, int32_t nterms,
                              const int32_t* term_qudit, const double* term_diag,
                              double* grad, double* loss, uint32_t flags, void* stream);

/* Autotuner flags. */
#define QF_TUNE_ADJOINT 1u  /* time a forward pass plus an adjoint gradient (of <Z_0>) */
#define QF_TUNE_BOUND   2u  /* only schedules the device-parameter mode accepts (stage  */
                            /* plans), each timed bound to the state's batch with one    */
                            /* angle vector shared by every register                     */

/* Autotuner: times candidate schedules of this plan's circuit on the caller's
 * state s (stage tiles of the default size +-1 qudit with every register-group
 * size: group 1 applies each qudit's run of one-qudit gates as a D x D matrix,
 * group 2 the runs of two qudits as one D^2 x D^2 block; the one-sweep-per-op
 * and pipelined stage kernels; without QF_TUNE_BOUND also two-qudit dense
 * blocks (fuse 3) and per-qudit-run sweeps (fuse 2)), each as two steps timed
 * with HIP events on `stream` after one warm-up step; with QF_TUNE_ADJOINT a
 * second round then varies the adjoint tile of the best stage plan (from one
 * qudit below its default up to the whole register).  It then rebuilds the plan
 * with the fastest options (written to *chosen if not NULL; the rebuilt plan
 * is not bound).  A step is a forward pass, plus the adjoint gradient with
 * QF_TUNE_ADJOINT (a scratch adjoint state of the state's size is allocated
 * for the call).  The winner is cached per (device architecture, D, n, dtype,
 * batch, gate structure, flags) for the life of the process; with
 * QF_TUNE_CACHE=<file> it is also appended to that file, and the file's
 * entries are read on the first call, so later processes skip the timing.
 * s is overwritten.  Synchronises `stream`.  Mixed-dimension plans:
 * QF_EUNSUPPORTED. */
qf_status qf_plan_autotune(qf_plan* plan, const qf_state* s, const double* theta, uint32_t flags,
                           qf_plan_opts* chosen, void* stream);

void qf_plan_destroy(qf_plan* plan);

/* ------------------------------------------------------------------------- */
/* Misc                                                                      */
/* ------------------------------------------------------------------------- */

/* Thread-local message for the calling thread's last non-OK status. */
const char* qf_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t qf_version(void);

/* Releases library-wide state: the autotuner's in-memory cache of chosen
 * options (a QF_TUNE_CACHE file is kept and read again on demand) and the
 * freed temporaries the devices' default stream-ordered pools keep for reuse
 * (up to 4 GiB per device).  Plans
 * stay valid (each owns its buffers until qf_plan_destroy).  Safe to call more
 * than once; the library re-creates the state on demand. */
void qf_shutdown(void);

/* Environment variables read by the library:
 *   QF_LOG=1               planner and autotuner choices on stderr;
 *   QF_CHECK_NORM=<tol>    after every qf_plan_forward, synchronise and fail
 *                          with QF_ERANGE if | |psi| - 1 | > tol for a register;
 *   QF_TEST_FAIL_ALLOC=1   every allocation fails with QF_ENOMEM (tests);
 *   QF_TUNE_CACHE=<file>   the autotuner's persistent cache of chosen options. */

#ifdef __cplusplus
}
#endif

#endif /* QF_H */
