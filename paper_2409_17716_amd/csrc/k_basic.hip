// Per-gate sweep kernels for gfx950: state init, one-qudit D x D mat-vec along
// an axis, controlled-shift permutations, diagonal phases, probabilities and
// diagonal expectation values.
//
// A register of n qudits is viewed, for a gate on qudit q, as [H][D][L] with
// D = d_q, L = S_q (the product of the dimensions after q) and H the rest
// (the decimal index puts qudit 0 first; qudits may differ in dimension).
// A "fibre" is the D amplitudes psi[h, :, l].
//  * L >= 64: one fibre per lane, lanes take consecutive l, so each of the D
//    loads of a wavefront is one contiguous 64-element run (coalesced).
//  * L <  64: a workgroup stages whole [D][L] rows (contiguous in HBM) through
//    LDS with coalesced loads/stores and each lane processes one fibre from LDS.
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "qf_internal.h"

namespace qf {
namespace {

constexpr int kBlock = 256;

template <typename T, int D>
struct MatArg {
    cplx<T> m[D * D];
};

// ---------------------------------------------------------------------------
// Fibre operations.
// ---------------------------------------------------------------------------

template <typename T, int D>
struct OpMat {
    MatArg<T, D> U;
    __device__ bool skip(uint32_t) const { return false; }
    __device__ void apply(cplx<T> (&v)[D], uint32_t) const {
        cplx<T> w[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            cplx<T> acc = cmake<T>(0, 0);
#pragma unroll
            for (int b = 0; b < D; ++b) cmac(acc, U.m[a * D + b], v[b]);
            w[a] = acc;
        }
#pragma unroll
        for (int a = 0; a < D; ++a) v[a] = w[a];
    }
};

// x_t -> x_t + shift[x_c] mod D (D = d_t); the control digit is read from
// the global index of the fibre (any element of the fibre has the same x_c).
template <typename T, int D>
struct OpShift {
    int32_t shift[kMaxDim];  // per control level, already reduced to [0, D)
    FastDiv strideC;         // x_c = (index / S_c) mod d_c
    FastDiv divDc;
    uint32_t dc;
    int32_t has_ctrl;
    __device__ int amount(uint32_t gidx) const {
        if (!has_ctrl) return shift[0];
        const uint32_t qv = strideC.div(gidx);
        const uint32_t c = qv - divDc.div(qv) * dc;
        int s = shift[0];
#pragma unroll
        for (int a = 1; a < kMaxDim; ++a) s = (c == uint32_t(a)) ? shift[a] : s;
        return s;
    }
    __device__ bool skip(uint32_t gidx) const { return amount(gidx) == 0; }
    // v[b] <- v[(b - s) mod D] as a barrel of rotations by 1, 2, 4, ...: every
    // register index is a compile-time constant, so nothing is spilled.
    __device__ void apply(cplx<T> (&v)[D], uint32_t gidx) const {
        const int s = amount(gidx);
#pragma unroll
        for (int bit = 1; bit < D; bit <<= 1) {
            const bool on = (s & bit) != 0;
            cplx<T> w[D];
#pragma unroll
            for (int b = 0; b < D; ++b) w[b] = v[(b - bit % D + D) % D];
#pragma unroll
            for (int b = 0; b < D; ++b) {
                v[b].re = on ? w[b].re : v[b].re;
                v[b].im = on ? w[b].im : v[b].im;
            }
        }
    }
};

// Multi-controlled shift x_t -> x_t + sign * prod_i x_{c_i} mod D (the
// Toffoli / multi-controlled NOT generalized like the CNOT index rule); the
// control digits are read from the global index of the fibre.
constexpr int kMaxMcxCtrl = 8;

template <typename T, int D>
struct OpShiftMulti {
    FastDiv strideC[kMaxMcxCtrl];
    FastDiv divDc[kMaxMcxCtrl];  // the controls' dimensions
    int32_t nctrl;
    int32_t inverse;
    __device__ int amount(uint32_t gidx) const {
        uint32_t prod = 1;
        for (int i = 0; i < nctrl; ++i) {
            const uint32_t qv = strideC[i].div(gidx);
            prod = (prod * (qv - divDc[i].div(qv) * divDc[i].d)) % D;
        }
        return inverse ? int((D - prod) % D) : int(prod);
    }
    __device__ bool skip(uint32_t gidx) const { return amount(gidx) == 0; }
    __device__ void apply(cplx<T> (&v)[D], uint32_t gidx) const {
        const int s = amount(gidx);
#pragma unroll
        for (int bit = 1; bit < D; bit <<= 1) {
            const bool on = (s & bit) != 0;
            cplx<T> w[D];
#pragma unroll
            for (int b = 0; b < D; ++b) w[b] = v[(b - bit % D + D) % D];
#pragma unroll
            for (int b = 0; b < D; ++b) {
                v[b].re = on ? w[b].re : v[b].re;
                v[b].im = on ? w[b].im : v[b].im;
            }
        }
    }
};

template <typename T, int D, class Op>
__global__ __launch_bounds__(kBlock) void k_axis_wide(cplx<T>* __restrict__ psi, uint32_t nfib,
                                                      uint32_t L, FastDiv divL, Op op) {
    const uint32_t f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= nfib) return;
    const uint32_t h = divL.div(f);
    const uint32_t l = f - h * L;
    const uint32_t base = h * (uint32_t(D) * L) + l;
    if (op.skip(base)) return;
    cplx<T> v[D];
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = psi[base + uint32_t(d) * L];
    op.apply(v, base);
#pragma unroll
    for (int d = 0; d < D; ++d) psi[base + uint32_t(d) * L] = v[d];
}

template <typename T, int D, class Op>
__global__ __launch_bounds__(kBlock) void k_axis_narrow(cplx<T>* __restrict__ psi, uint32_t total,
                                                        uint32_t L, uint32_t rows, Op op) {
    __shared__ cplx<T> tile[kBlock * D];
    const uint32_t E = rows * uint32_t(D) * L;  // <= kBlock * D
    const uint32_t start = blockIdx.x * E;
    const uint32_t cnt = min(E, total - start);
    const uint32_t nf = cnt / D;
    const uint32_t r = threadIdx.x / L;
    const uint32_t l = threadIdx.x - r * L;
    const uint32_t off = r * uint32_t(D) * L + l;
    // a block none of whose fibres changes (a permutation whose controls
    // select shift 0 here) is neither read nor written
    const bool act = threadIdx.x < nf && !op.skip(start + off);
    if (!__syncthreads_or(act)) return;
    for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) tile[i] = psi[start + i];
    __syncthreads();
    if (threadIdx.x < nf) {
        if (act) {
            cplx<T> v[D];
#pragma unroll
            for (int d = 0; d < D; ++d) v[d] = tile[off + uint32_t(d) * L];
            op.apply(v, start + off);
#pragma unroll
            for (int d = 0; d < D; ++d) tile[off + uint32_t(d) * L] = v[d];
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) psi[start + i] = tile[i];
}

template <typename T, int D, class Op>
qf_status run_axis(const StateView& s, int q, const Op& op, hipStream_t st, const char* what) {
    auto* psi = reinterpret_cast<cplx<T>*>(s.amps);
    const uint32_t L = s.strides[q];
    if (L >= 64) {
        const uint32_t nfib = s.total / D;
        const uint32_t grid = (nfib + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((k_axis_wide<T, D, Op>), dim3(grid), dim3(kBlock), 0, st, psi, nfib, L,
                           FastDiv(L), op);
    } else {
        const uint32_t rows = (kBlock / L) > 0 ? kBlock / L : 1;
        const uint32_t E = rows * D * L;
        const uint32_t grid = (s.total + E - 1) / E;
        hipLaunchKernelGGL((k_axis_narrow<T, D, Op>), dim3(grid), dim3(kBlock), 0, st, psi, s.total,
                           L, rows, op);
    }
    return check_launch(what);
}

// ---------------------------------------------------------------------------
// Compile-time dispatch on dtype and D.
// ---------------------------------------------------------------------------

template <class F>
qf_status with_dim(uint32_t D, F&& f) {
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

template <class F>
qf_status with_type(int dtype, F&& f) {
    if (dtype == QF_C64) return f(float{});
    if (dtype == QF_C128) return f(double{});
    return set_error(QF_EDTYPE, "unknown dtype %d", dtype);
}

// ---------------------------------------------------------------------------
// SWAP of two qudits a, b of one dimension D (strides S_a > S_b): lane r owns
// the D x D block {x0 + i S_a + j S_b} of one setting of the other digits and
// exchanges entries (i, j) and (j, i) for i < j (the diagonal stays).  The
// other digits split as x0 = hi (D S_a) + mid (D S_b) + lo, lo < S_b, and
// consecutive lanes take consecutive lo, so for S_b >= 64 every load and
// store of a wavefront is one contiguous run; both members of a pair are read
// and written by the same lane.
// ---------------------------------------------------------------------------

// Pair e of the strictly upper triangle of a D x D block, row by row.
template <int D>
__host__ __device__ constexpr int pair_row(int e) {
    int i = 0;
    while (e >= D - 1 - i) {
        e -= D - 1 - i;
        ++i;
    }
    return i;
}
template <int D>
__host__ __device__ constexpr int pair_col(int e) {
    int i = 0;
    while (e >= D - 1 - i) {
        e -= D - 1 - i;
        ++i;
    }
    return i + 1 + e;
}

// Exchanges pairs E, E + 1, ... of a block: each pair's two loads are issued
// before the later pairs' (recursion), its stores after them, so every load
// of the block is in flight at once with no private array.
template <typename T, int D, int E>
__device__ __forceinline__ void swap_pairs(cplx<T>* __restrict__ psi, uint32_t x0, uint32_t Sa, uint32_t Sb) {
    if constexpr (E < D * (D - 1) / 2) {
        constexpr uint32_t ia = uint32_t(pair_row<D>(E)), ib = uint32_t(pair_col<D>(E));
        const cplx<T> v = psi[x0 + ia * Sa + ib * Sb];
        const cplx<T> w = psi[x0 + ib * Sa + ia * Sb];
        swap_pairs<T, D, E + 1>(psi, x0, Sa, Sb);
        psi[x0 + ia * Sa + ib * Sb] = w;
        psi[x0 + ib * Sa + ia * Sb] = v;
    }
}

// The same for two blocks at once (the second only where has1): both blocks'
// loads are in flight before the first store.
template <typename T, int D, int E>
__device__ __forceinline__ void swap_pairs2(cplx<T>* __restrict__ psi, uint32_t x0, uint32_t x1, bool has1,
                                            uint32_t Sa, uint32_t Sb) {
    if constexpr (E < D * (D - 1) / 2) {
        constexpr uint32_t ia = uint32_t(pair_row<D>(E)), ib = uint32_t(pair_col<D>(E));
        const uint32_t oab = ia * Sa + ib * Sb, oba = ib * Sa + ia * Sb;
        const cplx<T> v0 = psi[x0 + oab];
        const cplx<T> w0 = psi[x0 + oba];
        cplx<T> v1 = cmake<T>(0, 0), w1 = cmake<T>(0, 0);
        if (has1) {
            v1 = psi[x1 + oab];
            w1 = psi[x1 + oba];
        }
        swap_pairs2<T, D, E + 1>(psi, x0, x1, has1, Sa, Sb);
        psi[x0 + oab] = w0;
        psi[x0 + oba] = v0;
        if (has1) {
            psi[x1 + oab] = w1;
            psi[x1 + oba] = v1;
        }
    }
}

// Blocks a lane exchanges per loop trip in k_swap: two for small blocks whose
// lower qudit has a stride of at least a wavefront (every load of a wavefront
// then reads one run, and it keeps twice the loads in flight); one otherwise
// (measured with the stride-1 qudit: two blocks per lane, each access spread
// over 24-byte steps, were 10% slower).
template <typename T, int D>
constexpr bool swap_two_blocks_ok() {
    return sizeof(T) == 4 && D <= 4;
}

template <typename T, int D>
__device__ __forceinline__ uint32_t swap_block_base(uint32_t r, const FastDiv& divSb, const FastDiv& divM, uint32_t Sa,
                                                    uint32_t Sb) {
    const uint32_t t = divSb.div(r);
    const uint32_t lo = r - t * Sb;
    const uint32_t hi = divM.div(t);
    const uint32_t mid = t - hi * divM.d;
    return hi * (uint32_t(D) * Sa) + mid * (uint32_t(D) * Sb) + lo;
}

template <typename T, int D, int BPL>
__global__ __launch_bounds__(kBlock) void k_swap(cplx<T>* __restrict__ psi, uint32_t nblk, FastDiv divSb, FastDiv divM,
                                                 uint32_t Sa, uint32_t Sb) {
    if constexpr (BPL == 2) {
        for (uint32_t r = blockIdx.x * (2 * kBlock) + threadIdx.x; r < nblk; r += gridDim.x * (2 * kBlock)) {
            const uint32_t r1 = r + kBlock;
            const bool has1 = r1 < nblk;
            const uint32_t x0 = swap_block_base<T, D>(r, divSb, divM, Sa, Sb);
            const uint32_t x1 = has1 ? swap_block_base<T, D>(r1, divSb, divM, Sa, Sb) : 0u;
            swap_pairs2<T, D, 0>(psi, x0, x1, has1, Sa, Sb);
        }
        return;
    }
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < nblk; r += gridDim.x * kBlock) {
        const uint32_t x0 = swap_block_base<T, D>(r, divSb, divM, Sa, Sb);
        // all pairs' loads in flight where that stays in registers (measured:
        // complex128 blocks beyond D = 3 go to scratch)
        if constexpr ((sizeof(T) == 4 && D <= 6) || D <= 3) {
            swap_pairs<T, D, 0>(psi, x0, Sa, Sb);
        } else {
            // larger D: one pair at a time
            for (uint32_t ia = 0; ia + 1 < uint32_t(D); ++ia)
                for (uint32_t ib = ia + 1; ib < uint32_t(D); ++ib) {
                    const cplx<T> v = psi[x0 + ia * Sa + ib * Sb];
                    const cplx<T> w = psi[x0 + ib * Sa + ia * Sb];
                    psi[x0 + ia * Sa + ib * Sb] = w;
                    psi[x0 + ib * Sa + ia * Sb] = v;
                }
        }
    }
}

// ---------------------------------------------------------------------------
// Init.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(cplx<T>* __restrict__ psi, uint32_t total, uint32_t N,
                                                 FastDiv divN, const uint32_t* __restrict__ idx,
                                                 uint32_t idx0) {
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < total; x += gridDim.x * kBlock) {
        const uint32_t b = divN.div(x);
        const uint32_t local = x - b * N;
        const uint32_t target = idx ? idx[b] : idx0;
        psi[x] = cmake<T>(local == target ? T(1) : T(0), T(0));
    }
}

uint32_t grid_for(uint32_t total, uint32_t per_block, uint32_t cap = 1u << 20) {
    uint32_t g = (total + per_block - 1) / per_block;
    return g < 1 ? 1 : (g > cap ? cap : g);
}

// ---------------------------------------------------------------------------
// Diagonal phases.
// ---------------------------------------------------------------------------

constexpr int kDiagBytes = 2048;

template <typename T>
struct DiagArg {
    static constexpr int kMax = kDiagBytes / int(sizeof(cplx<T>));
    FastDiv stride[8];
    FastDiv divd[8];  // dimensions of the listed qudits
    uint32_t k;
    uint32_t ntab;
    cplx<T> table[kMax];
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag(cplx<T>* __restrict__ psi, uint32_t total,
                                                 DiagArg<T> a) {
    __shared__ cplx<T> tab[DiagArg<T>::kMax];
    for (uint32_t i = threadIdx.x; i < a.ntab; i += kBlock) tab[i] = a.table[i];
    __syncthreads();
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < total; x += gridDim.x * kBlock) {
        uint32_t y = 0;
        for (uint32_t i = 0; i < a.k; ++i) {
            const uint32_t qv = a.stride[i].div(x);
            const uint32_t d = a.divd[i].d;
            y = y * d + (qv - a.divd[i].div(qv) * d);
        }
        psi[x] = cmul(psi[x], tab[y]);
    }
}

// ---------------------------------------------------------------------------
// Probabilities.
// ---------------------------------------------------------------------------

// O = T (the state's precision) or double (squares taken in FP64).
template <typename T, typename O>
__global__ __launch_bounds__(kBlock) void k_probs_full(const cplx<T>* __restrict__ psi, O* __restrict__ out,
                                                       uint32_t total) {
    // four grid strides per trip, loads first, 64-bit indices (a 32-bit index
    // plus the grid stride could wrap for totals near 2^32); measured at the
    // same speed as one element per trip on 3^16 (91-92 us)
    const uint64_t st = uint64_t(gridDim.x) * kBlock;
    uint64_t x = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    for (; x + 3 * st < total; x += 4 * st) {
        cplx<T> v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = psi[x + uint64_t(i) * st];
#pragma unroll
        for (int i = 0; i < 4; ++i) out[x + uint64_t(i) * st] = O(v[i].re) * O(v[i].re) + O(v[i].im) * O(v[i].im);
    }
    for (; x < total; x += st) {
        const cplx<T> v = psi[x];
        out[x] = O(v.re) * O(v.re) + O(v.im) * O(v.im);
    }
}

// Deterministic workgroup sum of one double per lane (fixed order; a
// workgroup of kBlock lanes): an xor butterfly inside each wavefront (partners
// add the same two values, so every lane ends with the same total), then the
// wavefront totals in wavefront order through LDS (sh holds kBlock / 64).
__device__ inline double block_sum(double v, double* sh) {
    constexpr int kWaves = kBlock / 64;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63u) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) r += sh[w];
    __syncthreads();
    return r;
}

constexpr int kMaxMarg = 32;

struct MargArg {
    uint32_t N;           // amplitudes per register
    uint32_t Z;           // elements per bin = N / bins
    uint32_t R;           // trailing contiguous run (digits below every measured qudit)
    FastDiv divR;
    uint32_t m;           // measured qudits
    uint32_t u;           // other (non-trailing, unmeasured) qudits
    uint32_t bins;        // product of the measured qudits' dimensions
    uint32_t chunk;       // elements of one bin summed by one workgroup
    uint32_t chunks;      // workgroups per bin
    uint32_t mstride[kMaxMarg];  // strides of measured qudits, listed order
    FastDiv mdiv[kMaxMarg];      // their dimensions
    uint32_t ostride[kMaxMarg];  // strides of the other qudits, most significant first
    FastDiv odiv[kMaxMarg];      // their dimensions
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_marg_partial(const cplx<T>* __restrict__ psi, MargArg a,
                                                         double* __restrict__ partial) {
    __shared__ double sh[kBlock];
    const uint32_t c = blockIdx.x % a.chunks;
    const uint32_t yb = blockIdx.x / a.chunks;
    const uint32_t b = yb / a.bins;
    const uint32_t y = yb - b * a.bins;
    // base offset of bin y in register b
    uint32_t base = b * a.N;
    {
        uint32_t yy = y;
        for (int i = int(a.m) - 1; i >= 0; --i) {
            const uint32_t q = a.mdiv[i].div(yy);
            base += (yy - q * a.mdiv[i].d) * a.mstride[i];
            yy = q;
        }
    }
    const uint32_t z0 = c * a.chunk;
    const uint32_t z1 = min(a.Z, z0 + a.chunk);
    double acc = 0.0;
    for (uint32_t z = z0 + threadIdx.x; z < z1; z += kBlock) {
        uint32_t zh = a.divR.div(z);
        const uint32_t zl = z - zh * a.R;
        uint32_t off = 0;
        for (int j = int(a.u) - 1; j >= 0; --j) {
            const uint32_t q = a.odiv[j].div(zh);
            off += (zh - q * a.odiv[j].d) * a.ostride[j];
            zh = q;
        }
        const cplx<T> v = psi[base + off + zl];
        acc += double(v.re) * double(v.re) + double(v.im) * double(v.im);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// One workgroup per bin: lanes sum chunks c = lane, lane + 256, ..., then a fixed tree.
template <typename O>
__global__ __launch_bounds__(kBlock) void k_marg_final(const double* __restrict__ partial, uint32_t chunks,
                                                       O* __restrict__ out) {
    __shared__ double sh[kBlock];
    const uint32_t i = blockIdx.x;
    double s = 0.0;
    for (uint32_t c = threadIdx.x; c < chunks; c += kBlock) s += partial[size_t(i) * chunks + c];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[i] = O(s);
}

// Marginals streamed in memory order.  A workgroup reads one chunk of
// per_wg elements, per_wg the stride of some qudit, so the digits of every
// qudit of at least that stride are constant over the chunk: the measured
// ones among them ("high") give the chunk one bin offset y_hi.  The other
// measured qudits ("low", at most 16 digit combinations c) vary inside it;
// each lane adds |psi_x|^2 in FP64 to its register copy of combination c(x)
// (a predicated add into every combination, so they stay in registers).  Each
// combination is summed over the wavefront by a fixed xor-butterfly and over
// the wavefronts in a fixed order; the workgroup writes one partial per bin
// (y_hi + y_lo(c), zero for the bins it does not reach): bitwise reproducible.
struct MargSmall {
    uint32_t N;
    uint32_t m;
    uint32_t bins;                 // all outcomes (<= 256)
    uint32_t per_wg;
    uint32_t wpr;                  // workgroups per register
    uint32_t nlow;                 // low measured qudits
    uint32_t ncomb;                // their digit combinations (<= 16)
    FastDiv stride[kMaxMarg];      // measured qudits, listed order
    FastDiv dim[kMaxMarg];
    uint32_t radix[kMaxMarg];      // bin weight of each measured qudit
    uint32_t low[kMaxMarg];        // indices (into the measured list) of the low qudits, listed order
    uint32_t ylo[16];              // bin offset of each combination
};

template <typename T, int NB>
__global__ __launch_bounds__(kBlock) void k_marg_stream(const cplx<T>* __restrict__ psi, MargSmall a,
                                                        double* __restrict__ partial) {
    __shared__ double sh[kBlock / 64][NB];
    const uint32_t b = blockIdx.x / a.wpr, w = blockIdx.x - b * a.wpr;
    const cplx<T>* reg = psi + size_t(b) * a.N;
    const uint32_t x0 = w * a.per_wg;
    const uint32_t x1 = min(a.N, x0 + a.per_wg);
    uint32_t yhi = 0;  // the high qudits' part of the bin, from the chunk's first index
    for (uint32_t i = 0; i < a.m; ++i) {
        const uint32_t qv = a.stride[i].div(x0);
        yhi += (qv - a.dim[i].div(qv) * a.dim[i].d) * a.radix[i];
    }
    for (uint32_t j = 0; j < a.nlow; ++j) {
        const uint32_t i = a.low[j];
        const uint32_t qv = a.stride[i].div(x0);
        yhi -= (qv - a.dim[i].div(qv) * a.dim[i].d) * a.radix[i];
    }
    double acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = 0.0;
#pragma unroll 8
    for (uint32_t x = x0 + threadIdx.x; x < x1; x += kBlock) {
        const cplx<T> v = reg[x];
        const double p = double(v.re) * double(v.re) + double(v.im) * double(v.im);
        uint32_t c = 0;
        for (uint32_t j = 0; j < a.nlow; ++j) {
            const uint32_t i = a.low[j];
            const uint32_t qv = a.stride[i].div(x);
            const uint32_t d = a.dim[i].d;
            c = c * d + (qv - a.dim[i].div(qv) * d);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j] += (c == uint32_t(j)) ? p : 0.0;
    }
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double v = acc[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) sh[wave][j] = v;
    }
    __syncthreads();
    for (uint32_t y = threadIdx.x; y < a.bins; y += kBlock) {
        double t = 0.0;
        for (uint32_t c = 0; c < a.ncomb; ++c)
            if (yhi + a.ylo[c] == y)
                for (uint32_t wv = 0; wv < blockDim.x / 64; ++wv) t += sh[wv][c];
        partial[size_t(blockIdx.x) * a.bins + y] = t;
    }
}

// out[b * bins + y] = sum over the register's workgroups of partial (fixed order).
template <typename O>
__global__ __launch_bounds__(kBlock) void k_marg_stream_final(const double* __restrict__ partial, uint32_t wpr,
                                                              uint32_t bins, O* __restrict__ out) {
    __shared__ double sh[kBlock];
    const uint32_t b = blockIdx.x / bins, y = blockIdx.x - b * bins;
    // kAcc accumulators per lane (independent loads in flight), met in a fixed tree
    constexpr int kAcc = 8;
    const double* p = partial + size_t(b) * wpr * bins + y;
    double acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
    uint32_t w = threadIdx.x;
    for (; uint64_t(w) + uint64_t(kAcc - 1) * kBlock < wpr; w += kAcc * kBlock) {
        double v[kAcc];
#pragma unroll
        for (int j = 0; j < kAcc; ++j) v[j] = p[size_t(w + uint32_t(j) * kBlock) * bins];
#pragma unroll
        for (int j = 0; j < kAcc; ++j) acc[j] += v[j];
    }
#pragma unroll
    for (int j = 0; j < kAcc - 1; ++j) {
        const uint64_t wj = uint64_t(w) + uint64_t(j) * kBlock;
        if (wj < wpr) acc[j] += p[size_t(wj) * bins];
    }
#pragma unroll
    for (int h = kAcc / 2; h > 0; h >>= 1)
#pragma unroll
        for (int j = 0; j < h; ++j) acc[j] += acc[j + h];
    double s = block_sum(acc[0], sh);
    if (threadIdx.x == 0) out[blockIdx.x] = O(s);
}

// ---------------------------------------------------------------------------
// Diagonal expectation values and the Hermitian part of a diagonal observable.
// ---------------------------------------------------------------------------

constexpr int kMaxActive = 32;
constexpr int kMaxTable = 128;
// Row table of the expectation kernel (doubles, complex): chunk / lane span entries.
constexpr int kMaxExpectRows = 512;

struct ObsArg {
    uint32_t nact;
    uint32_t ntab;                 // table entries (sum of the active qudits' dimensions)
    FastDiv stride[kMaxActive];
    FastDiv divd[kMaxActive];      // dimensions of the active qudits
    uint32_t off[kMaxActive];      // first table entry of each active qudit
    uint32_t nlow;                 // expectation chunks: terms whose digit varies inside a chunk
    uint32_t low[kMaxActive];      // their indices (the others are constant over a chunk)
    uint32_t span;                 // expectation lanes: a qudit stride L <= kBlock (digits below it per lane)
    uint32_t nrow;                 // chunk / L rows, whose other low digits are tabled per workgroup
    uint32_t rows_table;           // 1: the row table is used (nrow <= kMaxExpectRows)
    double table[2 * kMaxTable];   // complex, interleaved, active qudits back to back
};

__device__ inline void obs_value(const ObsArg& a, const double* tab, uint32_t x, double& fr, double& fi) {
    fr = 0.0;
    fi = 0.0;
    for (uint32_t t = 0; t < a.nact; ++t) {
        const uint32_t qv = a.stride[t].div(x);
        const uint32_t d = qv - a.divd[t].div(qv) * a.divd[t].d;
        fr += tab[2 * (a.off[t] + d)];
        fi += tab[2 * (a.off[t] + d) + 1];
    }
}

// A workgroup sums one chunk of a register, chunk = a qudit stride, so the
// terms on qudits of at least that stride are constant over the chunk (taken
// once from its first index); per element only the other ("low") terms are
// looked up.
// Expectation partial sums, one workgroup per chunk (a qudit stride).  The
// digits of qudits at or above the chunk size are constant over the chunk
// (taken once); the others vary.  Lanes walk the chunk in steps of
// T = L floor(kBlock / L), L a qudit stride: lane tid = r L + l visits
// x = x0 + tid + T j, whose digits below L are those of l (summed once per
// lane) and whose digits between L and the chunk size are those of row
// m = r + (T / L) j (summed once per workgroup into an LDS table).  Where that
// table would be too large, or no term varies inside the chunk, every element
// takes its varying digits itself.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_expect_partial(const cplx<T>* __restrict__ psi, uint32_t N,
                                                           uint32_t chunk, uint32_t nblk, ObsArg a,
                                                           double* __restrict__ partial) {
    __shared__ double tab[2 * kMaxTable];
    __shared__ double sh[kBlock];
    __shared__ double rowf[2 * kMaxExpectRows];
    for (uint32_t i = threadIdx.x; i < 2 * a.ntab; i += kBlock) tab[i] = a.table[i];
    __syncthreads();
    const uint32_t b = blockIdx.x / nblk;
    const uint32_t blk = blockIdx.x - b * nblk;
    const uint32_t x0 = blk * chunk;
    const uint32_t x1 = min(N, x0 + chunk);
    const cplx<T>* reg = psi + size_t(b) * N;
    // the chunk-constant part of f (all terms at x0 minus the low ones, which are
    // at digit 0 there since the chunk starts at a multiple of their period)
    double hr, hi;
    obs_value(a, tab, x0, hr, hi);
    for (uint32_t j = 0; j < a.nlow; ++j) {
        const uint32_t t = a.low[j];
        hr -= tab[2 * a.off[t]];
        hi -= tab[2 * a.off[t] + 1];
    }
    double ar = 0.0, ai = 0.0;
    if (a.rows_table) {
        const uint32_t L = a.span, R = kBlock / L, TL = R * L;
        const uint32_t r = threadIdx.x / L, l = threadIdx.x - r * L;
        // rows: the low terms at or above L, at x = m L
        for (uint32_t m = threadIdx.x; m < a.nrow; m += kBlock) {
            double fr = 0.0, fi = 0.0;
            for (uint32_t j = 0; j < a.nlow; ++j) {
                const uint32_t t = a.low[j];
                if (a.stride[t].d < L) continue;
                const uint32_t qv = a.stride[t].div(m * L);
                const uint32_t d = qv - a.divd[t].div(qv) * a.divd[t].d;
                fr += tab[2 * (a.off[t] + d)];
                fi += tab[2 * (a.off[t] + d) + 1];
            }
            rowf[2 * m] = fr;
            rowf[2 * m + 1] = fi;
        }
        // this lane: the low terms below L, at x = l
        double cr = hr, ci = hi;
        for (uint32_t j = 0; j < a.nlow; ++j) {
            const uint32_t t = a.low[j];
            if (a.stride[t].d >= L) continue;
            const uint32_t qv = a.stride[t].div(l);
            const uint32_t d = qv - a.divd[t].div(qv) * a.divd[t].d;
            cr += tab[2 * (a.off[t] + d)];
            ci += tab[2 * (a.off[t] + d) + 1];
        }
        __syncthreads();
        if (threadIdx.x < TL) {
            uint32_t m = r;
#pragma unroll 4
            for (uint32_t x = x0 + threadIdx.x; x < x1; x += TL, m += R) {
                const cplx<T> v = reg[x];
                const double p = double(v.re) * double(v.re) + double(v.im) * double(v.im);
                ar += p * (cr + rowf[2 * m]);
                ai += p * (ci + rowf[2 * m + 1]);
            }
        }
    } else {
#pragma unroll 4
        for (uint32_t x = x0 + threadIdx.x; x < x1; x += kBlock) {
            const cplx<T> v = reg[x];
            const double p = double(v.re) * double(v.re) + double(v.im) * double(v.im);
            double fr = hr, fi = hi;
            for (uint32_t j = 0; j < a.nlow; ++j) {
                const uint32_t t = a.low[j];
                const uint32_t qv = a.stride[t].div(x);
                const uint32_t d = qv - a.divd[t].div(qv) * a.divd[t].d;
                fr += tab[2 * (a.off[t] + d)];
                fi += tab[2 * (a.off[t] + d) + 1];
            }
            ar += p * fr;
            ai += p * fi;
        }
    }
    const double sr = block_sum(ar, sh);
    const double si = block_sum(ai, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sr;
        partial[2 * blockIdx.x + 1] = si;
    }
}

// One workgroup per register; a fixed summation order, so the result is bitwise reproducible.
__global__ __launch_bounds__(kBlock) void k_expect_final(const double* __restrict__ partial, uint32_t nblk,
                                                         double* __restrict__ out) {
    // Lane t takes the partials t, t + kBlock, ... into kAcc accumulators (the
    // j-th of each group of kAcc strides into the j-th), so kAcc independent
    // 16-byte loads are in flight per trip instead of one dependent chain; the
    // accumulators meet in a fixed pairwise tree, then the workgroup tree.
    constexpr int kAcc = 8;
    __shared__ double sh[kBlock];
    const uint32_t b = blockIdx.x;
    const double2* p = reinterpret_cast<const double2*>(partial) + size_t(b) * nblk;
    double ar[kAcc], ai[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) ar[j] = ai[j] = 0.0;
    uint32_t c = threadIdx.x;
    for (; uint64_t(c) + uint64_t(kAcc - 1) * kBlock < nblk; c += kAcc * kBlock) {
        double2 v[kAcc];
#pragma unroll
        for (int j = 0; j < kAcc; ++j) v[j] = p[c + uint32_t(j) * kBlock];
#pragma unroll
        for (int j = 0; j < kAcc; ++j) {
            ar[j] += v[j].x;
            ai[j] += v[j].y;
        }
    }
    // fewer than kAcc strides remain
#pragma unroll
    for (int j = 0; j < kAcc - 1; ++j) {
        const uint64_t cj = uint64_t(c) + uint64_t(j) * kBlock;
        if (cj < nblk) {
            const double2 v = p[cj];
            ar[j] += v.x;
            ai[j] += v.y;
        }
    }
#pragma unroll
    for (int w = kAcc / 2; w > 0; w >>= 1)
#pragma unroll
        for (int j = 0; j < w; ++j) {
            ar[j] += ar[j + w];
            ai[j] += ai[j + w];
        }
    double sr = ar[0], si = ai[0];
    sr = block_sum(sr, sh);
    si = block_sum(si, sh);
    if (threadIdx.x == 0) {
        out[2 * b] = sr;
        out[2 * b + 1] = si;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag_observable(const cplx<T>* __restrict__ psi,
                                                            cplx<T>* __restrict__ lam, uint32_t total,
                                                            FastDiv divN, uint32_t N, ObsArg a) {
    __shared__ double tab[2 * kMaxTable];
    for (uint32_t i = threadIdx.x; i < 2 * a.ntab; i += kBlock) tab[i] = a.table[i];
    __syncthreads();
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < total; x += gridDim.x * kBlock) {
        const uint32_t local = x - divN.div(x) * N;
        double fr, fi;
        obs_value(a, tab, local, fr, fi);
        const cplx<T> v = psi[x];
        lam[x] = cmake<T>(T(fr) * v.re, T(fr) * v.im);
    }
}

ObsArg make_obs(const StateView& s, const std::vector<int>& active, const std::vector<double>& table,
                bool real_only) {
    ObsArg a{};
    a.nact = uint32_t(active.size());
    uint32_t off = 0;
    for (size_t t = 0; t < active.size(); ++t) {
        a.stride[t].init(s.strides[active[t]]);
        a.divd[t].init(s.dims[active[t]]);
        a.off[t] = off;
        off += s.dims[active[t]];
    }
    a.ntab = off;
    for (uint32_t i = 0; i < off; ++i) {
        a.table[2 * i] = real_only ? table[i] : table[2 * i];
        a.table[2 * i + 1] = real_only ? 0.0 : table[2 * i + 1];
    }
    return a;
}

}  // namespace

// ===========================================================================
// Launchers.
// ===========================================================================

qf_status launch_init(const StateView& s, const std::vector<uint32_t>& index, hipStream_t st) {
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        uint32_t* didx = nullptr;
        uint32_t idx0 = index.empty() ? 0u : index[0];
        if (index.size() > 1) {
            QF_CHECK(dev_malloc_async(reinterpret_cast<void**>(&didx), index.size() * sizeof(uint32_t), st,
                                      "init digits"));
            QF_HIP_CHECK(hipMemcpyAsync(didx, index.data(), index.size() * sizeof(uint32_t),
                                        hipMemcpyHostToDevice, st));
        }
        hipLaunchKernelGGL(k_init<T>, dim3(grid_for(s.total, kBlock * 4)), dim3(kBlock), 0, st,
                           reinterpret_cast<cplx<T>*>(s.amps), s.total, s.N, FastDiv(s.N), didx, idx0);
        qf_status r = check_launch("k_init");
        if (didx) QF_HIP_CHECK(hipFreeAsync(didx, st));
        return r;
    });
}

qf_status launch_apply_1q(const StateView& s, int q, const double* U, hipStream_t st) {
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        return with_dim(s.dims[q], [&](auto dtag) -> qf_status {
            constexpr int D = decltype(dtag)::value;
            if constexpr (sizeof(MatArg<T, D>) > 2048) {
                return set_error(QF_ERANGE, "dim %d too large for a complex128 kernel-argument matrix", D);
            } else {
                OpMat<T, D> op;
                for (int i = 0; i < D * D; ++i) op.U.m[i] = cmake<T>(T(U[2 * i]), T(U[2 * i + 1]));
                return run_axis<T, D>(s, q, op, st, "qf_apply_1q");
            }
        });
    });
}

qf_status launch_ctrl(const StateView& s, int ctrl, int tgt, const int32_t* shift, hipStream_t st) {
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        return with_dim(s.dims[tgt], [&](auto dtag) -> qf_status {
            constexpr int D = decltype(dtag)::value;
            OpShift<T, D> op;
            const int nsh = ctrl < 0 ? 1 : int(s.dims[ctrl]);
            for (int i = 0; i < kMaxDim; ++i) {
                const int v = i < nsh ? shift[i] : 0;
                op.shift[i] = ((v % D) + D) % D;
            }
            op.has_ctrl = ctrl >= 0;
            op.strideC = FastDiv(ctrl >= 0 ? s.strides[ctrl] : 1u);
            op.dc = ctrl >= 0 ? s.dims[ctrl] : 1u;
            op.divDc = FastDiv(op.dc);
            return run_axis<T, D>(s, tgt, op, st, "qf_apply_ctrl");
        });
    });
}

qf_status launch_mcx(const StateView& s, int nctrl, const int32_t* ctrls, int tgt, bool inverse, hipStream_t st) {
    if (nctrl < 1 || nctrl > kMaxMcxCtrl) return set_error(QF_ERANGE, "%d controls outside 1..%d", nctrl, kMaxMcxCtrl);
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        return with_dim(s.dims[tgt], [&](auto dtag) -> qf_status {
            constexpr int D = decltype(dtag)::value;
            OpShiftMulti<T, D> op;
            op.nctrl = nctrl;
            op.inverse = inverse ? 1 : 0;
            for (int i = 0; i < kMaxMcxCtrl; ++i) {
                op.strideC[i] = FastDiv(i < nctrl ? s.strides[ctrls[i]] : 1u);
                op.divDc[i] = FastDiv(i < nctrl ? s.dims[ctrls[i]] : 1u);
            }
            return run_axis<T, D>(s, tgt, op, st, "multi-controlled shift");
        });
    });
}

qf_status launch_swap(const StateView& s, int a, int b, hipStream_t st) {
    if (a > b) std::swap(a, b);  // a: the more significant qudit
    const uint32_t Sa = s.strides[a], Sb = s.strides[b], Dq = s.dims[a];  // d_a = d_b
    const uint32_t nblk = s.total / (Dq * Dq);
    const uint32_t M = Sa / (Sb * Dq);  // settings of the digits between b and a
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        return with_dim(Dq, [&](auto dtag) -> qf_status {
            constexpr int D = decltype(dtag)::value;
            if constexpr (swap_two_blocks_ok<T, D>()) {
                if (Sb >= 64) {
                    hipLaunchKernelGGL((k_swap<T, D, 2>), dim3(grid_for(nblk, kBlock * 2)), dim3(kBlock), 0, st,
                                       reinterpret_cast<cplx<T>*>(s.amps), nblk, FastDiv(Sb), FastDiv(M), Sa, Sb);
                    return check_launch("swap");
                }
            }
            hipLaunchKernelGGL((k_swap<T, D, 1>), dim3(grid_for(nblk, kBlock)), dim3(kBlock), 0, st,
                               reinterpret_cast<cplx<T>*>(s.amps), nblk, FastDiv(Sb), FastDiv(M), Sa, Sb);
            return check_launch("swap");
        });
    });
}

qf_status launch_diag(const StateView& s, int k, const int32_t* qudits, const double* phases,
                      hipStream_t st) {
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        DiagArg<T> a{};
        a.k = uint32_t(k);
        a.ntab = 1;
        for (int i = 0; i < k; ++i) a.ntab *= s.dims[qudits[i]];
        if (a.ntab > uint32_t(DiagArg<T>::kMax))
            return set_error(QF_ERANGE, "D^k = %u exceeds %d table entries", a.ntab, DiagArg<T>::kMax);
        for (int i = 0; i < k; ++i) {
            a.stride[i].init(s.strides[qudits[i]]);
            a.divd[i].init(s.dims[qudits[i]]);
        }
        for (uint32_t i = 0; i < a.ntab; ++i) a.table[i] = cmake<T>(T(phases[2 * i]), T(phases[2 * i + 1]));
        hipLaunchKernelGGL(k_diag<T>, dim3(grid_for(s.total, kBlock * 4)), dim3(kBlock), 0, st,
                           reinterpret_cast<cplx<T>*>(s.amps), s.total, a);
        return check_launch("qf_apply_diag");
    });
}

qf_status launch_probs_full(const StateView& s, void* out, bool f64, hipStream_t st) {
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        const dim3 g(grid_for(s.total, kBlock * 4));
        const auto* psi = reinterpret_cast<const cplx<T>*>(s.amps);
        if (f64)
            hipLaunchKernelGGL((k_probs_full<T, double>), g, dim3(kBlock), 0, st, psi,
                               reinterpret_cast<double*>(out), s.total);
        else
            hipLaunchKernelGGL((k_probs_full<T, T>), g, dim3(kBlock), 0, st, psi, reinterpret_cast<T*>(out),
                               s.total);
        return check_launch("qf_probs");
    });
}

template <int NB>
qf_status launch_marg_stream(const StateView& s, const MargSmall& a, void* out, bool f64, hipStream_t st) {
    const uint64_t nwg = uint64_t(a.wpr) * s.batch;
    if (nwg >= (1ull << 31)) return set_error(QF_ERANGE, "marginal grid too large");
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        double* partial = nullptr;
        QF_CHECK(dev_malloc_async(reinterpret_cast<void**>(&partial), nwg * a.bins * sizeof(double), st,
                                  "marginal partial sums"));
        hipLaunchKernelGGL((k_marg_stream<T, NB>), dim3(uint32_t(nwg)), dim3(kBlock), 0, st,
                           reinterpret_cast<const cplx<T>*>(s.amps), a, partial);
        qf_status r1 = check_launch("qf_probs marginal (streamed)");
        const uint32_t nout = a.bins * s.batch;
        if (f64)
            hipLaunchKernelGGL(k_marg_stream_final<double>, dim3(nout), dim3(kBlock), 0, st, partial, a.wpr, a.bins,
                               reinterpret_cast<double*>(out));
        else
            hipLaunchKernelGGL(k_marg_stream_final<T>, dim3(nout), dim3(kBlock), 0, st, partial, a.wpr, a.bins,
                               reinterpret_cast<T*>(out));
        qf_status r2 = check_launch("qf_probs marginal final (streamed)");
        QF_HIP_CHECK(hipFreeAsync(partial, st));
        return r1 != QF_OK ? r1 : r2;
    });
}

qf_status launch_probs_marginal(const StateView& s, int m, const int32_t* qudits, void* out, bool f64,
                                hipStream_t st) {
    uint32_t nbins = 1;
    for (int i = 0; i < m; ++i) nbins *= s.dims[qudits[i]];
    // streamed when the measured qudits below the chunk stride have at most 16
    // digit combinations and there are at most 256 outcomes; gathered otherwise
    if (nbins <= 256) {
        MargSmall a{};
        a.N = s.N;
        a.m = uint32_t(m);
        a.bins = nbins;
        // chunk: the largest qudit stride <= 16384 (the register if smaller)
        a.per_wg = s.N;
        if (s.N > 16384) {
            a.per_wg = 1;
            for (int q = int(s.n) - 1; q >= 0 && s.strides[q] <= 16384; --q) a.per_wg = s.strides[q];
        }
        a.wpr = s.N / a.per_wg;
        uint32_t radix = 1, ncomb = 1;
        for (int i = m - 1; i >= 0; --i) {
            a.radix[i] = radix;
            radix *= s.dims[qudits[i]];
        }
        for (int i = 0; i < m; ++i) {
            a.stride[i].init(s.strides[qudits[i]]);
            a.dim[i].init(s.dims[qudits[i]]);
            if (s.strides[qudits[i]] < a.per_wg) {
                a.low[a.nlow++] = uint32_t(i);
                ncomb *= s.dims[qudits[i]];
            }
        }
        if (ncomb <= 16) {
            a.ncomb = ncomb;
            // bin offset of combination c: its low digits, last low qudit fastest
            for (uint32_t c = 0; c < ncomb; ++c) {
                uint32_t cc = c, y = 0;
                for (int j = int(a.nlow) - 1; j >= 0; --j) {
                    const uint32_t i = a.low[j], d = s.dims[qudits[i]];
                    y += (cc % d) * a.radix[i];
                    cc /= d;
                }
                a.ylo[c] = y;
            }
            if (ncomb <= 4) return launch_marg_stream<4>(s, a, out, f64, st);
            if (ncomb <= 8) return launch_marg_stream<8>(s, a, out, f64, st);
            return launch_marg_stream<16>(s, a, out, f64, st);
        }
    }
    MargArg a{};
    a.N = s.N;
    a.m = uint32_t(m);
    a.bins = 1;
    int maxp = -1;
    std::vector<bool> meas(s.n, false);
    for (int i = 0; i < m; ++i) {
        meas[qudits[i]] = true;
        maxp = qudits[i] > maxp ? qudits[i] : maxp;
        a.mstride[i] = s.strides[qudits[i]];
        a.mdiv[i].init(s.dims[qudits[i]]);
        a.bins *= s.dims[qudits[i]];
    }
    a.Z = s.N / a.bins;
    a.R = s.strides[maxp];
    a.divR.init(a.R);
    uint32_t u = 0;
    for (int p = 0; p < maxp; ++p)
        if (!meas[p]) {
            a.ostride[u] = s.strides[p];
            a.odiv[u++].init(s.dims[p]);
        }
    a.u = u;
    a.chunk = kBlock * 16;
    a.chunks = (a.Z + a.chunk - 1) / a.chunk;
    const uint64_t nblocks = uint64_t(a.chunks) * a.bins * s.batch;
    if (nblocks >= (1ull << 31)) return set_error(QF_ERANGE, "marginal grid too large");
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        double* partial = nullptr;
        QF_CHECK(dev_malloc_async(reinterpret_cast<void**>(&partial), nblocks * sizeof(double), st,
                                  "marginal partial sums"));
        hipLaunchKernelGGL(k_marg_partial<T>, dim3(uint32_t(nblocks)), dim3(kBlock), 0, st,
                           reinterpret_cast<const cplx<T>*>(s.amps), a, partial);
        qf_status r1 = check_launch("qf_probs marginal");
        const uint32_t nb = a.bins * s.batch;
        if (f64)
            hipLaunchKernelGGL(k_marg_final<double>, dim3(nb), dim3(kBlock), 0, st, partial, a.chunks,
                               reinterpret_cast<double*>(out));
        else
            hipLaunchKernelGGL(k_marg_final<T>, dim3(nb), dim3(kBlock), 0, st, partial, a.chunks,
                               reinterpret_cast<T*>(out));
        qf_status r2 = check_launch("qf_probs marginal final");
        QF_HIP_CHECK(hipFreeAsync(partial, st));
        return r1 != QF_OK ? r1 : r2;
    });
}

// Expectation chunk: the smallest qudit stride of at least 4096 amplitudes (the
// register if there is none), so a register has at most ceil(N / 4096) chunks.
static uint32_t expect_chunk(const StateView& s) {
    uint32_t c = s.N;
    for (int q = int(s.n) - 1; q >= 0; --q)
        if (s.strides[q] >= 4096) {
            c = s.strides[q];
            break;
        }
    return c;
}

static void set_low_terms(ObsArg& a, const StateView& s, const std::vector<int>& active, uint32_t chunk) {
    a.nlow = 0;
    for (size_t t = 0; t < active.size(); ++t)
        if (s.strides[active[t]] < chunk) a.low[a.nlow++] = uint32_t(t);
    // lanes span the largest qudit stride of at most kBlock amplitudes (and of
    // at most the chunk); the chunk is a multiple of it
    a.span = 1;
    for (int q = int(s.n) - 1; q >= 0; --q)
        if (s.strides[q] <= uint32_t(kBlock) && s.strides[q] <= chunk) a.span = s.strides[q];
    a.nrow = chunk / a.span;
    // (without low terms the plain loop has no per-element digit work)
    a.rows_table = a.nlow > 0 && a.nrow <= uint32_t(kMaxExpectRows) ? 1u : 0u;
}

size_t expect_ws_doubles(const StateView& s) {
    const uint32_t chunk = expect_chunk(s);
    const uint32_t nblk = (s.N + chunk - 1) / chunk;
    return size_t(nblk) * s.batch * 2;
}

qf_status launch_expect_ws(const StateView& s, const std::vector<int>& active, const std::vector<double>& table,
                           double* out, double* partial, hipStream_t st) {
    ObsArg a = make_obs(s, active, table, false);
    const uint32_t chunk = expect_chunk(s);
    set_low_terms(a, s, active, chunk);
    const uint32_t nblk = (s.N + chunk - 1) / chunk;
    const uint64_t nblocks = uint64_t(nblk) * s.batch;
    if (nblocks >= (1ull << 31)) return set_error(QF_ERANGE, "expectation grid too large");
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        hipLaunchKernelGGL(k_expect_partial<T>, dim3(uint32_t(nblocks)), dim3(kBlock), 0, st,
                           reinterpret_cast<const cplx<T>*>(s.amps), s.N, chunk, nblk, a, partial);
        QF_CHECK(check_launch("qf_expect"));
        hipLaunchKernelGGL(k_expect_final, dim3(s.batch), dim3(kBlock), 0, st, partial, nblk, out);
        return check_launch("qf_expect final");
    });
}

qf_status launch_expect(const StateView& s, const std::vector<int>& active, const std::vector<double>& table,
                        double* out, hipStream_t st) {
    ObsArg a = make_obs(s, active, table, false);
    const uint32_t chunk = expect_chunk(s);
    set_low_terms(a, s, active, chunk);
    const uint32_t nblk = (s.N + chunk - 1) / chunk;
    const uint64_t nblocks = uint64_t(nblk) * s.batch;
    if (nblocks >= (1ull << 31)) return set_error(QF_ERANGE, "expectation grid too large");
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        double* partial = nullptr;
        QF_CHECK(dev_malloc_async(reinterpret_cast<void**>(&partial), nblocks * 2 * sizeof(double), st,
                                  "expectation partial sums"));
        hipLaunchKernelGGL(k_expect_partial<T>, dim3(uint32_t(nblocks)), dim3(kBlock), 0, st,
                           reinterpret_cast<const cplx<T>*>(s.amps), s.N, chunk, nblk, a, partial);
        qf_status r1 = check_launch("qf_expect");
        hipLaunchKernelGGL(k_expect_final, dim3(s.batch), dim3(kBlock), 0, st, partial, nblk, out);
        qf_status r2 = check_launch("qf_expect final");
        QF_HIP_CHECK(hipFreeAsync(partial, st));
        return r1 != QF_OK ? r1 : r2;
    });
}

// ---------------------------------------------------------------------------
// Expectation values without allocation: the partial sums of every call on a
// GPU go to one file-scope device array, `scratch` (each GPU holds its own copy
// until the process ends).  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device, looked up once per
// device on the first call there.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchDoubles = size_t(1) << 19;  // 4 MiB
__device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_addr;  // device address of scratch, per device id
}  // namespace

static qf_status scratch_address(double** out) {
    int dev = 0;
    QF_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (size_t(dev) >= g_scratch_addr.size()) g_scratch_addr.resize(size_t(dev) + 1, nullptr);
    if (g_scratch_addr[size_t(dev)] == nullptr) {
        void* p = nullptr;
        QF_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_addr[size_t(dev)] = static_cast<double*>(p);
    }
    *out = g_scratch_addr[size_t(dev)];
    return QF_OK;
}

qf_status launch_expect_noalloc(const StateView& s, const std::vector<int>& active, const std::vector<double>& table,
                                double* out, hipStream_t st) {
    const size_t need = expect_ws_doubles(s);
    if (need > kScratchDoubles)
        return set_error(QF_ERANGE, "qf_expect_noalloc: %zu partial sums exceed the %zu of the library's scratch "
                         "array (batch * chunks per register must be <= %zu)", need / 2, kScratchDoubles / 2,
                         kScratchDoubles / 2);
    double* ws = nullptr;
    QF_CHECK(scratch_address(&ws));
    // every partial is written before it is read: nothing to clear
    return launch_expect_ws(s, active, table, out, ws, st);
}

qf_status launch_diag_observable(const StateView& s, void* lam_amps, const std::vector<int>& active,
                                 const std::vector<double>& table_re, hipStream_t st) {
    ObsArg a = make_obs(s, active, table_re, true);
    return with_type(s.dtype, [&](auto tag) -> qf_status {
        using T = decltype(tag);
        hipLaunchKernelGGL(k_diag_observable<T>, dim3(grid_for(s.total, kBlock * 4)), dim3(kBlock), 0, st,
                           reinterpret_cast<const cplx<T>*>(s.amps), reinterpret_cast<cplx<T>*>(lam_amps),
                           s.total, FastDiv(s.N), s.N, a);
        return check_launch("diag observable");
    });
}

}  // namespace qf
