// Fused LDS stages: one HBM pass applies every gate of a stage to a tile of k
// qudits held in LDS.
//
// Load/store: tile element e lives at base + offhi[e / R] + e % R; consecutive
// lanes take consecutive e, so each wavefront reads contiguous runs of R = D^r
// amplitudes (r low qudits are always in the tile).  Workgroups map to tiles
// through tile_of_block, which keeps neighbouring tiles on one XCD.
//
// Ops (read from a device array; every lane reads the same op, so the loads are
// scalar):
//   SOP_U      dense D x D matrix on one tile qudit.
//   SOP_SHIFT  x_t -> x_t + shifts[x_c] mod D on a tile qudit t; the control may
//              be any qudit, inside or outside the tile.  Pure data movement.
//   SOP_PHASE  product of two-qudit diagonal factors table[x_a * D + x_b]; a and
//              b may be any qudits.
//
// Kernels: k_stage (one LDS sweep per op), k_stage_rounds (register rounds, the
// default; see "Register rounds" below), k_stage_pipe (register rounds in a
// persistent grid with the next tile prefetched into registers), and the
// reverse-stage kernels k_stage_adj / k_stage_adj_rounds, which apply the
// inverted ops to psi and lam and accumulate the adjoint's M matrices.
#include <algorithm>
#include <type_traits>

#include "qf_internal.h"

namespace qf {
namespace {

constexpr int kSB = 256;

// Workgroup barrier for LDS data only: waits for this wave's LDS operations
// (lgkmcnt) and meets the other waves, without the fence of __syncthreads that
// would also wait for every outstanding global load (the pipelined kernel keeps
// the next tile's loads in flight across these barriers).  The memory clobber
// keeps the compiler from moving memory accesses across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Logical tile (register-major) of this workgroup.  Workgroups are dispatched
// round-robin over the 8 XCDs, each with its own L2; with g.xcd set, this
// bijection of [0, gridDim.x) hands every XCD a contiguous range of tiles, so
// neighbouring tiles (whose runs share cache lines when runs are short) go
// through the same L2 at about the same time.
constexpr uint32_t kXCD = 8;

__device__ inline uint32_t xcd_range_start(uint32_t x, uint32_t total) {
    const uint32_t q = total / kXCD, rem = total % kXCD;
    return x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
}

__device__ inline uint32_t tile_of_block(const StageGeom& g) {
    if (!g.xcd) return blockIdx.x;
    return xcd_range_start(blockIdx.x % kXCD, gridDim.x) + blockIdx.x / kXCD;
}

template <int D>
__device__ inline uint32_t tile_base(const StageGeom& g, uint32_t blk) {
    const uint32_t b = blk / g.ntiles;
    uint32_t t = blk - b * g.ntiles;
    uint32_t base = b * g.N;
    for (int j = int(g.nout) - 1; j >= 0; --j) {
        const uint32_t q = t / D;
        base += (t - q * D) * g.out_stride[j];
        t = q;
    }
    return base;
}

template <int D>
__device__ inline void build_offhi(const StageGeom& g, uint32_t* offhi) {
    const int nh = int(g.k - g.r);
    for (uint32_t h = threadIdx.x; h < g.nhi; h += blockDim.x) {
        uint32_t hh = h, off = 0;
        for (int i = nh - 1; i >= 0; --i) {
            const uint32_t q = hh / D;
            off += (hh - q * D) * g.hi_stride[i];
            hh = q;
        }
        offhi[h] = off;
    }
}

__device__ inline uint32_t global_index(const StageGeom& g, const uint32_t* offhi, uint32_t base, uint32_t e) {
    const uint32_t eh = g.divR.div(e);
    return base + offhi[eh] + (e - eh * g.R);
}

// Loads and stores go in batches of kIO per lane so that kIO global accesses
// per lane are in flight before the first one is waited on.
constexpr int kIO = 8;

// Tile I/O by runs: the tile is nhi runs of R contiguous amplitudes (run h
// starts at base + offhi[h] in HBM and at h * R in LDS).  A lane keeps one
// offset o inside a run and walks runs, so no per-element division is needed:
// with R < 256 the lanes form G = 256 / R groups of R (group gr takes runs
// gr, gr + G, ...); otherwise every lane strides through each run by 256.
template <typename T, bool LOAD, typename Ref>
__device__ __forceinline__ void tile_io_runs(cplx<T>* tile, const StageGeom& g, uint32_t G, uint32_t gr, uint32_t o,
                                             Ref&& at) {
    uint32_t h = gr;
    for (; h + (kIO - 1) * G < g.nhi; h += G * kIO) {
        cplx<T> t[kIO];
        if (LOAD) {
#pragma unroll
            for (int j = 0; j < kIO; ++j) t[j] = at(h + j * G);
#pragma unroll
            for (int j = 0; j < kIO; ++j) tile[(h + j * G) * g.R + o] = t[j];
        } else {
#pragma unroll
            for (int j = 0; j < kIO; ++j) t[j] = tile[(h + j * G) * g.R + o];
#pragma unroll
            for (int j = 0; j < kIO; ++j) at(h + j * G) = t[j];
        }
    }
    for (; h < g.nhi; h += G) {
        if (LOAD)
            tile[h * g.R + o] = at(h);
        else
            at(h) = tile[h * g.R + o];
    }
}

template <typename T, bool LOAD>
__device__ inline void tile_io(cplx<T>* __restrict__ psi, cplx<T>* tile, const StageGeom& g, const uint32_t* offhi,
                               uint32_t base) {
    if (g.R < blockDim.x) {
        const uint32_t G = blockDim.x / g.R;
        const uint32_t gr = threadIdx.x / g.R;
        const uint32_t o = threadIdx.x - gr * g.R;
        if (gr >= G) return;
        if (uint64_t(g.N) * sizeof(cplx<T>) <= 0xffffffffull) {
            // registers below 4 GB: one uniform 64-bit tile pointer and 32-bit
            // byte offsets (scalar-base addressing, one VALU op per access)
            char* pb = reinterpret_cast<char*>(psi + base);
            tile_io_runs<T, LOAD>(tile, g, G, gr, o, [&](uint32_t h) -> cplx<T>& {
                return *reinterpret_cast<cplx<T>*>(pb + (offhi[h] + o) * uint32_t(sizeof(cplx<T>)));
            });
            return;
        }
        tile_io_runs<T, LOAD>(tile, g, G, gr, o, [&](uint32_t h) -> cplx<T>& { return psi[base + offhi[h] + o]; });
        return;
    }
    for (uint32_t h = 0; h < g.nhi; ++h) {
        const uint32_t gb = base + offhi[h];
        for (uint32_t o = threadIdx.x; o < g.R; o += blockDim.x) {
            if (LOAD)
                tile[h * g.R + o] = psi[gb + o];
            else
                psi[gb + o] = tile[h * g.R + o];
        }
    }
}

template <typename T>
__device__ inline void tile_load(const cplx<T>* __restrict__ psi, cplx<T>* tile, const StageGeom& g,
                                 const uint32_t* offhi, uint32_t base) {
    tile_io<T, true>(const_cast<cplx<T>*>(psi), tile, g, offhi, base);
}

template <typename T>
__device__ inline void tile_store(cplx<T>* __restrict__ psi, const cplx<T>* tile, const StageGeom& g,
                                  const uint32_t* offhi, uint32_t base) {
    tile_io<T, false>(psi, const_cast<cplx<T>*>(tile), g, offhi, base);
}

template <typename T, int D>
__device__ inline void matvec(const cplx<T>* __restrict__ M, bool real, const cplx<T> (&v)[D], cplx<T> (&w)[D]) {
    if (real) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                const T m = M[a * D + b].re;
                re = fma(m, v[b].re, re);
                im = fma(m, v[b].im, im);
            }
            w[a] = cmake<T>(re, im);
        }
    } else {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            cplx<T> acc = cmake<T>(0, 0);
#pragma unroll
            for (int b = 0; b < D; ++b) cmac(acc, M[a * D + b], v[b]);
            w[a] = acc;
        }
    }
}

template <typename T, int D>
__device__ inline void op_u(cplx<T>* tile, const StageGeom& g, const StageOp& op, const cplx<T>* __restrict__ M) {
    const uint32_t nf = g.TE / D;
    const uint32_t ls = op.ls;
    const bool real = op.real != 0;
    for (uint32_t f = threadIdx.x; f < nf; f += kSB) {
        const uint32_t hi = op.divls.div(f);
        const uint32_t lb = hi * (uint32_t(D) * ls) + (f - hi * ls);
        cplx<T> v[D], w[D];
#pragma unroll
        for (int d = 0; d < D; ++d) v[d] = tile[lb + uint32_t(d) * ls];
        matvec<T, D>(M, real, v, w);
#pragma unroll
        for (int d = 0; d < D; ++d) tile[lb + uint32_t(d) * ls] = w[d];
    }
}

template <int D>
__device__ inline int shift_amount(const StageOp& op, uint32_t gidx) {
    if (!op.has_ctrl) return op.shifts[0];
    const uint32_t xc = op.ctrl_stride.div(gidx) % D;
    int s = op.shifts[0];
#pragma unroll
    for (int a = 1; a < D; ++a) s = (xc == uint32_t(a)) ? op.shifts[a] : s;
    return s;
}

// v[b] <- v[(b - s) mod D] as a barrel of rotations by 1, 2, 4, ...: every
// register index is a compile-time constant, so nothing is spilled.
template <typename T, int D>
__device__ inline void shift_fibre(cplx<T>* tile, uint32_t lb, uint32_t ls, int s) {
    cplx<T> v[D];
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = tile[lb + uint32_t(d) * ls];
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
#pragma unroll
    for (int d = 0; d < D; ++d) tile[lb + uint32_t(d) * ls] = v[d];
}

template <int D>
__device__ inline uint32_t fibre_lb(const StageOp& op, uint32_t f) {
    const uint32_t hi = op.divls.div(f);
    return hi * (uint32_t(D) * op.ls) + (f - hi * op.ls);
}

template <typename T, int D>
__device__ inline cplx<T> phase_of(const StageOp& op, const cplx<T>* __restrict__ M, uint32_t gidx) {
    cplx<T> ph = cmake<T>(1, 0);
    for (int p = 0; p < op.npairs; ++p) {
        const uint32_t xa = op.pa[p].div(gidx) % D;
        const uint32_t xb = op.pb[p].div(gidx) % D;
        ph = cmul(ph, M[op.ptab[p] + xa * D + xb]);
    }
    return ph;
}

template <typename T, int D>
__global__ __launch_bounds__(kSB) void k_stage(cplx<T>* __restrict__ psi, StageGeom g,
                                               const StageOp* __restrict__ ops, int nops,
                                               const cplx<T>* __restrict__ mats, size_t mat_stride) {
    const uint32_t blk = tile_of_block(g);
    mats += size_t(blk / g.ntiles) * mat_stride;  // per-register matrices (stride 0: shared)
    extern __shared__ unsigned char smem[];
    cplx<T>* tile = reinterpret_cast<cplx<T>*>(smem);
    uint32_t* offhi = reinterpret_cast<uint32_t*>(tile + g.TE);
    const uint32_t base = tile_base<D>(g, blk);
    build_offhi<D>(g, offhi);
    __syncthreads();
    tile_load(psi, tile, g, offhi, base);
    __syncthreads();
    for (int oi = 0; oi < nops; ++oi) {
        const StageOp& op = ops[oi];
        if (op.type == SOP_U) {
            op_u<T, D>(tile, g, op, mats + op.mat);
        } else if (op.type == SOP_SHIFT) {
            const uint32_t nf = g.TE / D;
            for (uint32_t f = threadIdx.x; f < nf; f += kSB) {
                const uint32_t lb = fibre_lb<D>(op, f);
                const int s = shift_amount<D>(op, global_index(g, offhi, base, lb));
                if (s != 0) shift_fibre<T, D>(tile, lb, op.ls, s);
            }
        } else {
            for (uint32_t e = threadIdx.x; e < g.TE; e += kSB)
                tile[e] = cmul(tile[e], phase_of<T, D>(op, mats, global_index(g, offhi, base, e)));
        }
        __syncthreads();
    }
    tile_store(psi, tile, g, offhi, base);
}

// Reverse stage on psi and lam.  Before a U with slot >= 0, lane (entry, part)
// sums psi_f[a] conj(lam_f[c]) over the fibres f = part, part + P, ... and the
// parts are then added in a fixed order.
template <typename T, int D>
__global__ __launch_bounds__(kSB) void k_stage_adj(cplx<T>* __restrict__ psi, cplx<T>* __restrict__ lam,
                                                   StageGeom g, const StageOp* __restrict__ ops, int nops,
                                                   const cplx<T>* __restrict__ mats, size_t mat_stride,
                                                   double* __restrict__ partial) {
    const uint32_t blk = tile_of_block(g);
    mats += size_t(blk / g.ntiles) * mat_stride;
    extern __shared__ unsigned char smem[];
    cplx<T>* tp = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* tl = tp + g.TE;
    uint32_t* offhi = reinterpret_cast<uint32_t*>(tl + g.TE);
    __shared__ double red[2][kSB];
    constexpr int E = D * D;
    constexpr int P = kSB / E;
    const uint32_t nblocks = gridDim.x;
    const uint32_t base = tile_base<D>(g, blk);
    build_offhi<D>(g, offhi);
    __syncthreads();
    tile_load(psi, tp, g, offhi, base);
    tile_load(lam, tl, g, offhi, base);
    __syncthreads();
    const uint32_t nf = g.TE / D;
    for (int oi = 0; oi < nops; ++oi) {
        const StageOp& op = ops[oi];
        if (op.type == SOP_U) {
            if (op.slot >= 0) {
                const int e = threadIdx.x % E;
                const int part = threadIdx.x / E;
                double ar = 0.0, ai = 0.0;
                if (part < P) {
                    const uint32_t a = uint32_t(e / D), c = uint32_t(e % D);
                    for (uint32_t f = part; f < nf; f += P) {
                        const uint32_t lb = fibre_lb<D>(op, f);
                        const cplx<T> x = tp[lb + a * op.ls];
                        const cplx<T> y = tl[lb + c * op.ls];
                        ar += double(x.re) * double(y.re) + double(x.im) * double(y.im);
                        ai += double(x.im) * double(y.re) - double(x.re) * double(y.im);
                    }
                }
                red[0][threadIdx.x] = ar;
                red[1][threadIdx.x] = ai;
                __syncthreads();
                if (int(threadIdx.x) < E) {
                    double sr = 0.0, si = 0.0;
                    for (int p = 0; p < P; ++p) {
                        sr += red[0][p * E + threadIdx.x];
                        si += red[1][p * E + threadIdx.x];
                    }
                    double* o = partial + ((size_t(op.slot) * nblocks + blk) * E + threadIdx.x) * 2;
                    o[0] = sr;
                    o[1] = si;
                }
                __syncthreads();
            }
            op_u<T, D>(tp, g, op, mats + op.mat);
            op_u<T, D>(tl, g, op, mats + op.mat);
        } else if (op.type == SOP_SHIFT) {
            for (uint32_t f = threadIdx.x; f < nf; f += kSB) {
                const uint32_t lb = fibre_lb<D>(op, f);
                const int s = shift_amount<D>(op, global_index(g, offhi, base, lb));
                if (s != 0) {
                    shift_fibre<T, D>(tp, lb, op.ls, s);
                    shift_fibre<T, D>(tl, lb, op.ls, s);
                }
            }
        } else {
            for (uint32_t e = threadIdx.x; e < g.TE; e += kSB) {
                const cplx<T> ph = phase_of<T, D>(op, mats, global_index(g, offhi, base, e));
                tp[e] = cmul(tp[e], ph);
                tl[e] = cmul(tl[e], ph);
            }
        }
        __syncthreads();
    }
    tile_store(psi, tp, g, offhi, base);
    tile_store(lam, tl, g, offhi, base);
}

// One workgroup per (register, slot, entry): lanes sum the tiles
// i = lane, lane + 256, ... of the register, then a fixed tree.
__global__ __launch_bounds__(kSB) void k_stage_mreduce(const double* __restrict__ partial, uint32_t nslots,
                                                       uint32_t ntiles, uint32_t batch, uint32_t E,
                                                       double* __restrict__ mout, uint32_t nslots_total,
                                                       uint32_t slot0) {
    __shared__ double red[2][kSB];
    const uint32_t e = blockIdx.x % E;
    const uint32_t bj = blockIdx.x / E;
    const uint32_t b = bj / nslots;
    const uint32_t j = bj - b * nslots;
    const uint32_t nblocks = ntiles * batch;
    double ar = 0.0, ai = 0.0;
    for (uint32_t i = threadIdx.x; i < ntiles; i += kSB) {
        const double* p = partial + ((size_t(j) * nblocks + b * ntiles + i) * E + e) * 2;
        ar += p[0];
        ai += p[1];
    }
    red[0][threadIdx.x] = ar;
    red[1][threadIdx.x] = ai;
    __syncthreads();
    for (int w = kSB / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = mout + ((size_t(b) * nslots_total + slot0 + j) * E + e) * 2;
        o[0] = red[0][0];
        o[1] = red[1][0];
    }
}

// ---------------------------------------------------------------------------
// Register rounds.  Register index i of a lane's sub-tile has digits
// (i_0, ..., i_{M-1}) (i_0 most significant); digit j belongs to the round's
// j-th group qudit.  All register indices are compile-time constants.
//
// A round loads every lane's sub-tile from LDS, applies its in-place ops (U on
// any group position, PHASE) in registers and stores the sub-tile back.  A
// round may also carry permutation ops (SHIFT): they move data only, so they
// are folded into the LDS addresses of the loads (before the in-place ops) or
// of the stores (after them) and cost no register moves (load_addrs).
// ---------------------------------------------------------------------------

constexpr int cpow(int b, int e) { return e == 0 ? 1 : b * cpow(b, e - 1); }

template <int D, int M, int J>
__device__ constexpr int rdigit(int i) {
    return (i / cpow(D, M - 1 - J)) % D;
}

// U on group position J: every fibre along J (digits of the other positions
// fixed) is multiplied by U.  The matrix is uniform and held in scalar
// registers; REAL uses only its real parts.
template <typename T, int D, int M, int J, bool REAL>
__device__ __forceinline__ void r_u(cplx<T> (&v)[cpow(D, M)], const cplx<T>* __restrict__ U) {
    constexpr int SJ = cpow(D, M - 1 - J);
    constexpr int NF = cpow(D, M - 1);
    // matrices up to 4 x 4 are read once into scalar registers; larger ones
    // are read from memory where used (a local copy spills into vector
    // registers and lowers occupancy)
    constexpr bool kCopy = D <= 4;
    cplx<T> m[kCopy ? D * D : 1];
    if constexpr (kCopy) {
#pragma unroll
        for (int e = 0; e < D * D; ++e) m[e] = U[e];
    }
    auto mat = [&](int e) -> cplx<T> {
        if constexpr (kCopy) return m[e];
        else return U[e];
    };
#pragma unroll
    for (int c = 0; c < NF; ++c) {
        const int b0 = (c / SJ) * SJ * D + (c % SJ);
        cplx<T> y[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if constexpr (REAL) {
                T re = 0, im = 0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const T w = mat(a * D + d).re;
                    re = fma(w, v[b0 + d * SJ].re, re);
                    im = fma(w, v[b0 + d * SJ].im, im);
                }
                y[a] = cmake<T>(re, im);
            } else {
                cplx<T> acc = cmake<T>(0, 0);
#pragma unroll
                for (int d = 0; d < D; ++d) cmac(acc, mat(a * D + d), v[b0 + d * SJ]);
                y[a] = acc;
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) v[b0 + d * SJ] = y[d];
    }
}

template <typename T, int D, int M, int J>
__device__ __forceinline__ void r_u_any(cplx<T> (&v)[cpow(D, M)], const cplx<T>* __restrict__ U, bool real) {
    if (real)
        r_u<T, D, M, J, true>(v, U);
    else
        r_u<T, D, M, J, false>(v, U);
}

// CZ factors multiply amplitude x by w^e(x) with e(x) = sum over factors of
// x_a x_b.  Within a lane's sub-tile the digits outside the group are
// constant, so e is a quadratic form in the group digits d_j:
//   e = e0 + sum_j lin_j d_j + sum_{j<l} quad_jl d_j d_l,
// whose coefficients are accumulated once per sub-tile.
template <typename T, int D, int M>
__device__ __forceinline__ void r_phase(cplx<T> (&v)[cpow(D, M)], const StageOp& op, const cplx<T>* __restrict__ mats,
                               uint32_t gidx0) {
    constexpr int DM = cpow(D, M);
    int e0 = 0;
    int lin[M];
    int quad[M][M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        lin[j] = 0;
#pragma unroll
        for (int l = 0; l < M; ++l) quad[j][l] = 0;
    }
    for (int p = 0; p < op.npairs; ++p) {
        const int ag = op.agpos[p], bg = op.bgpos[p];
        const int ca = ag < 0 ? int(op.pa[p].div(gidx0) % D) : 0;
        const int cb = bg < 0 ? int(op.pb[p].div(gidx0) % D) : 0;
        if (ag < 0 && bg < 0) e0 += ca * cb;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            lin[j] += (ag == j && bg < 0) ? cb : 0;
            lin[j] += (bg == j && ag < 0) ? ca : 0;
#pragma unroll
            for (int l = 0; l < M; ++l) quad[j][l] += ((ag == j && bg == l) || (ag == l && bg == j)) ? 1 : 0;
        }
    }
    const cplx<T>* W = mats + op.wtab;
#pragma unroll
    for (int i = 0; i < DM; ++i) {
        int e = e0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int dj = (i / cpow(D, M - 1 - j)) % D;
            e += lin[j] * dj;
#pragma unroll
            for (int l = j + 1; l < M; ++l) e += quad[j][l] * dj * ((i / cpow(D, M - 1 - l)) % D);
        }
        v[i] = cmul(v[i], W[e % D]);
    }
}

// LDS byte offset of register i over group positions 1 .. M-1 (glsb: the
// group's byte strides; uniform, so this is scalar work).
template <int D, int M>
__device__ __forceinline__ uint32_t rest_offset(int i, const uint32_t* glsb) {
    uint32_t o = 0;
#pragma unroll
    for (int j = 1; j < M; ++j) o += uint32_t((i / cpow(D, M - 1 - j)) % D) * glsb[j];
    return o;
}

// (d + s) mod D for d, s in [0, D)
template <int D>
__device__ __forceinline__ uint32_t add_mod(uint32_t d, uint32_t s) {
    const uint32_t t = d + s;
    return t >= uint32_t(D) ? t - uint32_t(D) : t;
}

// LDS byte offset of register i over group positions 2 .. M-1.
template <int D, int M>
__device__ __forceinline__ uint32_t rest2_offset(int i, const uint32_t* glsb) {
    uint32_t o = 0;
#pragma unroll
    for (int j = 2; j < M; ++j) o += uint32_t((i / cpow(D, M - 1 - j)) % D) * glsb[j];
    return o;
}

// LDS access by 32-bit LDS byte address: a tile's base is added once to a
// sub-tile's base address, not once per access.
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return uint32_t(uintptr_t((const __attribute__((address_space(3))) unsigned char*)p));
}

template <typename T>
__device__ __forceinline__ cplx<T> lds_ld(uint32_t a) {
    typedef typename Vec2<T>::type V;
    const V x = *(const __attribute__((address_space(3))) V*)uintptr_t(a);
    return cmake<T>(x.x, x.y);
}

template <typename T>
__device__ __forceinline__ void lds_st(uint32_t a, cplx<T> v) {
    typedef typename Vec2<T>::type V;
    V x;
    x.x = v.re;
    x.y = v.im;
    *(__attribute__((address_space(3))) V*)uintptr_t(a) = x;
}

// Shift of a permutation op whose control is not a group qudit: one value per
// lane (the control digit is constant over the sub-tile), or shifts[0] when
// the op has no control.
template <int D, class Perm>
__device__ __forceinline__ uint32_t lane_shift(const Perm& P, uint32_t gidx0) {
    uint32_t sh = uint32_t(P.shifts[0]);
    if (P.has_ctrl) {
        const uint32_t xc = P.ctrl_stride.div(gidx0) % D;
        if (P.shift_mul >= 0) {
            // affine table shifts[c] = (mul * c + shifts[0]) mod D (CSUM: mul = 1)
            sh = (uint32_t(P.shift_mul) * xc + sh) % D;
        } else {
#pragma unroll
            for (int c = 1; c < D; ++c) sh = xc == uint32_t(c) ? uint32_t(P.shifts[c]) : sh;
        }
    }
    return sh;
}

template <int D>
__device__ __forceinline__ uint32_t neg_mod(uint32_t s) {
    return s == 0 ? 0u : uint32_t(D) - s;
}

// Permutation ops of a round (each x_t -> x_t + shifts[x_c] mod D):
//   pre0  target group position 0, control position 1, per lane or none;
//   pre1  target position 1, control position 0;
//   post  target position 0, control position 1, per lane or none.
// pre0 then pre1 act before the in-place ops: register (d0, d1) loads the
// amplitude they bring there, from (d0 - s0, d1 - s1(d0)).  post acts after
// them: register (d0, d1) stores to (d0 + s(d1), d1).  Addresses are LDS byte
// addresses (tbb: the sub-tile's register 0).
template <int D, int M>
__device__ __forceinline__ void load_addrs(uint32_t (&a)[cpow(D, M)], uint32_t tbb, const RoundDesc& rd,
                                           uint32_t gidx0) {
    constexpr int DM = cpow(D, M);
    const uint32_t g0 = rd.glsb[0];
    if constexpr (M >= 2) {
        if (rd.pre1 >= 0) {
            uint32_t od[D];
            const uint32_t s0 = rd.pre0 >= 0 ? neg_mod<D>(lane_shift<D>(rd.perm[0], gidx0)) : 0u;
#pragma unroll
            for (int d = 0; d < D; ++d) od[d] = tbb + __umul24(add_mod<D>(uint32_t(d), s0), g0);
            const uint32_t g1 = rd.glsb[1];
#pragma unroll
            for (int i = 0; i < DM; ++i) {
                const int d0 = rdigit<D, M, 0>(i);
                const uint32_t e1 = add_mod<D>(uint32_t(rdigit<D, M, 1>(i)), neg_mod<D>(uint32_t(rd.perm[1].shifts[d0])));
                a[i] = od[d0] + (e1 * g1 + rest2_offset<D, M>(i, rd.glsb));
            }
            return;
        }
    }
    if (rd.pre0 < 0) {
#pragma unroll
        for (int i = 0; i < DM; ++i) a[i] = tbb + (uint32_t(rdigit<D, M, 0>(i)) * g0 + rest_offset<D, M>(i, rd.glsb));
        return;
    }
    const PermDesc& P = rd.perm[0];
    if constexpr (M >= 2) {
        if (P.ctrl_gpos == 1) {
#pragma unroll
            for (int i = 0; i < DM; ++i) {
                const uint32_t s = neg_mod<D>(uint32_t(P.shifts[rdigit<D, M, 1>(i)]));
                a[i] = tbb + (add_mod<D>(uint32_t(rdigit<D, M, 0>(i)), s) * g0 + rest_offset<D, M>(i, rd.glsb));
            }
            return;
        }
    }
    const uint32_t s = neg_mod<D>(lane_shift<D>(P, gidx0));
    uint32_t od[D];
#pragma unroll
    for (int d = 0; d < D; ++d) od[d] = tbb + __umul24(add_mod<D>(uint32_t(d), s), g0);
#pragma unroll
    for (int i = 0; i < DM; ++i) a[i] = od[rdigit<D, M, 0>(i)] + rest_offset<D, M>(i, rd.glsb);
}

// Digits of sub-tile u over the k - M other tile qudits, least significant
// first, one byte each; the first 8 digits.
struct SubDigits {
    uint32_t w[2];
};

// pre2 on the load addresses (after pre0 and pre1): its target is one of the
// lane's own digits x_t and its control is group position 1, so register i
// loads from x_t - s(d_1(i)), an offset per value of that digit.  The
// amplitudes come from other lanes' sub-tiles (see run_round).
template <int D, int M>
__device__ __forceinline__ void add_pre2(uint32_t (&a)[cpow(D, M)], const RoundDesc& rd, const SubDigits& dg) {
    constexpr int DM = cpow(D, M);
    const int b = rd.pre2_byte;
    const uint32_t xt = (((b >> 2) != 0 ? dg.w[1] : dg.w[0]) >> (8 * (b & 3))) & 0xffu;
    const uint32_t ls = rd.pre2_lsb;
    uint32_t o2[D];
#pragma unroll
    for (int d = 0; d < D; ++d) o2[d] = (add_mod<D>(xt, neg_mod<D>(uint32_t(rd.pre2_shifts[d]))) - xt) * ls;
#pragma unroll
    for (int i = 0; i < DM; ++i) a[i] += o2[rdigit<D, M, 1>(i)];
}

template <int D, int M>
__device__ __forceinline__ void store_addrs(uint32_t (&a)[cpow(D, M)], uint32_t tbb, const RoundDesc& rd,
                                            uint32_t gidx0) {
    constexpr int DM = cpow(D, M);
    const uint32_t g0 = rd.glsb[0];
    if (rd.post < 0) {
#pragma unroll
        for (int i = 0; i < DM; ++i) a[i] = tbb + (uint32_t(rdigit<D, M, 0>(i)) * g0 + rest_offset<D, M>(i, rd.glsb));
        return;
    }
    const PermDesc& P = rd.perm[2];
    if constexpr (M >= 2) {
        if (P.ctrl_gpos == 1) {
#pragma unroll
            for (int i = 0; i < DM; ++i) {
                const uint32_t s = uint32_t(P.shifts[rdigit<D, M, 1>(i)]);
                a[i] = tbb + (add_mod<D>(uint32_t(rdigit<D, M, 0>(i)), s) * g0 + rest_offset<D, M>(i, rd.glsb));
            }
            return;
        }
    }
    const uint32_t s = lane_shift<D>(P, gidx0);
    uint32_t od[D];
#pragma unroll
    for (int d = 0; d < D; ++d) od[d] = tbb + __umul24(add_mod<D>(uint32_t(d), s), g0);
#pragma unroll
    for (int i = 0; i < DM; ++i) a[i] = od[rdigit<D, M, 0>(i)] + rest_offset<D, M>(i, rd.glsb);
}

template <typename T, int D, int M>
__device__ __forceinline__ void round_ops(cplx<T> (&v)[cpow(D, M)], const RoundDesc& rd, const StageOp* __restrict__ ops,
                                 const cplx<T>* __restrict__ mats, uint32_t gidx0) {
    for (int oi = rd.op0; oi < rd.op0 + rd.nops; ++oi) {
        const StageOp& op = ops[oi];
        if (op.type == SOP_U) {
            const cplx<T>* U = mats + op.mat;
            const bool real = op.real != 0;
            switch (op.gpos) {
                case 0: r_u_any<T, D, M, 0>(v, U, real); break;
                case 1: if constexpr (M > 1) r_u_any<T, D, M, 1>(v, U, real); break;
                case 2: if constexpr (M > 2) r_u_any<T, D, M, 2>(v, U, real); break;
                case 3: if constexpr (M > 3) r_u_any<T, D, M, 3>(v, U, real); break;
                case 4: if constexpr (M > 4) r_u_any<T, D, M, 4>(v, U, real); break;
            }
        } else {
            r_phase<T, D, M>(v, op, mats, gidx0);
        }
    }
}

template <int D>
__device__ __forceinline__ SubDigits sub_digits(uint32_t u, int nother) {
    SubDigits s;
    s.w[0] = s.w[1] = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (j < nother) {
            const uint32_t q = u / D;
            s.w[j >> 2] |= (u - q * D) << (8 * (j & 3));
            u = q;
        }
    }
    return s;
}

typedef unsigned short qf_u16x2 __attribute__((ext_vector_type(2)));

// LDS index of the sub-tile's register 0 in round rd: dot products of the digit
// pairs with the round's stride pairs (v_dot2_u32_u16).  Rounds have at most 8
// other qudits (the planner runs larger tiles op by op).
template <int D>
__device__ __forceinline__ uint32_t sub_base(const SubDigits& s, const RoundDesc& rd) {
    uint32_t tb = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        if (2 * w < rd.nother) {
            // bytes 2w, 2w+1 of the digits as the two 16-bit halves (v_perm_b32)
            const uint32_t pr = __builtin_amdgcn_perm(0u, s.w[w >> 1], (w & 1) ? 0x0C030C02u : 0x0C010C00u);
            tb = __builtin_amdgcn_udot2(__builtin_bit_cast(qf_u16x2, pr), __builtin_bit_cast(qf_u16x2, rd.spair[w]),
                                        tb, false);
        }
    return tb;
}

// Adjoint M of a fused run U (the first op of its round, on group position J):
// M = sum over the fibres f along J of psi_f lam_f^dagger.  Each lane sums its
// own fibres in registers (MAcc); mreduce_block then adds the lanes in a fixed
// order (DPP butterflies inside 16-lane rows, then the rows in order, in FP64).
template <typename T, int D>
struct MAcc {
    T re[D * D], im[D * D];
};

template <typename T, int D, int M, int J>
__device__ __forceinline__ void macc_add(MAcc<T, D>& m, const cplx<T> (&p)[cpow(D, M)],
                                         const cplx<T> (&l)[cpow(D, M)]) {
    constexpr int SJ = cpow(D, M - 1 - J);
    constexpr int NF = cpow(D, M - 1);
#pragma unroll
    for (int c = 0; c < NF; ++c) {
        const int b0 = (c / SJ) * SJ * D + (c % SJ);
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int e = 0; e < D; ++e) {
                const cplx<T> x = p[b0 + a * SJ], y = l[b0 + e * SJ];
                m.re[a * D + e] = fma(x.re, y.re, fma(x.im, y.im, m.re[a * D + e]));
                m.im[a * D + e] = fma(x.im, y.re, fma(-x.re, y.im, m.im[a * D + e]));
            }
    }
}

// DPP moves (lane permutations inside 16-lane rows; VALU only, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, 0xf, 0xf, false));
    const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, 0xf, 0xf, false));
    return __builtin_bit_cast(double, uint64_t(lo) | (uint64_t(hi) << 32));
}

// Row sums by DPP (every lane of a 16-lane row then holds its row's sum); the
// first lane of each row writes it to LDS, and E lanes add the rows of all
// wavefronts in a fixed order in FP64.
template <typename T>
__device__ __forceinline__ T row_sum(T v) {
    if constexpr (sizeof(T) == 4) {
        v += dpp_f32<0xB1>(v);   // quad_perm [1,0,3,2]
        v += dpp_f32<0x4E>(v);   // quad_perm [2,3,0,1]
        v += dpp_f32<0x124>(v);  // row_ror:4
        v += dpp_f32<0x128>(v);  // row_ror:8
    } else {
        v += dpp_f64<0xB1>(v);
        v += dpp_f64<0x4E>(v);
        v += dpp_f64<0x124>(v);
        v += dpp_f64<0x128>(v);
    }
    return v;
}

template <typename T, int D>
__device__ __forceinline__ void mreduce_block(MAcc<T, D>& m, double (*red)[kSB], double* __restrict__ out) {
    constexpr int E = D * D;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        m.re[e] = row_sum(m.re[e]);
        m.im[e] = row_sum(m.im[e]);
    }
    const uint32_t row = threadIdx.x / 16, nrows = (blockDim.x + 15) / 16;
    if ((threadIdx.x & 15) == 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            red[0][row * E + e] = double(m.re[e]);
            red[1][row * E + e] = double(m.im[e]);
        }
    }
    __syncthreads();
    if (threadIdx.x < uint32_t(E)) {
        double sr = 0.0, si = 0.0;
        for (uint32_t q = 0; q < nrows; ++q) {
            sr += red[0][q * E + threadIdx.x];
            si += red[1][q * E + threadIdx.x];
        }
        out[2 * threadIdx.x] = sr;
        out[2 * threadIdx.x + 1] = si;
    }
    __syncthreads();
}

// Arguments of the M accumulation of an adjoint round (mslot < 0: none).
struct MArgs {
    int mslot = -1;
    int mpos = 0;
    double (*red)[kSB] = nullptr;
    double* partial = nullptr;
    uint32_t blk = 0;
};

// One round on the tiles t[0 .. NT) (the adjoint runs psi and lam together).
// The common round shapes (one U on position 0 or 1, two U on positions 0 and
// 1, one PHASE, permutations only) run straight from the LDS loads to the LDS stores
// (no op dispatch while the sub-tile is live in registers, so no register
// copies where dispatch paths meet); any other round goes through round_ops.
template <typename T, int D, int M, int NT, bool MACC = false>
__device__ __forceinline__ void run_round(cplx<T>* const (&t)[NT], const StageGeom& g, const uint32_t* offhi,
                                          uint32_t base, const RoundDesc& rd, const StageOp* __restrict__ ops,
                                          const cplx<T>* __restrict__ mats, const SubDigits& dig0,
                                          const MArgs& ma = MArgs{}) {
    constexpr int DM = cpow(D, M);
    constexpr uint32_t ESZ = uint32_t(sizeof(cplx<T>));
    MAcc<T, D> macc;
    if constexpr (MACC) {
#pragma unroll
        for (int e = 0; e < D * D; ++e) macc.re[e] = macc.im[e] = T(0);
    }
    const uint32_t nsub = g.TE / DM;
    // LDS byte addresses: tile 0's base goes into each sub-tile base; the
    // other tile is a uniform distance away
    const uint32_t lb0 = lds_addr(t[0]);
    uint32_t dt[NT];
#pragma unroll
    for (int x = 0; x < NT; ++x) dt[x] = x == 0 ? 0u : lds_addr(t[x]) - lb0;
    const int kind = rd.kind;
    // U shapes: the matrices of position 0 (or the one U) and position 1
    const cplx<T>* U0 = mats + rd.mat0;
    const cplx<T>* U1 = mats + rd.mat1;
    if constexpr (NT == 1 && M == 2) {
        if (rd.pre2 >= 0) {
            // a pair round with pre2 (forward lists, one sub-tile per lane):
            // its loads read other lanes' sub-tiles, so every lane loads and
            // multiplies before any lane stores
            const bool act = threadIdx.x < nsub;
            cplx<T> v[DM];
            uint32_t tb = 0, gidx0 = 0;
            if (act) {
                tb = sub_base<D>(dig0, rd);
                gidx0 = rd.need_gidx ? global_index(g, offhi, base, tb) : 0u;
                uint32_t al[DM];
                load_addrs<D, M>(al, lb0 + tb * ESZ, rd, gidx0);
                add_pre2<D, M>(al, rd, dig0);
#pragma unroll
                for (int i = 0; i < DM; ++i) v[i] = lds_ld<T>(al[i]);
                r_u<T, D, M, 0, false>(v, U0);
                asm volatile("" ::: "memory");
                r_u<T, D, M, 1, false>(v, U1);
            }
            __syncthreads();
            if (act) {
                uint32_t as[DM];
                store_addrs<D, M>(as, lb0 + tb * ESZ, rd, gidx0);
#pragma unroll
                for (int i = 0; i < DM; ++i) lds_st<T>(as[i], v[i]);
            }
            return;
        }
    }
    for (uint32_t u = threadIdx.x; u < nsub; u += blockDim.x) {
        const uint32_t tb = sub_base<D>(u == threadIdx.x ? dig0 : sub_digits<D>(u, rd.nother), rd);
        const uint32_t gidx0 = rd.need_gidx ? global_index(g, offhi, base, tb) : 0u;
        uint32_t al[DM];
        load_addrs<D, M>(al, lb0 + tb * ESZ, rd, gidx0);
        // the tiles one after the other (one sub-tile live at a time)
#pragma unroll
        for (int x = 0; x < NT; ++x) {
            cplx<T> v[DM];
#pragma unroll
            for (int i = 0; i < DM; ++i) v[i] = lds_ld<T>(al[i] + dt[x]);
            if constexpr (MACC && NT == 2) {
                if (x == 0 && ma.mslot >= 0) {
                    cplx<T> w[DM];
#pragma unroll
                    for (int i = 0; i < DM; ++i) w[i] = lds_ld<T>(al[i] + dt[1]);
                    if (ma.mpos == 0) {
                        macc_add<T, D, M, 0>(macc, v, w);
                    } else {
                        if constexpr (M >= 2) macc_add<T, D, M, 1>(macc, v, w);
                    }
                }
            }
            // each shape stores from its own branch
            auto store = [&]() {
                uint32_t as[DM];
                store_addrs<D, M>(as, lb0 + tb * ESZ, rd, gidx0);
#pragma unroll
                for (int i = 0; i < DM; ++i) lds_st<T>(as[i] + dt[x], v[i]);
            };
            if (kind == RK_U0) {
                r_u<T, D, M, 0, false>(v, U0);
                store();
            } else if (kind == RK_U01) {
                if constexpr (M >= 2) {
                    r_u<T, D, M, 0, false>(v, U0);
                    // keep the second matrix's loads after the first product
                    // (hoisting them would hold both matrices in registers)
                    asm volatile("" ::: "memory");
                    r_u<T, D, M, 1, false>(v, U1);
                }
                store();
            } else if (kind == RK_U0_REAL) {
                r_u<T, D, M, 0, true>(v, U0);
                store();
            } else if (kind == RK_U1) {
                if constexpr (M >= 2) r_u<T, D, M, 1, false>(v, U0);
                store();
            } else if (kind == RK_U1_REAL) {
                if constexpr (M >= 2) r_u<T, D, M, 1, true>(v, U0);
                store();
            } else if (kind == RK_PHASE) {
                r_phase<T, D, M>(v, ops[rd.op0], mats, gidx0);
                store();
            } else if (kind == RK_NONE) {
                store();
            } else {
                // generic rounds exist only for groups of 3 or more qudits
                if constexpr (M >= 3) round_ops<T, D, M>(v, rd, ops, mats, gidx0);
                store();
            }
        }
    }
    if constexpr (MACC) {
        if (ma.mslot >= 0)
            mreduce_block<T, D>(macc, ma.red, ma.partial + (size_t(ma.mslot) * gridDim.x + ma.blk) * (D * D) * 2);
    }
}

template <typename T, int D, int M>
__device__ __forceinline__ void stage_rounds(cplx<T>* __restrict__ psi, const StageGeom& g,
                                             const RoundDesc* __restrict__ rounds, int nrounds,
                                             const StageOp* __restrict__ ops, const cplx<T>* __restrict__ mats,
                                             size_t mat_stride) {
    const uint32_t blk = tile_of_block(g);
    mats += size_t(blk / g.ntiles) * mat_stride;
    extern __shared__ unsigned char smem[];
    cplx<T>* tile = reinterpret_cast<cplx<T>*>(smem);
    uint32_t* offhi = reinterpret_cast<uint32_t*>(tile + g.TE);
    const uint32_t base = tile_base<D>(g, blk);
    build_offhi<D>(g, offhi);
    __syncthreads();
    tile_load(psi, tile, g, offhi, base);
    __syncthreads();
    const SubDigits dig0 = sub_digits<D>(threadIdx.x, nrounds > 0 ? rounds[0].nother : 0);
    cplx<T>* const tl[1] = {tile};
    for (int ri = 0; ri < nrounds; ++ri) {
        run_round<T, D, M, 1>(tl, g, offhi, base, rounds[ri], ops, mats, dig0);
        __syncthreads();
    }
    tile_store(psi, tile, g, offhi, base);
}

template <typename T, int D, int M>
__global__ __launch_bounds__(kSB) void k_stage_rounds(cplx<T>* __restrict__ psi, StageGeom g,
                                                      const RoundDesc* __restrict__ rounds, int nrounds,
                                                      const StageOp* __restrict__ ops,
                                                      const cplx<T>* __restrict__ mats, size_t mat_stride) {
    stage_rounds<T, D, M>(psi, g, rounds, nrounds, ops, mats, mat_stride);
}

// The same kernel compiled for 8 waves per SIMD.  The default build of these
// instantiations holds 106 scalar registers, which caps a SIMD at 7 waves
// (800 scalar registers each); this one is held to 78 at the price of at
// most 64 bytes of spill per lane (measured 2% faster for D = 10 in
// complex64, and 4% for D = 3 groups of 2, whose pair rounds need no spill).
template <typename T, int D, int M>
__global__ __launch_bounds__(kSB) __attribute__((amdgpu_waves_per_eu(8))) void k_stage_rounds_w8(
    cplx<T>* __restrict__ psi, StageGeom g, const RoundDesc* __restrict__ rounds, int nrounds,
    const StageOp* __restrict__ ops, const cplx<T>* __restrict__ mats, size_t mat_stride) {
    stage_rounds<T, D, M>(psi, g, rounds, nrounds, ops, mats, mat_stride);
}

// Instantiations that take k_stage_rounds_w8: default occupancy below 8 and
// the 8-wave build spills at most 64 bytes per lane.
template <typename T, int D, int M>
constexpr bool rounds_w8() {
    if constexpr (sizeof(T) == 4) return M == 2 ? (D == 2 || D == 3) : (M == 1 && D >= 5 && D <= 11);
    else return M == 2 ? D == 2 : (M == 1 && D >= 3 && D <= 5);
}

// Pipelined persistent variant: a workgroup walks a strided sequence of
// tiles; the global loads of the next tile are issued into
// registers before the current tile's rounds run from LDS, so their latency
// overlaps the compute and the stores.  Runs are shorter than the workgroup
// (R < 256): lane (gr, o) handles offset o of runs gr, gr + G, ... (at most
// MAXE of them).
template <int MAXE>
struct RunPlan {
    uint32_t G, gr, o, cnt;
};

template <typename T, int MAXE>
__device__ __forceinline__ void pipe_prefetch(const cplx<T>* __restrict__ psi, const StageGeom& g, const uint32_t* offhi,
                                     uint32_t base, const RunPlan<MAXE>& rp, cplx<T> (&buf)[MAXE]) {
    // unpredicated loads (the run index is clamped; surplus values are never
    // stored) keep buf in registers
#pragma unroll
    for (int j = 0; j < MAXE; ++j) {
        const uint32_t h = min(rp.gr + uint32_t(j) * rp.G, g.nhi - 1);
        buf[j] = psi[base + offhi[h] + rp.o];
    }
}

template <typename T, int D, int M, int MAXE>
__global__ __launch_bounds__(kSB) void k_stage_pipe(cplx<T>* __restrict__ psi, StageGeom g,
                                                    const RoundDesc* __restrict__ rounds, int nrounds,
                                                    const StageOp* __restrict__ ops,
                                                    const cplx<T>* __restrict__ mats0, size_t mat_stride,
                                                    uint32_t total) {
    extern __shared__ unsigned char smem[];
    cplx<T>* tile = reinterpret_cast<cplx<T>*>(smem);
    uint32_t* offhi = reinterpret_cast<uint32_t*>(tile + g.TE);
    build_offhi<D>(g, offhi);
    RunPlan<MAXE> rp;
    rp.G = kSB / g.R;
    rp.gr = threadIdx.x / g.R;
    rp.o = threadIdx.x - rp.gr * g.R;
    rp.cnt = rp.gr < rp.G && rp.gr < g.nhi ? (g.nhi - rp.gr + rp.G - 1) / rp.G : 0;
    __syncthreads();
    cplx<T> buf[MAXE];
    // tiles of this workgroup: t, t + stride, ... below end (with g.xcd and a
    // grid that is a multiple of 8, a contiguous range per XCD)
    uint32_t t = blockIdx.x, stride = gridDim.x, end = total;
    if (g.xcd && gridDim.x % kXCD == 0) {
        const uint32_t x = blockIdx.x % kXCD;
        stride = gridDim.x / kXCD;
        t = xcd_range_start(x, total) + blockIdx.x / kXCD;
        end = xcd_range_start(x + 1, total);
    }
    if (t < end) pipe_prefetch<T, MAXE>(psi, g, offhi, tile_base<D>(g, t), rp, buf);
    const SubDigits dig0 = sub_digits<D>(threadIdx.x, nrounds > 0 ? rounds[0].nother : 0);
    cplx<T>* const tl[1] = {tile};
    for (; t < end; t += stride) {
        const uint32_t base = tile_base<D>(g, t);
        const cplx<T>* mats = mats0 + size_t(t / g.ntiles) * mat_stride;
        lds_barrier();  // the previous tile's stores have read LDS
        // clamped like the loads: a surplus register rewrites the last run's
        // element with the value it already holds
#pragma unroll
        for (int j = 0; j < MAXE; ++j) tile[min(rp.gr + uint32_t(j) * rp.G, g.nhi - 1) * g.R + rp.o] = buf[j];
        lds_barrier();
        const uint32_t nxt = t + stride;
        if (nxt < end) pipe_prefetch<T, MAXE>(psi, g, offhi, tile_base<D>(g, nxt), rp, buf);
        for (int ri = 0; ri < nrounds; ++ri) {
            run_round<T, D, M, 1>(tl, g, offhi, base, rounds[ri], ops, mats, dig0);
            lds_barrier();
        }
        // store this tile
        if (rp.gr < rp.G)
            for (uint32_t h = rp.gr; h < g.nhi; h += rp.G) psi[base + offhi[h] + rp.o] = tile[h * g.R + rp.o];
    }
}

// M = sum over the tile's fibres along the op's qudit of psi_f lam_f^dagger,
// from the LDS tiles, into partial[(slot * nblocks + block) * D*D] (complex
// FP64).  Lane (block, part) sums a B x B block of entries (B = 2 for even
// D >= 4: two psi and two lam reads feed four products) over the fibres
// part, part + P, ... in the state's precision; the parts are then added in
// FP64 in a fixed order.
template <typename T, int D>
__device__ inline void tile_m(const cplx<T>* tp, const cplx<T>* tl, const StageGeom& g, const StageOp& op,
                              uint32_t blk, double (*red)[kSB], double* __restrict__ partial) {
    constexpr uint32_t E = D * D;
    constexpr int B = (D % 2 == 0 && D >= 4) ? 2 : 1;
    constexpr uint32_t NBR = D / B, NB = NBR * NBR;
    const uint32_t nt = blockDim.x;
    const uint32_t nf = g.TE / D;
    double* out = partial + (size_t(op.slot) * gridDim.x + blk) * E * 2;
    auto block_sum = [&](uint32_t bi, uint32_t f0, uint32_t step, T (&ar)[B * B], T (&ai)[B * B]) {
        const uint32_t a0 = (bi / NBR) * B, c0 = (bi % NBR) * B;
#pragma unroll
        for (int j = 0; j < B * B; ++j) ar[j] = ai[j] = T(0);
        for (uint32_t f = f0; f < nf; f += step) {
            const uint32_t lb = fibre_lb<D>(op, f);
            cplx<T> x[B], y[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                x[i] = tp[lb + (a0 + i) * op.ls];
                y[i] = tl[lb + (c0 + i) * op.ls];
            }
#pragma unroll
            for (int i = 0; i < B; ++i)
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    ar[i * B + j] = fma(x[i].re, y[j].re, fma(x[i].im, y[j].im, ar[i * B + j]));
                    ai[i * B + j] = fma(x[i].im, y[j].re, fma(-x[i].re, y[j].im, ai[i * B + j]));
                }
        }
    };
    auto entry = [&](uint32_t bi, int j) { return ((bi / NBR) * B + j / B) * D + (bi % NBR) * B + j % B; };
    if (nt >= NB) {
        const uint32_t P = nt / NB;
        const uint32_t bi = threadIdx.x % NB, part = threadIdx.x / NB;
        T ar[B * B], ai[B * B];
        block_sum(bi, part, P, ar, ai);
        for (uint32_t q = 0; q < P; ++q) {
            if (part == q) {
#pragma unroll
                for (int j = 0; j < B * B; ++j) {
                    const uint32_t e = entry(bi, j);
                    red[0][e] = (q ? red[0][e] : 0.0) + double(ar[j]);
                    red[1][e] = (q ? red[1][e] : 0.0) + double(ai[j]);
                }
            }
            __syncthreads();
        }
        for (uint32_t e = threadIdx.x; e < E; e += nt) {
            out[2 * e] = red[0][e];
            out[2 * e + 1] = red[1][e];
        }
    } else {
        for (uint32_t bi = threadIdx.x; bi < NB; bi += nt) {
            T ar[B * B], ai[B * B];
            block_sum(bi, 0, 1, ar, ai);
#pragma unroll
            for (int j = 0; j < B * B; ++j) {
                out[2 * entry(bi, j)] = double(ar[j]);
                out[2 * entry(bi, j) + 1] = double(ai[j]);
            }
        }
    }
    __syncthreads();
}

// Reverse stage in register rounds on psi and lam.  A U that owns an M slot
// always opens its round, so its M is taken from the LDS tiles before the
// round's ops run in registers.
template <typename T, int D, int M>
__global__ __launch_bounds__(kSB) void k_stage_adj_rounds(cplx<T>* __restrict__ psi, cplx<T>* __restrict__ lam,
                                                          StageGeom g, const RoundDesc* __restrict__ rounds,
                                                          int nrounds, const StageOp* __restrict__ ops,
                                                          const cplx<T>* __restrict__ mats, size_t mat_stride,
                                                          double* __restrict__ partial) {
    const uint32_t blk = tile_of_block(g);
    mats += size_t(blk / g.ntiles) * mat_stride;
    extern __shared__ unsigned char smem[];
    cplx<T>* tp = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* tl = tp + g.TE;
    uint32_t* offhi = reinterpret_cast<uint32_t*>(tl + g.TE);
    __shared__ double red[2][kSB];
    const uint32_t base = tile_base<D>(g, blk);
    build_offhi<D>(g, offhi);
    __syncthreads();
    tile_load(psi, tp, g, offhi, base);
    tile_load(lam, tl, g, offhi, base);
    __syncthreads();
    const SubDigits dig0 = sub_digits<D>(threadIdx.x, nrounds > 0 ? rounds[0].nother : 0);
    cplx<T>* const tt[2] = {tp, tl};
    for (int ri = 0; ri < nrounds; ++ri) {
        const RoundDesc& rd = rounds[ri];
        // a slotted U opens its round (never after a leading permutation)
        MArgs ma;
        ma.mslot = rd.mslot;
        ma.mpos = rd.mpos;
        if constexpr (D <= 4) {
            // M from the registers of the round
            ma.red = red;
            ma.partial = partial;
            ma.blk = blk;
            run_round<T, D, M, 2, true>(tt, g, offhi, base, rd, ops, mats, dig0, ma);
        } else {
            if (ma.mslot >= 0) tile_m<T, D>(tp, tl, g, ops[rd.op0], blk, red, partial);
            run_round<T, D, M, 2>(tt, g, offhi, base, rd, ops, mats, dig0);
        }
        __syncthreads();
    }
    tile_store(psi, tp, g, offhi, base);
    tile_store(lam, tl, g, offhi, base);
}

template <class F>
qf_status with_dim_s(uint32_t D, F&& f) {
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

// Dynamic LDS of a stage workgroup: the tile(s), then the nhi run offsets.
size_t stage_lds_bytes(const StageGeom& g, int dtype, bool adjoint) {
    const size_t esz = dtype == QF_C64 ? 8 : 16;
    return size_t(g.TE) * esz * (adjoint ? 2 : 1) + size_t(g.nhi) * sizeof(uint32_t);
}

qf_status launch_stage(const StateView& s, const StageGeom& g, const StageOp* dops, int nops, const void* dmats,
                       hipStream_t st, size_t mat_stride) {
    const uint32_t grid = g.ntiles * s.batch;
    const size_t lds = stage_lds_bytes(g, s.dtype, false);
    return with_dim_s(s.D, [&](auto dtag) -> qf_status {
        constexpr int D = decltype(dtag)::value;
        if (s.dtype == QF_C64)
            hipLaunchKernelGGL((k_stage<float, D>), dim3(grid), dim3(kSB), lds, st,
                               reinterpret_cast<cplx<float>*>(s.amps), g, dops, nops,
                               reinterpret_cast<const cplx<float>*>(dmats), mat_stride);
        else
            hipLaunchKernelGGL((k_stage<double, D>), dim3(grid), dim3(kSB), lds, st,
                               reinterpret_cast<cplx<double>*>(s.amps), g, dops, nops,
                               reinterpret_cast<const cplx<double>*>(dmats), mat_stride);
        return check_launch("stage");
    });
}

// Register group sizes compiled per D (D^M <= 32 amplitudes per lane).
int max_group_size(uint32_t D) { return D == 2 ? 5 : D == 3 ? 3 : D <= 5 ? 2 : 1; }

// Workgroup size of a register-round stage: the sub-tile count rounded up to
// whole wavefronts, at most 256 (small sub-tile counts then leave no lanes idle
// in the rounds and allow more resident workgroups).
static uint32_t rounds_threads(const StageGeom& g, int DM) {
    const uint32_t nsub = g.TE / uint32_t(DM);
    uint32_t t = (nsub + 63) / 64 * 64;
    return t < 64 ? 64 : t > uint32_t(kSB) ? uint32_t(kSB) : t;
}

template <typename T, int D, int M>
static qf_status launch_rounds_m(const StateView& s, const StageGeom& g, const RoundDesc* drounds, int nrounds,
                                 const StageOp* dops, const void* dmats, size_t mat_stride, hipStream_t st) {
    const uint32_t grid = g.ntiles * s.batch;
    const size_t lds = stage_lds_bytes(g, s.dtype, false);
    const uint32_t nthr = rounds_threads(g, cpow(D, M));
    if constexpr (rounds_w8<T, D, M>())
        hipLaunchKernelGGL((k_stage_rounds_w8<T, D, M>), dim3(grid), dim3(nthr), lds, st,
                           reinterpret_cast<cplx<T>*>(s.amps), g, drounds, nrounds, dops,
                           reinterpret_cast<const cplx<T>*>(dmats), mat_stride);
    else
        hipLaunchKernelGGL((k_stage_rounds<T, D, M>), dim3(grid), dim3(nthr), lds, st,
                           reinterpret_cast<cplx<T>*>(s.amps), g, drounds, nrounds, dops,
                           reinterpret_cast<const cplx<T>*>(dmats), mat_stride);
    return check_launch("stage rounds");
}

template <typename T, int D, int M>
static qf_status launch_pipe_m(const StateView& s, const StageGeom& g, const RoundDesc* drounds, int nrounds,
                               const StageOp* dops, const void* dmats, size_t mat_stride, int wgs_per_cu,
                               hipStream_t st) {
    const uint32_t total = g.ntiles * s.batch;
    const size_t lds = stage_lds_bytes(g, s.dtype, false);
    const uint32_t G = kSB / g.R;
    const uint32_t per = (g.nhi + G - 1) / G;
    // never more workgroups per CU than can be resident at once: a persistent
    // workgroup that waits for a slot only starts after others have finished
    auto kern = per <= 8 ? (const void*)k_stage_pipe<T, D, M, 8>
                         : per <= 16 ? (const void*)k_stage_pipe<T, D, M, 16> : (const void*)k_stage_pipe<T, D, M, 32>;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kSB, lds) != hipSuccess || occ < 1) occ = 1;
    int ncu = 256;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 256;
    }
    const uint32_t cap = uint32_t(ncu) * uint32_t(std::min(wgs_per_cu, occ));
    const uint32_t grid = total < cap ? total : cap;
    if (per <= 8)
        hipLaunchKernelGGL((k_stage_pipe<T, D, M, 8>), dim3(grid), dim3(kSB), lds, st,
                           reinterpret_cast<cplx<T>*>(s.amps), g, drounds, nrounds, dops,
                           reinterpret_cast<const cplx<T>*>(dmats), mat_stride, total);
    else if (per <= 16)
        hipLaunchKernelGGL((k_stage_pipe<T, D, M, 16>), dim3(grid), dim3(kSB), lds, st,
                           reinterpret_cast<cplx<T>*>(s.amps), g, drounds, nrounds, dops,
                           reinterpret_cast<const cplx<T>*>(dmats), mat_stride, total);
    else
        hipLaunchKernelGGL((k_stage_pipe<T, D, M, 32>), dim3(grid), dim3(kSB), lds, st,
                           reinterpret_cast<cplx<T>*>(s.amps), g, drounds, nrounds, dops,
                           reinterpret_cast<const cplx<T>*>(dmats), mat_stride, total);
    return check_launch("stage (pipelined)");
}

bool stage_pipe_ok(const StageGeom& g) {
    if (g.R >= uint32_t(kSB)) return false;
    const uint32_t G = kSB / g.R;
    return (g.nhi + G - 1) / G <= 32;
}

qf_status launch_stage_pipe(const StateView& s, int M, const StageGeom& g, const RoundDesc* drounds, int nrounds,
                            const StageOp* dops, const void* dmats, int wgs_per_cu, hipStream_t st,
                            size_t mat_stride) {
    return with_dim_s(s.D, [&](auto dtag) -> qf_status {
        constexpr int D = decltype(dtag)::value;
        auto go = [&](auto tag) -> qf_status {
            using T = decltype(tag);
            if constexpr (D > 12) {
                return set_error(QF_EUNSUPPORTED, "pipelined stage for D = %d", D);
            } else {
            switch (M) {
                case 1: return launch_pipe_m<T, D, 1>(s, g, drounds, nrounds, dops, dmats, mat_stride, wgs_per_cu, st);
                case 2:
                    if constexpr (D <= 5)
                        return launch_pipe_m<T, D, 2>(s, g, drounds, nrounds, dops, dmats, mat_stride, wgs_per_cu, st);
                    break;
                case 3:
                    if constexpr (D <= 3)
                        return launch_pipe_m<T, D, 3>(s, g, drounds, nrounds, dops, dmats, mat_stride, wgs_per_cu, st);
                    break;
            }
            return set_error(QF_EUNSUPPORTED, "pipelined stage with a group of %d qudits for D = %d", M, D);
            }
        };
        if (s.dtype != QF_C64) return set_error(QF_EUNSUPPORTED, "the pipelined stage runs complex64 only");
        return go(float{});
    });
}

qf_status launch_stage_rounds(const StateView& s, int M, const StageGeom& g, const RoundDesc* drounds, int nrounds,
                              const StageOp* dops, const void* dmats, hipStream_t st, size_t mat_stride) {
    return with_dim_s(s.D, [&](auto dtag) -> qf_status {
        constexpr int D = decltype(dtag)::value;
        auto go = [&](auto tag) -> qf_status {
            using T = decltype(tag);
            switch (M) {
                case 1: return launch_rounds_m<T, D, 1>(s, g, drounds, nrounds, dops, dmats, mat_stride, st);
                case 2: if constexpr (D <= 5) return launch_rounds_m<T, D, 2>(s, g, drounds, nrounds, dops, dmats, mat_stride, st);
                        break;
                case 3: if constexpr (D <= 3) return launch_rounds_m<T, D, 3>(s, g, drounds, nrounds, dops, dmats, mat_stride, st);
                        break;
                case 4: if constexpr (D <= 2) return launch_rounds_m<T, D, 4>(s, g, drounds, nrounds, dops, dmats, mat_stride, st);
                        break;
                case 5: if constexpr (D <= 2) return launch_rounds_m<T, D, 5>(s, g, drounds, nrounds, dops, dmats, mat_stride, st);
                        break;
            }
            return set_error(QF_EUNSUPPORTED, "register group of %d qudits for D = %d", M, D);
        };
        return s.dtype == QF_C64 ? go(float{}) : go(double{});
    });
}

template <typename T, int D, int M>
static qf_status launch_adj_rounds_m(const StateView& s, void* lam, const StageGeom& g, const RoundDesc* drounds,
                                     int nrounds, const StageOp* dops, const void* dmats, double* partial,
                                     size_t mat_stride, hipStream_t st) {
    const uint32_t grid = g.ntiles * s.batch;
    const size_t lds = stage_lds_bytes(g, s.dtype, true);
    const uint32_t nthr = rounds_threads(g, cpow(D, M));
    hipLaunchKernelGGL((k_stage_adj_rounds<T, D, M>), dim3(grid), dim3(nthr), lds, st,
                       reinterpret_cast<cplx<T>*>(s.amps), reinterpret_cast<cplx<T>*>(lam), g, drounds, nrounds, dops,
                       reinterpret_cast<const cplx<T>*>(dmats), mat_stride, partial);
    return check_launch("stage adjoint rounds");
}

qf_status launch_stage_adj_rounds(const StateView& s, void* lam, int M, const StageGeom& g, const RoundDesc* drounds,
                                  int nrounds, const StageOp* dops, const void* dmats, double* partial, hipStream_t st,
                                  size_t mat_stride) {
    return with_dim_s(s.D, [&](auto dtag) -> qf_status {
        constexpr int D = decltype(dtag)::value;
        auto go = [&](auto tag) -> qf_status {
            using T = decltype(tag);
            switch (M) {
                case 1:
                    return launch_adj_rounds_m<T, D, 1>(s, lam, g, drounds, nrounds, dops, dmats, partial, mat_stride,
                                                        st);
                case 2:
                    if constexpr (D <= 5 && (sizeof(T) == 4 || D <= 3))
                        return launch_adj_rounds_m<T, D, 2>(s, lam, g, drounds, nrounds, dops, dmats, partial,
                                                            mat_stride, st);
                    break;
            }
            return set_error(QF_EUNSUPPORTED, "adjoint register group of %d qudits for D = %d", M, D);
        };
        return s.dtype == QF_C64 ? go(float{}) : go(double{});
    });
}

qf_status launch_stage_adj(const StateView& s, void* lam, const StageGeom& g, const StageOp* dops, int nops,
                           const void* dmats, double* partial, hipStream_t st, size_t mat_stride) {
    const uint32_t grid = g.ntiles * s.batch;
    const size_t lds = stage_lds_bytes(g, s.dtype, true);
    return with_dim_s(s.D, [&](auto dtag) -> qf_status {
        constexpr int D = decltype(dtag)::value;
        if (s.dtype == QF_C64)
            hipLaunchKernelGGL((k_stage_adj<float, D>), dim3(grid), dim3(kSB), lds, st,
                               reinterpret_cast<cplx<float>*>(s.amps), reinterpret_cast<cplx<float>*>(lam), g, dops,
                               nops, reinterpret_cast<const cplx<float>*>(dmats), mat_stride, partial);
        else
            hipLaunchKernelGGL((k_stage_adj<double, D>), dim3(grid), dim3(kSB), lds, st,
                               reinterpret_cast<cplx<double>*>(s.amps), reinterpret_cast<cplx<double>*>(lam), g, dops,
                               nops, reinterpret_cast<const cplx<double>*>(dmats), mat_stride, partial);
        return check_launch("stage adjoint");
    });
}

qf_status launch_stage_mreduce(const double* partial, uint32_t nslots, uint32_t ntiles, uint32_t batch, uint32_t E,
                               double* mout, uint32_t nslots_total, uint32_t slot0, hipStream_t st) {
    if (nslots == 0) return QF_OK;
    hipLaunchKernelGGL(k_stage_mreduce, dim3(batch * nslots * E), dim3(kSB), 0, st, partial, nslots, ntiles, batch,
                       E, mout, nslots_total, slot0);
    return check_launch("stage M reduce");
}

}  // namespace qf
