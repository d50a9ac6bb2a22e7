// Measurement shots (the histogram of the paper's measure(..., shots),
// section "Code style") by inversion of the cumulative distribution:
//   1. probabilities of the measured qudits in FP64 (full register or marginal),
//   2. an inclusive prefix sum per register in FP64, in a fixed order
//      (segmented block scans, recursively over the block totals; above 4096
//      outcomes the block offsets are not added to the elements: a search
//      finds the block on an array of block ends, then the element, adding
//      its block's offset as it compares),
//   3. one lane per shot: the first bin whose cumulative sum exceeds
//      u * total (a draw whose product reaches the total goes to the last
//      bin of non-zero probability), counted with integer atomics (an exact,
//      order-independent histogram); up to 4096 outcomes per register the
//      counts first go to a workgroup histogram in LDS, flushed once per
//      workgroup, so that many shots on few outcomes do not serialise on a
//      few global counters.
// The uniforms u are inputs: the caller draws them.
#include <algorithm>
#include <type_traits>

#include "qf_internal.h"

namespace qf {
namespace {

constexpr int kT = 256;         // threads per scan block
constexpr int kPer = 4;         // elements per thread
constexpr int kSpan = kT * kPer;  // elements per scan block
constexpr int kSub = 32;           // elements per sub-block (the searches' middle level)
constexpr int kMid = kSpan / kSub; // sub-blocks per scan block

// Inclusive scan of segments of length seg (a segment never shares a block with
// another): block blk covers elements [s * seg + lb * kSpan, ...) of segment
// s = blk / bps, lb = blk % bps.  Each thread sums its kPer elements in order,
// the thread totals are scanned within each wavefront by lane shifts (six
// doubling steps), the four wavefront totals are added in order through LDS
// (one barrier), and the block total goes to sums[blk] (sums are laid out as
// [segment][bps]).  Full blocks whose source and destination are 16-byte
// aligned move their elements with 16-byte loads and stores.
// Src = double: scan data in place; Src = cplx<float> / cplx<double>: the
// values are |psi_x|^2 of the state src (taken in FP64), written scanned to data.
template <typename Src>
__device__ inline double scan_value(const Src* p, uint64_t e) {
    if constexpr (std::is_same<Src, double>::value) {
        return p[e];
    } else {
        const Src v = p[e];
        return double(v.re) * double(v.re) + double(v.im) * double(v.im);
    }
}

__device__ inline double sq2(float a, float b) { return double(a) * double(a) + double(b) * double(b); }

// A thread's kPer values of a full block, 16 bytes per load where the element
// is narrower than that.
template <typename Src>
__device__ inline void scan_values_vec(const Src* q, double (&x)[kPer]) {
    static_assert(kPer % 2 == 0, "pairs of elements per 16-byte load");
    if constexpr (std::is_same<Src, double>::value) {
        const double2* p = reinterpret_cast<const double2*>(q);
#pragma unroll
        for (int i = 0; i < kPer / 2; ++i) {
            const double2 a = p[i];
            x[2 * i] = a.x;
            x[2 * i + 1] = a.y;
        }
    } else if constexpr (sizeof(Src) == 8) {
        const float4* p = reinterpret_cast<const float4*>(q);
#pragma unroll
        for (int i = 0; i < kPer / 2; ++i) {
            const float4 a = p[i];
            x[2 * i] = sq2(a.x, a.y);
            x[2 * i + 1] = sq2(a.z, a.w);
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i) x[i] = scan_value(q, uint64_t(i));
    }
}

// With mids (the first level of a block-local scan), the local sum at the end
// of each kSub-element sub-block (the block's last element ending the last
// one) also goes to mids[blk * kMid + sub-block].
template <typename Src>
__global__ __launch_bounds__(kT) void k_scan_block(const Src* __restrict__ src, double* __restrict__ data,
                                                   uint64_t seg, uint32_t bps, double* __restrict__ sums,
                                                   double* __restrict__ mids) {
    constexpr int kW = kT / 64;
    __shared__ double wt[kW];
    const uint32_t blk = blockIdx.x;
    const uint32_t s = blk / bps, lb = blk - s * bps;
    const uint64_t lo = uint64_t(lb) * kSpan;
    const uint64_t n = seg - lo < uint64_t(kSpan) ? seg - lo : uint64_t(kSpan);
    const Src* q = src + s * seg + lo;
    double* d = data + s * seg + lo;
    const bool vec = n == uint64_t(kSpan) &&
                     ((reinterpret_cast<uintptr_t>(q) | reinterpret_cast<uintptr_t>(d)) & 15u) == 0;
    double v[kPer];
    if (vec) {
        scan_values_vec<Src>(q + size_t(threadIdx.x) * kPer, v);
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const uint64_t e = uint64_t(threadIdx.x) * kPer + i;
            v[i] = e < n ? scan_value(q, e) : 0.0;
        }
    }
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        run += v[i];
        v[i] = run;
    }
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    double incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(incl, off, 64);
        if (lane >= uint32_t(off)) incl += y;
    }
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 0.0;
    if (lane == 63) wt[wv] = incl;
    __syncthreads();
    double wpre = 0.0;
    for (uint32_t w = 0; w < wv; ++w) wpre += wt[w];
    const double before = wpre + excl;
    if (vec) {
        double2* p = reinterpret_cast<double2*>(d + size_t(threadIdx.x) * kPer);
#pragma unroll
        for (int i = 0; i < kPer / 2; ++i) p[i] = make_double2(before + v[2 * i], before + v[2 * i + 1]);
        // a full block: sub-block t ends at element t * kSub + kSub - 1, the
        // last of lane t * (kSub / kPer) + kSub / kPer - 1
        if (mids && (threadIdx.x % (kSub / kPer)) == kSub / kPer - 1)
            mids[size_t(blk) * kMid + threadIdx.x / (kSub / kPer)] = before + v[kPer - 1];
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const uint64_t e = uint64_t(threadIdx.x) * kPer + i;
            if (e < n) {
                d[e] = before + v[i];
                if (mids && (e % kSub == kSub - 1 || e == n - 1)) mids[size_t(blk) * kMid + e / kSub] = before + v[i];
            }
        }
    }
    if (threadIdx.x == kT - 1) sums[blk] = wpre + incl;
}

// data[s * seg + lb * kSpan + e] += (scanned block totals)[s][lb - 1] for lb >= 1.
__global__ __launch_bounds__(kT) void k_scan_add(double* __restrict__ data, uint64_t seg, uint32_t bps,
                                                 const double* __restrict__ sums) {
    const uint32_t blk = blockIdx.x;
    const uint32_t s = blk / bps, lb = blk - s * bps;
    if (lb == 0) return;
    const uint64_t lo = uint64_t(lb) * kSpan;
    const uint64_t n = seg - lo < uint64_t(kSpan) ? seg - lo : uint64_t(kSpan);
    const double off = sums[uint64_t(s) * bps + lb - 1];
    double* d = data + s * seg + lo;
    for (uint64_t e = threadIdx.x; e < n; e += kT) d[e] += off;
}

__global__ __launch_bounds__(kT) void k_fill_u64(unsigned long long* __restrict__ p, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kT) p[i] = 0ull;
}

// First index of c[0..K) with c[idx] > x, or K if none.
__device__ inline uint32_t upper_bound(const double* c, uint32_t K, double x) {
    uint32_t lo = 0, hi = K;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (c[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// First index of c[0..K) with c[idx] >= x.
__device__ inline uint32_t lower_bound(const double* c, uint32_t K, double x) {
    uint32_t lo = 0, hi = K;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (c[mid] >= x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Registers scanned without the last offset pass (more than kLdsBins outcomes):
// the cumulative sum at x in scan block lb is off(lb) + local(x), off(lb) the
// scanned block totals before lb (the same FP64 sum the offset pass forms).
// ends[lb] = off(lb) + local(last element of lb), a short array the first
// search runs on.
__global__ __launch_bounds__(kT) void k_block_ends(const double* __restrict__ local, uint64_t seg, uint32_t bps,
                                                   uint64_t nseg, const double* __restrict__ sums,
                                                   double* __restrict__ ends) {
    for (uint64_t i = uint64_t(blockIdx.x) * kT + threadIdx.x; i < nseg * bps; i += uint64_t(gridDim.x) * kT) {
        const uint64_t s = i / bps, lb = i - s * bps;
        const uint64_t last = std::min<uint64_t>(seg, (lb + 1) * kSpan) - 1;
        const double off = lb > 0 ? sums[i - 1] : 0.0;
        ends[i] = off + local[s * seg + last];
    }
}

// First j of c[0..n) with off + c[j] > x (n if none); with GE, >= x.
template <bool GE>
__device__ inline uint32_t bound_off(const double* c, uint32_t n, double off, double x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        const double v = off + c[mid];
        if (GE ? v >= x : v > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// One lane per shot on block-local sums: the block first (on ends), then the
// element; counts with 64-bit integer atomics.
__global__ __launch_bounds__(kT) void k_sample_blocks(const double* __restrict__ local, uint32_t K, uint32_t bps,
                                                      const double* __restrict__ sums, const double* __restrict__ ends,
                                                      uint64_t shots, uint64_t total, const double* __restrict__ u,
                                                      unsigned long long* __restrict__ counts,
                                                      int32_t* __restrict__ samples) {
    for (uint64_t i = uint64_t(blockIdx.x) * kT + threadIdx.x; i < total; i += uint64_t(gridDim.x) * kT) {
        const uint64_t b = i / shots;
        const double* c = local + b * K;
        const double* e = ends + b * bps;
        const double* so = sums + b * bps;
        const double sum = e[bps - 1];
        const double x = u[i] * sum;
        uint32_t lb = upper_bound(e, bps, x);
        uint32_t idx = K;
        if (lb < bps) {
            const uint32_t n = std::min<uint32_t>(kSpan, K - lb * kSpan);
            idx = lb * kSpan + bound_off<false>(c + size_t(lb) * kSpan, n, lb > 0 ? so[lb - 1] : 0.0, x);
        }
        if (idx >= K) {
            // the draw reached the total: the first element whose sum reaches it
            lb = lower_bound(e, bps, sum);
            const uint32_t n = std::min<uint32_t>(kSpan, K - lb * kSpan);
            idx = lb * kSpan + bound_off<true>(c + size_t(lb) * kSpan, n, lb > 0 ? so[lb - 1] : 0.0, sum);
        }
        atomicAdd(counts + b * K + idx, 1ull);
        if (samples) samples[i] = int32_t(idx);
    }
}

// The same draws with the first search split in two: every G-th block end
// (G = 2^gsh, at most kTop of them) sits in LDS and is searched first, then
// the G block ends of the group found.  The first end above x lies in the
// first group whose last end is above x, so the block (and the outcome) is the
// one the whole-array search finds.  Workgroup (blockIdx.x % bpr) of register
// b = blockIdx.x / bpr takes shots j = that index * kT + lane, + bpr * kT, ...
constexpr uint32_t kTop = 2048;  // 16 KB of FP64 group ends

__global__ __launch_bounds__(kT) void k_sample_blocks2(const double* __restrict__ local, uint32_t K, uint32_t bps,
                                                       uint32_t gsh, uint32_t bpr,
                                                       const double* __restrict__ sums,
                                                       const double* __restrict__ ends,
                                                       const double* __restrict__ mids, uint64_t shots,
                                                       const double* __restrict__ u,
                                                       unsigned long long* __restrict__ counts,
                                                       int32_t* __restrict__ samples) {
    __shared__ double top[kTop];
    const uint32_t b = blockIdx.x / bpr, w = blockIdx.x - b * bpr;
    const double* c = local + size_t(b) * K;
    const double* e = ends + size_t(b) * bps;
    const double* so = sums + size_t(b) * bps;
    const uint32_t G = 1u << gsh;
    const uint32_t ntop = (bps + G - 1) >> gsh;  // <= kTop (host check)
    for (uint32_t t = threadIdx.x; t < ntop; t += kT) top[t] = e[min((t + 1) << gsh, bps) - 1];
    __syncthreads();
    const double sum = e[bps - 1];
    for (uint64_t j = uint64_t(w) * kT + threadIdx.x; j < shots; j += uint64_t(bpr) * kT) {
        const uint64_t i = uint64_t(b) * shots + j;
        const double x = u[i] * sum;
        const uint32_t t = upper_bound(top, ntop, x);
        uint32_t lb = bps;
        if (t < ntop) {
            const uint32_t g0 = t << gsh;
            lb = g0 + upper_bound(e + g0, min(G, bps - g0), x);
        }
        uint32_t idx = K;
        if (lb < bps) {
            // the sub-block on the mids (one short run), then inside it
            const uint32_t n = std::min<uint32_t>(kSpan, K - lb * kSpan);
            const uint32_t nsub = (n + kSub - 1) / kSub;
            const double off = lb > 0 ? so[lb - 1] : 0.0;
            const uint32_t sb = bound_off<false>(mids + (size_t(b) * bps + lb) * kMid, nsub, off, x);
            idx = lb * kSpan + n;
            if (sb < nsub) {
                const uint32_t j0 = sb * kSub;
                idx = lb * kSpan + j0 +
                      bound_off<false>(c + size_t(lb) * kSpan + j0, std::min<uint32_t>(kSub, n - j0), off, x);
            }
        }
        if (idx >= K) {
            // the draw reached the total: the first element whose sum reaches it
            lb = lower_bound(e, bps, sum);
            const uint32_t n = std::min<uint32_t>(kSpan, K - lb * kSpan);
            idx = lb * kSpan + bound_off<true>(c + size_t(lb) * kSpan, n, lb > 0 ? so[lb - 1] : 0.0, sum);
        }
        atomicAdd(counts + size_t(b) * K + idx, 1ull);
        if (samples) samples[i] = int32_t(idx);
    }
}

constexpr uint32_t kLdsBins = 4096;  // 32 KB of 64-bit counters

// Workgroup (blockIdx.x % bpr) of register b = blockIdx.x / bpr draws shots
// i = that index, + bpr * kT, ... of the register into an LDS histogram.
__global__ __launch_bounds__(kT) void k_sample_lds(const double* __restrict__ cdf, uint32_t K, uint64_t shots,
                                                   uint32_t bpr, const double* __restrict__ u,
                                                   unsigned long long* __restrict__ counts,
                                                   int32_t* __restrict__ samples) {
    __shared__ unsigned long long h[kLdsBins];
    for (uint32_t i = threadIdx.x; i < K; i += kT) h[i] = 0ull;
    __syncthreads();
    const uint32_t b = blockIdx.x / bpr, w = blockIdx.x - b * bpr;
    const double* c = cdf + uint64_t(b) * K;
    const double sum = c[K - 1];
    for (uint64_t i = uint64_t(w) * kT + threadIdx.x; i < shots; i += uint64_t(bpr) * kT) {
        const uint64_t d = uint64_t(b) * shots + i;
        uint32_t idx = upper_bound(c, K, u[d] * sum);
        if (idx >= K) idx = lower_bound(c, K, sum);
        atomicAdd(h + idx, 1ull);
        if (samples) samples[d] = int32_t(idx);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < K; i += kT)
        if (h[i]) atomicAdd(counts + uint64_t(b) * K + i, h[i]);
}

uint32_t grid_of(uint64_t n) {
    const uint64_t g = (n + kT - 1) / kT;
    return uint32_t(g < 1 ? 1 : g > (1u << 20) ? (1u << 20) : g);
}

// In-place inclusive scan of nseg segments of length seg; ws holds the block
// totals of every level.
// The first level may read its values from src (|psi|^2 of a state) instead
// of data.
template <typename Src = double>
qf_status scan_segments(double* data, uint64_t seg, uint64_t nseg, double* ws, hipStream_t st,
                        const Src* src = nullptr, bool local_only = false, double* mids = nullptr) {
    const uint32_t bps = uint32_t((seg + kSpan - 1) / kSpan);
    const uint64_t nblk = nseg * bps;
    if (nblk >= (1ull << 31)) return set_error(QF_ERANGE, "prefix sum grid too large");
    if constexpr (std::is_same<Src, double>::value)
        hipLaunchKernelGGL(k_scan_block<double>, dim3(uint32_t(nblk)), dim3(kT), 0, st, src ? src : data, data, seg,
                           bps, ws, mids);
    else
        hipLaunchKernelGGL(k_scan_block<Src>, dim3(uint32_t(nblk)), dim3(kT), 0, st, src, data, seg, bps, ws, mids);
    QF_CHECK(check_launch("prefix sum"));
    if (bps > 1) {
        QF_CHECK(scan_segments(ws, bps, nseg, ws + nblk, st));
        // local_only: the block offsets stay in ws (scanned), data keeps block-local sums
        if (!local_only) {
            hipLaunchKernelGGL(k_scan_add, dim3(uint32_t(nblk)), dim3(kT), 0, st, data, seg, bps, ws);
            QF_CHECK(check_launch("prefix sum add"));
        }
    }
    return QF_OK;
}

// Doubles of block totals all levels of scan_segments need.
uint64_t scan_ws_doubles(uint64_t seg, uint64_t nseg) {
    uint64_t total = 0;
    while (true) {
        const uint64_t bps = (seg + kSpan - 1) / kSpan;
        total += bps * nseg;
        if (bps <= 1) break;
        seg = bps;
    }
    return total;
}

}  // namespace

qf_status launch_sample(const StateView& s, int m, const int32_t* qudits, uint64_t shots, const double* u,
                        int64_t* counts, int32_t* samples, hipStream_t st) {
    uint64_t K = s.N;
    if (m > 0) {
        K = 1;
        for (int i = 0; i < m; ++i) K *= s.dims[qudits[i]];
    }
    const uint64_t bins = K * s.batch;
    const uint64_t draws = shots * s.batch;
    QF_RETURN_IF(bins >= (1ull << 32) || draws >= (1ull << 32), QF_ERANGE, "batch * bins or batch * shots >= 2^32");
    const uint64_t wsd = scan_ws_doubles(K, s.batch);
    // more than kLdsBins outcomes: block-local sums and a block-end array
    // (bps entries per register) searched first
    const bool blocks = K > kLdsBins;
    const uint64_t bps = (K + kSpan - 1) / kSpan;
    const uint64_t nends = blocks ? bps * s.batch : 0;
    const uint64_t nmids = nends * kMid;
    double* cdf = nullptr;
    QF_CHECK(dev_malloc_async(reinterpret_cast<void**>(&cdf), (bins + wsd + nends + nmids) * sizeof(double), st,
                              "sampling"));
    double* ws = cdf + bins;
    double* ends = ws + wsd;
    double* mids = ends + nends;
    qf_status rs = QF_OK;
    if (m == 0) {
        // the full register: |psi|^2 is taken inside the first scan level
        if (s.dtype == QF_C64)
            rs = scan_segments(cdf, K, s.batch, ws, st, reinterpret_cast<const cplx<float>*>(s.amps), blocks,
                               blocks ? mids : nullptr);
        else
            rs = scan_segments(cdf, K, s.batch, ws, st, reinterpret_cast<const cplx<double>*>(s.amps), blocks,
                               blocks ? mids : nullptr);
    } else {
        rs = launch_probs_marginal(s, m, qudits, cdf, true, st);
        if (rs == QF_OK) rs = scan_segments<double>(cdf, K, s.batch, ws, st, nullptr, blocks, blocks ? mids : nullptr);
    }
    if (rs == QF_OK && blocks) {
        hipLaunchKernelGGL(k_block_ends, dim3(grid_of(nends)), dim3(kT), 0, st, cdf, K, uint32_t(bps),
                           uint64_t(s.batch), ws, ends);
        rs = check_launch("sampling block ends");
    }
    if (rs == QF_OK) {
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_of(bins)), dim3(kT), 0, st,
                           reinterpret_cast<unsigned long long*>(counts), bins);
        rs = check_launch("histogram clear");
    }
    if (rs == QF_OK && draws > 0) {
        if (K <= kLdsBins) {
            // about 16 shots per lane, at most 1024 workgroups in all
            uint64_t bpr = (shots + 16 * kT - 1) / (16 * kT);
            const uint64_t cap = std::max<uint64_t>(1, 1024 / s.batch);
            bpr = std::min(bpr, cap);
            hipLaunchKernelGGL(k_sample_lds, dim3(uint32_t(bpr * s.batch)), dim3(kT), 0, st, cdf, uint32_t(K), shots,
                               uint32_t(bpr), u, reinterpret_cast<unsigned long long*>(counts), samples);
        } else {
            // group ends in LDS: G = 2^gsh block ends per group, at most kTop groups
            uint32_t gsh = 5;
            while (((bps + (uint64_t(1) << gsh) - 1) >> gsh) > kTop) ++gsh;
            // about 4 shots per lane, at most 2048 workgroups in all
            uint64_t bpr = (shots + 4 * kT - 1) / (4 * kT);
            bpr = std::min<uint64_t>(bpr, std::max<uint64_t>(1, 2048 / s.batch));
            if (uint64_t(s.batch) * bpr < (1ull << 31) && gsh < 32) {
                hipLaunchKernelGGL(k_sample_blocks2, dim3(uint32_t(bpr * s.batch)), dim3(kT), 0, st, cdf,
                                   uint32_t(K), uint32_t(bps), gsh, uint32_t(bpr), ws, ends, mids, shots, u,
                                   reinterpret_cast<unsigned long long*>(counts), samples);
            } else {
                hipLaunchKernelGGL(k_sample_blocks, dim3(grid_of(draws)), dim3(kT), 0, st, cdf, uint32_t(K),
                                   uint32_t(bps), ws, ends, shots, draws, u,
                                   reinterpret_cast<unsigned long long*>(counts), samples);
            }
        }
        const qf_status rl = check_launch("sampling");
        if (rs == QF_OK) rs = rl;
    }
    (void)hipFreeAsync(cdf, st);
    return rs;
}

}  // namespace qf
