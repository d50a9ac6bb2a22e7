// Interfaces between the C-ABI layer (abi.cpp, plan.cpp) and the kernel
// launchers (*.hip).  Everything here is host code; arguments are validated by
// the caller.
#pragma once

#include <vector>

#include "qf_common.h"

namespace qf {

constexpr int kMaxDim = 16;

// A validated view of a qf_state.
struct StateView {
    void* amps;
    uint32_t n;
    uint32_t D;
    uint32_t N;       // D^n
    uint32_t batch;
    uint32_t total;   // batch * N  (< 2^32)
    int dtype;        // QF_C64 / QF_C128
};

inline uint32_t ipow(uint32_t b, uint32_t e) {
    uint32_t r = 1;
    while (e--) r *= b;
    return r;
}

// ---- per-gate launchers (k_basic.hip) ----
qf_status launch_init(const StateView& s, const std::vector<uint32_t>& index, hipStream_t st);
qf_status launch_apply_1q(const StateView& s, int q, const double* U, hipStream_t st);
qf_status launch_ctrl(const StateView& s, int ctrl, int tgt, const int32_t* shift, hipStream_t st);
qf_status launch_diag(const StateView& s, int k, const int32_t* qudits, const double* phases,
                      hipStream_t st);
qf_status launch_probs_full(const StateView& s, void* out, hipStream_t st);
qf_status launch_probs_marginal(const StateView& s, int m, const int32_t* qudits, void* out,
                                hipStream_t st);
// table: per active qudit D complex values (combined terms), active: qudit list
qf_status launch_expect(const StateView& s, const std::vector<int>& active,
                        const std::vector<double>& table, double* out, hipStream_t st);
// Elementwise lam = f(x) * psi with f(x) = sum over active qudits of the real
// table value (the Hermitian part of a diagonal observable).
qf_status launch_diag_observable(const StateView& psi, void* lam_amps, const std::vector<int>& active,
                                 const std::vector<double>& table_re, hipStream_t st);

// ---- fused dense blocks (k_fused.hip) ----
qf_status launch_fused(const StateView& s, int k, int q0, const void* B, hipStream_t st);

}  // namespace qf
