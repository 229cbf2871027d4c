// Internal helpers shared by the batch and serving runtimes.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace hhlsv {

// One lowered op of a batch instance (device layout).
struct BOp {
    int type;        // OP_DENSE / OP_DIAG / OP_WIDE / OP_UCRY
    int k;           // targets (UCRY: controls)
    int target;      // UCRY target
    int control;     // OP_WIDE control, -1 = none
    int contiguous;  // targets (UCRY: controls) are q[0], q[0]+1, ...
    int q[kMaxUcryControls];
    int control2;    // OP_WIDE second and third controls (a MUX: tables for
    int control3;    // control values 1..2^r-1), -1 = none
    int pad2;
    unsigned long long off;   // byte offset of the op's table in the instance's tables
};

// One instance of a batch launch: its program and buffers in device memory.
struct BInst {
    int n, ns, op_count, pad;
    const BOp *ops;
    const unsigned char *tables;
    unsigned char *state;   // HBM state (2^n amplitudes) when it does not fit in LDS
    double *out;            // [P(ancilla=1), 0, y_0.re, y_0.im, ...], 2 + 2^(ns+1) doubles
};

// LDS budget of one batch workgroup and whether an n-qubit state runs in it.
// By default states above kResidentStateMax run through the grouped sweep
// kernels: a state of up to 128 KiB would fit, but leave one workgroup per
// CU.  The autotuner may raise the cut per shape (resident_max).
constexpr int kBatchThreads = 256;
constexpr int kBatchLdsLimit = 160 * 1024;
constexpr size_t kResidentStateMax = 64 * 1024;
constexpr size_t kResidentStateLimit = 128 * 1024;
// LDS ahead of the state: the matrix of the current dense op (up to 4 KiB,
// 4 qubits at complex128), and the final reduction's partial sums
constexpr int kBatchScratchBytes = 4096;
inline size_t batch_lds_bytes(int n, sv_dtype d, bool *resident, size_t resident_max = kResidentStateMax)
{
    const size_t red = kBatchScratchBytes;
    const size_t sb = (d == SV_C128 ? size_t(16) : size_t(8)) << n;
    *resident = sb <= resident_max && sb + red <= (size_t)kBatchLdsLimit;
    return red + (*resident ? sb : 0);
}

// Launch the batch kernel over count instances (insts[order[i]]) that all
// have n qubits and whose dense ops are at most kmax qubits wide, with the
// state in LDS (resident) or in its HBM buffer; grid chosen from the LDS
// footprint, a leaner kernel when kmax <= 3.
sv_status launch_batch_class(const BInst *d_insts, const int *d_order, int count, int n, int kmax,
                             bool resident, sv_dtype dtype, hipStream_t st);

// Lower a (fused) HHL circuit into batch ops and a table buffer of
// *device_bytes.  tables holds the host-built tables (its first
// tables.size() bytes); deferred evolutions get a region after them and an
// entry in evo (out_off set, vt_off / w_off left for the caller).
struct EvoJob;
void lower_for_batch(const Circuit &f, sv_dtype dtype, std::vector<BOp> &ops, std::vector<unsigned char> &tables,
                     std::vector<EvoJob> &evo, size_t *device_bytes);

// k_max used for batch instances when the batch was created with k_max = 0
// and the autotuner has no entry for the instance's shape.
constexpr int kDefaultBatchK = 3;

// Launch choices of a batch instance's shape (dtype, ns, m), as the
// autotuner picks them (defaults otherwise).  None changes an instance's
// arithmetic except k (the fusion) and resident_kib (LDS-resident kernel or
// grouped sweeps); both are parity-tested either way.
struct BatchTune {
    int k = kDefaultBatchK;       // fusion width
    int group_max = 256;          // instances per grouped launch (states in HBM)
    int wave_target = 1024;       // waves a grouped wide-gate launch aims to keep busy
    int resident_kib = 64;        // largest state (KiB) run with the state in LDS
};

// The tuned choices for a shape; false (and defaults) when the autotuner has
// no entry.  batch_tuned_k: the tuned k, 0 when unknown.
bool batch_tuned(sv_dtype dtype, int ns, int m, BatchTune *out);
void batch_set_tuned(sv_dtype dtype, int ns, int m, const BatchTune &t);
int batch_tuned_k(sv_dtype dtype, int ns, int m);

// Sec. III-A step 4 from [P(ancilla = 1), pad, y_0.re, y_0.im, ...]:
// x_hat = Re(y) / ||Re(y)|| over the first dim entries, scale = ||b|| ||Re y|| / C.
sv_status recover_solution(const HHLParams &h, const double *p1_y, double *x_hat, int dim,
                           sv_solution_info *info);

}  // namespace hhlsv
