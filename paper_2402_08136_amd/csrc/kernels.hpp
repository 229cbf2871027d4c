// Device-side data structures shared by the kernel launchers and the state /
// batch runtimes (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace hhlsv {

// One device operation, lowered from a circuit gate.
enum OpType : int {
    OP_DENSE = 0,   // dense 2^k x 2^k matrix on sorted targets, k <= 5
    OP_DIAG = 1,    // diagonal 2^k entries on sorted targets, k <= 12
    OP_WIDE = 2,    // dense matrix on sorted targets, k <= 12, optional control
    OP_UCRY = 3     // uniformly controlled RY: table of (cos, sin) half angles
};

struct DevOp {
    int type = OP_DENSE;
    int k = 0;               // targets (UCRY: controls)
    int q[kMaxUcryControls] = {0};   // sorted targets / UCRY control list
    int target = -1;         // UCRY target
    int control = -1;        // OP_WIDE control qubit, -1 = none
    size_t off = 0;          // byte offset of the op's table in the buffer
};

struct DeviceProgram {
    int device = -1;
    sv_dtype dtype = SV_C128;
    void *dbuf = nullptr;    // one allocation holding every table
    size_t bytes = 0;
    std::vector<DevOp> ops;
};

// Lower a circuit to device ops and upload its tables (FP64 built, rounded
// once to FP32 for SV_C64).  Returns nullptr and sets the error on failure.
DeviceProgram *get_device_program(const Circuit &c, sv_dtype dtype, sv_status *st);

// Launch one op on a 2^n state on the given stream; *family (may be NULL)
// receives the sv_kernel_family used.
sv_status launch_op(const DevOp &op, const DeviceProgram &prog, void *psi, int n,
                    sv_dtype dtype, hipStream_t stream, int *family = nullptr);

// Kernels used by the state runtime.
sv_status launch_init_zero_state(void *psi, int n, sv_dtype dtype, hipStream_t s);
// Sum of |psi_i|^2 over [lo, hi) into *dev_out (double), deterministic
// two-stage reduction using dev_partials (kReducePartials doubles).
constexpr int kReducePartials = 1024;
sv_status launch_norm2_range(const void *psi, uint64_t lo, uint64_t hi, sv_dtype dtype,
                             double *dev_partials, double *dev_out, hipStream_t s);
sv_status launch_gather(const void *psi, const uint64_t *dev_idx, size_t count,
                        void *dev_out, sv_dtype dtype, hipStream_t s);

inline size_t amp_bytes(sv_dtype d) { return d == SV_C128 ? 16 : 8; }

}  // namespace hhlsv
