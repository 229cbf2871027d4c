// Internal host-side types of libhhlsv (not part of the ABI).
#pragma once

#include <complex>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "hhlsv.h"

namespace hhlsv {

using cd = std::complex<double>;

// Thread-local error message plumbing: every ABI entry point returns a status
// and leaves a readable message here.
void set_error(const std::string &msg);
sv_status fail(sv_status st, const std::string &msg);

constexpr int kMaxQubits = 34;
constexpr int kMaxDenseQubits = 12;   // DENSE / CDENSE / DIAG target width
constexpr int kMaxUcryControls = 20;

struct Gate {
    int kind = 0;                 // sv_gate_kind
    std::vector<int> qubits;      // as given (DENSE/DIAG after fusion: sorted)
    std::vector<double> params;   // angles, or interleaved complex entries
};

// Parameters an HHL circuit was built with (Sec. III-A step 1).
struct HHLParams {
    bool is_hhl = false;
    int dim = 0, ns = 0, m = 0, j0 = 0, n_qpe_est = 0;
    double t = 0, C = 0, lambda_lo = 0, lambda_hi = 0, kappa = 0, b_norm = 0;
};

struct DeviceProgram;  // device copy of a circuit's tables (device.hip)

struct Circuit {
    int n = 0;
    std::vector<Gate> gates;
    HHLParams hhl;
    // Device copies of the matrices / tables, per (device, dtype); filled
    // lazily by the first sv_apply and reused afterwards.
    mutable std::mutex dev_mu;
    mutable std::vector<DeviceProgram *> dev;
    ~Circuit();
};

// Gate metadata helpers shared by the builder, fusion and the device lowering.
int gate_nparams_named(int kind);            // -1 for variable-size kinds
bool gate_is_diagonal(int kind);
// Dense 2^k x 2^k matrix (row-major) of any non-UCRY gate, over the gate's
// qubit list in the given order (CDENSE: over (c, targets...)).
std::vector<cd> gate_matrix(const Gate &g);
// Diagonal entries of a diagonal gate over its qubit list.
std::vector<cd> gate_diagonal(const Gate &g);

sv_status validate_gate(int n, int kind, const int *qubits, int nq,
                        const double *params, int nparams);

// Symmetric eigen-decomposition (Householder tridiagonalisation followed by
// implicit QL with Wilkinson shifts): A = V diag(w) V^T, ascending w, V
// row-major with eigenvector k in column k.  Returns false if QL fails to
// converge.
bool sym_eig(const std::vector<double> &A, int N, std::vector<double> &w,
             std::vector<double> &V);

}  // namespace hhlsv

struct sv_circuit {
    hhlsv::Circuit c;
};
