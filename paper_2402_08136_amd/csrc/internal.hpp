// Internal host-side types of libhhlsv (not part of the ABI).
#pragma once

#include <complex>
#include <cstdint>
#include <memory>
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
    // HHL evolution gates e^{iAt 2^j} (CDENSE on the system register): j and
    // whether it is the inverse.  With empty params the matrix is "deferred":
    // it is built from the circuit's eigen-decomposition where it is needed
    // (on the device when applied, on the host by materialize()).
    int evo_j = -1;
    bool evo_inv = false;
    // MUX2 / MUX3 of evolution gates: the other controls' j (U_v =
    // e^{iAt p_v}, p_v the sum of 2^j over the controls set in v).
    int evo_j2 = -1, evo_j3 = -1;
};

inline bool gate_deferred(const Gate &g) { return g.evo_j >= 0 && g.params.empty(); }
// Control qubits of a CDENSE (1), MUX2 (2) or MUX3 (3) gate, 0 otherwise.
inline int gate_controls(const Gate &g)
{
    return g.kind == SV_GATE_MUX3 ? 3 : g.kind == SV_GATE_MUX2 ? 2 : g.kind == SV_GATE_CDENSE ? 1 : 0;
}
// Matrices a gate carries: 2^r - 1 for a MUX of r controls, else one.
inline int gate_matrices(const Gate &g)
{
    return g.kind == SV_GATE_MUX2 || g.kind == SV_GATE_MUX3 ? (1 << gate_controls(g)) - 1 : 1;
}
// The j of each control of a deferred evolution gate, in control order.
inline std::vector<int> gate_evo_js(const Gate &g)
{
    std::vector<int> js{g.evo_j};
    if (gate_controls(g) >= 2) js.push_back(g.evo_j2);
    if (gate_controls(g) >= 3) js.push_back(g.evo_j3);
    return js;
}

// Eigen-decomposition of the padded system matrix, A' = V diag(w) V^T, with
// the eigenvectors as the rows of Vt (Vt[k * D + i] = V[i][k]).
struct Spectral {
    int D = 0;
    std::vector<double> Vt;
    std::vector<double> w;
    double t = 0;
};

// Parameters an HHL circuit was built with (Sec. III-A step 1).
struct HHLParams {
    bool is_hhl = false;
    int dim = 0, ns = 0, m = 0, j0 = 0, n_qpe_est = 0;
    double t = 0, C = 0, lambda_lo = 0, lambda_hi = 0, kappa = 0, b_norm = 0;
    int x_off = 0;          // x sits at system indices x_off .. x_off + dim - 1
    bool sign_qubit = false, dilated = false, preconditioned = false;
    std::shared_ptr<const Spectral> spec;
};

// Interleaved complex entries of e^{+-i A' t 2^j} = V diag(e^{+-i phi}) V^T,
// phi_k = fmod(w_k t 2^j, 2 pi) (FP64, on the host).
std::vector<double> evolution_params(const Spectral &sp, int j, bool inverse);
// The same for e^{+-i A' t p} with any real power p (phi_k = fmod(w_k (t p), 2 pi)).
std::vector<double> evolution_params_pow(const Spectral &sp, double p, bool inverse);
// Fill a deferred gate's params from the circuit's eigen-decomposition.
void materialize(Gate &g, const HHLParams &h);

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
