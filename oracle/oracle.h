/*
 * oracle.h -- plain FP64 CPU reference for the HHL state-vector path.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU
 * baseline may call it; the library never does.  It shares no code, header,
 * table or helper with the device library.  Everything is written for
 * clarity: one unfused gate at a time over all 2^n amplitudes, in double
 * precision, compiled without FMA contraction.
 *
 * Conventions (the paper fixes none of them; these are the readings used):
 *   - qubit q is bit q of the amplitude index (little-endian);
 *   - a state of n qubits is 2^n complex amplitudes stored as interleaved
 *     (re, im) doubles, caller-owned;
 *   - a k-qubit matrix acting on the qubit list (q_0..q_{k-1}) is a row-major
 *     2^k x 2^k complex matrix (interleaved re, im) whose row/column index is
 *     r = sum_l bit(q_l) * 2^l;
 *   - HHL registers: system qubits 0..ns-1, clock qubits ns..ns+m-1 (clock
 *     bit j is qubit ns+j), ancilla qubit ns+m.
 *
 * Return codes: 0 on success, negative on error (see ORC_E*).
 */
#ifndef HHL_ORACLE_H
#define HHL_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Gate kinds understood by the oracle. */
enum {
    ORC_H = 0,       /* Hadamard                                           */
    ORC_X = 1,       /* Pauli X                                            */
    ORC_RY = 2,      /* RY(theta) = [[c, -s], [s, c]], c,s of theta/2     */
    ORC_RZ = 3,      /* RZ(theta) = diag(e^{-i theta/2}, e^{i theta/2})   */
    ORC_P = 4,       /* P(phi) = diag(1, e^{i phi})                       */
    ORC_U3 = 5,      /* U3(theta, phi, lambda), OpenQASM convention       */
    ORC_CX = 6,      /* qubits (control, target)                          */
    ORC_CP = 7,      /* controlled phase e^{i phi} on |11>                */
    ORC_SWAP = 8,
    ORC_DENSE = 9,   /* params: 2^k x 2^k complex matrix                  */
    ORC_CDENSE = 10, /* qubits (c, targets...): matrix where bit c is 1   */
    ORC_UCRY = 11    /* qubits (t, c_0..c_{r-1}); params: 2^r angles      */
};

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_ENOMEM = -2,
    ORC_ENOTSYM = -4,
    ORC_ENOTPD = -5,
    ORC_ESINGULAR = -6
};

/* HHL variants (Sec. III-A step 1c, Sec. III-B n_neg). */
enum {
    ORC_HHL_SIGNED = 1,  /* sign qubit: the m clock qubits hold a two's-
                            complement eigenvalue estimate (m >= 2)       */
    ORC_HHL_DILATE = 2,  /* solve [[0, A'], [A'^T, 0]] [0; x] = [b; 0]
                            for a general square A (implies SIGNED)      */
    ORC_HHL_GS = 4       /* Gauss-Seidel: solve (M^{-1} A) x = M^{-1} b,
                            M = lower triangle of A with the diagonal
                            (implies DILATE); beta = ||M^{-1} b||        */
};

/* Apply one gate to psi (2^n complex).  nparams counts doubles. */
int orc_apply_gate(double *psi, int n, int kind, const int *qubits, int nq,
                   const double *params, long nparams);

/* Apply a flat gate list: gate g has kind kinds[g], qubits
 * qubits[qoff[g]..qoff[g+1]) and params params[poff[g]..poff[g+1]). */
int orc_apply_circuit(double *psi, int n, int ngates, const int *kinds,
                      const int *qoff, const int *qubits, const long *poff,
                      const double *params);

/* Matrix (2^k x 2^k complex, interleaved) of a named gate of kind H..SWAP. */
int orc_gate_matrix(int kind, const double *params, double *out);

/* QFT (inverse = 0) or its inverse (inverse = 1) on qubits q0..q0+m-1,
 * as the H / controlled-phase / SWAP sequence. */
int orc_qft(double *psi, int n, int q0, int m, int inverse);

/* Cyclic Jacobi eigen-decomposition of a symmetric N x N matrix A
 * (row-major): A = V diag(lam) V^T, V row-major with eigenvector k in
 * column k.  Eigenvalues are returned in ascending order. */
int orc_jacobi(const double *A, int N, double *V, double *lam, int *sweeps);

/* Gaussian elimination with partial pivoting: solve A x = b (N x N). */
int orc_ge_solve(const double *A, const double *b, int N, double *x);

/* Qubit-count estimate of the resources section (Sec. III-B), in the
 * reading that reproduces Table I: n_qpe = max(n_data + 1,
 * ceil(log2(kappa + 1))) + n_neg, n_total = n_data + n_qpe + 1. */
int orc_qubit_count(int dim, double kappa, int has_negative, int *n_data,
                    int *n_qpe, int *n_total);

typedef struct {
    int ns, m, n, j0;
    double beta, t, C, lambda_lo, lambda_hi, kappa;
    double p1;        /* P(ancilla = 1)                                   */
    double p10;       /* P(ancilla = 1 and clock = 0)                     */
    double max_imag;  /* max |Im y_s| over the postselected block         */
    double pad_leak;  /* norm of y over the padded system indices         */
    double x_norm;    /* ||x|| recovered as sqrt(p10) / C times beta      */
    int x_off;        /* x sits at system indices x_off .. x_off + N - 1  */
    int sign_qubit;   /* 1 if the clock value is read in two's complement */
} orc_hhl_info;

/* Full HHL solve of A x = b (A symmetric positive definite on the span of b,
 * N x N) with m clock qubits.  t > 0 fixes the evolution time; t <= 0 selects the
 * automatic rule.  Outputs (each may be NULL): psi_out (2^n complex final
 * state), x_hhl (N, the recovered solution), x_hat (N, unit norm). */
int orc_hhl_solve(const double *A, const double *b, int N, int m, double t,
                  double *psi_out, double *x_hhl, double *x_hat,
                  orc_hhl_info *info);

/* Spectral parameters only (no state): fills ns, m, n, j0, beta, t, C,
 * lambda_lo, lambda_hi, kappa, x_off, sign_qubit. */
int orc_hhl_params(const double *A, const double *b, int N, int m, double t,
                   orc_hhl_info *info);

/* The same with ORC_HHL_* flags (0 = the calls above).  With the sign
 * qubit, lambda_lo / lambda_hi / kappa are over |lambda|; a zero eigenvalue
 * that b reaches gives ORC_ESINGULAR. */
int orc_hhl_solve_ex(const double *A, const double *b, int N, int m,
                     double t, int flags, double *psi_out, double *x_hhl,
                     double *x_hat, orc_hhl_info *info);
int orc_hhl_params_ex(const double *A, const double *b, int N, int m,
                      double t, int flags, orc_hhl_info *info);

/* The Hermitian system the circuit encodes (padded, dilated with
 * ORC_HHL_DILATE): H (dim x dim, row-major) and the normalised right-hand
 * side b_hat (dim), either may be NULL; *x_off as in orc_hhl_info.
 * Returns dim (> 0) or an error. */
int orc_hhl_system(const double *A, const double *b, int N, int flags,
                   double *H, double *b_hat, int *x_off);

/* Newton-Raphson AC power flow (Sec. III).  Buses 0..nb-1 with type 0
 * (slack, exactly one), 1 (PV) or 2 (PQ); branch e joins from[e] and to[e]
 * with series impedance r[e] + j x[e] and total line charging bsh[e] (p.u.).
 * pspec / qspec: net injected power (generation minus load); vset: the
 * magnitude held at slack and PV buses.  Unknowns: angles of non-slack
 * buses, then magnitudes of PQ buses, in bus order.
 *
 * orc_pf_eval: injections P, Q (nb each), the mismatch F (N, may be NULL) and
 * the Jacobian dF/dx of the injections (N x N row-major, may be NULL) at
 * (vm, va); returns N.
 * orc_pf_newton: flat start, then x += J^{-1} F until max |F| < tol or
 * max_iter iterations; solver 0 solves exactly (Gaussian elimination),
 * solver 1 with orc_hhl_solve_ex(J, F, m clock qubits, automatic t, flags)
 * (flags must include ORC_HHL_DILATE or ORC_HHL_GS: J is not symmetric). */
#define ORC_PF_HISTORY 64
typedef struct {
    int iterations;     /* updates applied                               */
    int converged;      /* max |F| < tol reached                          */
    int n_unknowns;
    double mismatch;    /* final max |F|                                  */
    double history[ORC_PF_HISTORY];   /* max |F| before each update       */
} orc_pf_info;

int orc_pf_eval(int nb, int nbr, const int *from, const int *to,
                const double *r, const double *x, const double *bsh,
                const int *type, const double *pspec, const double *qspec,
                const double *vm, const double *va, double *P, double *Q,
                double *F, double *J);
int orc_pf_newton(int nb, int nbr, const int *from, const int *to,
                  const double *r, const double *x, const double *bsh,
                  const int *type, const double *pspec, const double *qspec,
                  const double *vset, int solver, int m, int flags,
                  int max_iter, double tol, double *vm, double *va,
                  orc_pf_info *info);

#ifdef __cplusplus
}
#endif
#endif
