/*
 * oracle.c -- plain FP64 CPU reference for the HHL state-vector path.
 *
 * TEST INFRASTRUCTURE ONLY: called by tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the library.  No code is shared
 * with the device library.  Build: gcc -std=c11 -O2 -ffp-contract=off
 * -fno-fast-math -fPIC -shared (no FMA contraction, IEEE double rounding).
 *
 * What it follows (M. Zheng et al., "Early Exploration of a Flexible
 * Framework for Efficient Quantum Linear Solvers in Power Systems", PESGM
 * 2024):
 *   - the n-qubit state is a 2^n complex vector (Sec. I);
 *   - HHL computes |x> = A^{-1}|b> = sum_i lambda_i^{-1} b_i |v_i> through
 *     phase estimation with controlled e^{iAt} (Sec. III-A);
 *   - the "Practical HHL procedures" box of Sec. III-A: normalise b and keep
 *     ||b|| (step 1), pad to a power of two (step 1b), build the circuit
 *     (step 2, Fig. 5), read the state vector directly (step 3, simulator
 *     case), recover the norm and x (step 4); the Hermitian dilation of
 *     step 1c for a general A and the sign qubit of Sec. III-B;
 *   - the qubit-count estimate of Sec. III-B and Table I.
 * Readings where the paper is silent or inconsistent are stated at each
 * function (register order, QFT convention, choice of t, norm recovery).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

typedef struct { double re, im; } cplx;

static cplx c_make(double re, double im) { cplx z; z.re = re; z.im = im; return z; }
static cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static cplx c_mul(cplx a, cplx b)
{
    return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
static cplx c_expi(double phi) { return c_make(cos(phi), sin(phi)); }
static cplx c_conj(cplx a) { return c_make(a.re, -a.im); }
static double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }

/* ------------------------------------------------------------------------
 * Gate application by definition.
 *
 * A k-qubit matrix M on qubits (q_0..q_{k-1}) maps, for every index i whose
 * target bits are all zero (a "group base"), the 2^k amplitudes
 * psi[i + sum_l bit_l(r) 2^{q_l}], r = 0..2^k-1, to M times that vector.
 * With a control qubit c >= 0, only groups whose bit c is 1 are touched.
 * ---------------------------------------------------------------------- */
static int apply_matrix(cplx *psi, int n, const int *q, int k, const cplx *M,
                        int control)
{
    const long dim = 1L << n;
    const long K = 1L << k;
    long tmask = 0;
    for (int l = 0; l < k; ++l) {
        if (q[l] < 0 || q[l] >= n || (tmask >> q[l]) & 1L)
            return ORC_EINVAL;
        tmask |= 1L << q[l];
    }
    if (control >= n || (control >= 0 && ((tmask >> control) & 1L)))
        return ORC_EINVAL;
    long *idx = (long *)malloc(sizeof(long) * K);
    cplx *v = (cplx *)malloc(sizeof(cplx) * K);
    if (!idx || !v) { free(idx); free(v); return ORC_ENOMEM; }
    for (long i = 0; i < dim; ++i) {
        if (i & tmask)
            continue;
        if (control >= 0 && !((i >> control) & 1L))
            continue;
        for (long r = 0; r < K; ++r) {
            long off = 0;
            for (int l = 0; l < k; ++l)
                if ((r >> l) & 1L)
                    off |= 1L << q[l];
            idx[r] = i | off;
            v[r] = psi[idx[r]];
        }
        for (long r = 0; r < K; ++r) {
            cplx acc = c_make(0.0, 0.0);
            for (long c = 0; c < K; ++c)
                acc = c_add(acc, c_mul(M[r * K + c], v[c]));
            psi[idx[r]] = acc;
        }
    }
    free(idx);
    free(v);
    return ORC_OK;
}

/* Matrices of the named gates (textbook / OpenQASM definitions). */
static int named_matrix(int kind, const double *p, cplx *M)
{
    const double s2 = 1.0 / sqrt(2.0);
    switch (kind) {
    case ORC_H:
        M[0] = c_make(s2, 0); M[1] = c_make(s2, 0);
        M[2] = c_make(s2, 0); M[3] = c_make(-s2, 0);
        return 1;
    case ORC_X:
        M[0] = c_make(0, 0); M[1] = c_make(1, 0);
        M[2] = c_make(1, 0); M[3] = c_make(0, 0);
        return 1;
    case ORC_RY: {
        double c = cos(p[0] / 2), s = sin(p[0] / 2);
        M[0] = c_make(c, 0); M[1] = c_make(-s, 0);
        M[2] = c_make(s, 0); M[3] = c_make(c, 0);
        return 1;
    }
    case ORC_RZ:
        M[0] = c_expi(-p[0] / 2); M[1] = c_make(0, 0);
        M[2] = c_make(0, 0);      M[3] = c_expi(p[0] / 2);
        return 1;
    case ORC_P:
        M[0] = c_make(1, 0); M[1] = c_make(0, 0);
        M[2] = c_make(0, 0); M[3] = c_expi(p[0]);
        return 1;
    case ORC_U3: {
        double c = cos(p[0] / 2), s = sin(p[0] / 2);
        cplx el = c_expi(p[2]), ep = c_expi(p[1]), epl = c_expi(p[1] + p[2]);
        M[0] = c_make(c, 0);
        M[1] = c_make(-el.re * s, -el.im * s);
        M[2] = c_make(ep.re * s, ep.im * s);
        M[3] = c_make(epl.re * c, epl.im * c);
        return 1;
    }
    case ORC_CX: /* qubit list (control, target): r = bit_c + 2 bit_t */
        for (int i = 0; i < 16; ++i) M[i] = c_make(0, 0);
        M[0 * 4 + 0] = c_make(1, 0);
        M[2 * 4 + 2] = c_make(1, 0);
        M[1 * 4 + 3] = c_make(1, 0);
        M[3 * 4 + 1] = c_make(1, 0);
        return 2;
    case ORC_CP:
        for (int i = 0; i < 16; ++i) M[i] = c_make(0, 0);
        M[0] = c_make(1, 0); M[5] = c_make(1, 0); M[10] = c_make(1, 0);
        M[15] = c_expi(p[0]);
        return 2;
    case ORC_SWAP:
        for (int i = 0; i < 16; ++i) M[i] = c_make(0, 0);
        M[0 * 4 + 0] = c_make(1, 0);
        M[1 * 4 + 2] = c_make(1, 0);
        M[2 * 4 + 1] = c_make(1, 0);
        M[3 * 4 + 3] = c_make(1, 0);
        return 2;
    default:
        return -1;
    }
}

static int named_nparams(int kind)
{
    switch (kind) {
    case ORC_RY: case ORC_RZ: case ORC_P: case ORC_CP: return 1;
    case ORC_U3: return 3;
    default: return 0;
    }
}

int orc_gate_matrix(int kind, const double *params, double *out)
{
    cplx M[16];
    int k = named_matrix(kind, params, M);
    if (k < 0)
        return ORC_EINVAL;
    memcpy(out, M, sizeof(cplx) * (size_t)(1 << k) * (size_t)(1 << k));
    return k;
}

/* Uniformly controlled RY: RY(theta[v]) on qubit t where v is the value of
 * the control qubits (c_0 is the least significant bit of v). */
static int apply_ucry(cplx *psi, int n, int t, const int *c, int r,
                      const double *theta)
{
    const long dim = 1L << n;
    if (t < 0 || t >= n)
        return ORC_EINVAL;
    for (int l = 0; l < r; ++l)
        if (c[l] < 0 || c[l] >= n || c[l] == t)
            return ORC_EINVAL;
    for (long i = 0; i < dim; ++i) {
        if ((i >> t) & 1L)
            continue;
        long v = 0;
        for (int l = 0; l < r; ++l)
            v |= ((i >> c[l]) & 1L) << l;
        double cs = cos(theta[v] / 2), sn = sin(theta[v] / 2);
        cplx a0 = psi[i], a1 = psi[i | (1L << t)];
        psi[i] = c_make(cs * a0.re - sn * a1.re, cs * a0.im - sn * a1.im);
        psi[i | (1L << t)] = c_make(sn * a0.re + cs * a1.re,
                                    sn * a0.im + cs * a1.im);
    }
    return ORC_OK;
}

int orc_apply_gate(double *psi_d, int n, int kind, const int *qubits, int nq,
                   const double *params, long nparams)
{
    cplx *psi = (cplx *)psi_d;
    if (n < 1 || n > 40)
        return ORC_EINVAL;
    if (kind >= ORC_H && kind <= ORC_SWAP) {
        cplx M[16];
        if (nparams < named_nparams(kind))
            return ORC_EINVAL;
        int k = named_matrix(kind, params, M);
        if (nq != k)
            return ORC_EINVAL;
        return apply_matrix(psi, n, qubits, k, M, -1);
    }
    if (kind == ORC_DENSE || kind == ORC_CDENSE) {
        int ctrl = kind == ORC_CDENSE ? qubits[0] : -1;
        const int *tq = kind == ORC_CDENSE ? qubits + 1 : qubits;
        int k = kind == ORC_CDENSE ? nq - 1 : nq;
        if (k < 1 || k > 20 || nparams != 2L * (1L << k) * (1L << k))
            return ORC_EINVAL;
        return apply_matrix(psi, n, tq, k, (const cplx *)params, ctrl);
    }
    if (kind == ORC_UCRY) {
        int r = nq - 1;
        if (r < 0 || r > 24 || nparams != (1L << r))
            return ORC_EINVAL;
        return apply_ucry(psi, n, qubits[0], qubits + 1, r, params);
    }
    return ORC_EINVAL;
}

int orc_apply_circuit(double *psi, int n, int ngates, const int *kinds,
                      const int *qoff, const int *qubits, const long *poff,
                      const double *params)
{
    for (int g = 0; g < ngates; ++g) {
        int rc = orc_apply_gate(psi, n, kinds[g], qubits + qoff[g],
                                qoff[g + 1] - qoff[g], params + poff[g],
                                poff[g + 1] - poff[g]);
        if (rc < 0)
            return rc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Quantum Fourier transform on m consecutive qubits.
 *
 * Reading (the paper only names QPE; its circuit figure is not available):
 * QFT|x> = 2^{-m/2} sum_y e^{+2 pi i x y / 2^m} |y>, with clock bit j on
 * qubit q0 + j.  Gate sequence: for j = m-1 down to 0, H on j, then for
 * k = j-1 down to 0 a controlled phase pi / 2^{j-k} between k and j; finally
 * swap j and m-1-j for j < m/2.  The inverse runs the sequence backwards
 * with negated phases.
 * ---------------------------------------------------------------------- */
static int gate1(cplx *psi, int n, int kind, int q, const double *p)
{
    return orc_apply_gate((double *)psi, n, kind, &q, 1, p, named_nparams(kind));
}

static int gate2(cplx *psi, int n, int kind, int a, int b, const double *p)
{
    int qs[2] = {a, b};
    return orc_apply_gate((double *)psi, n, kind, qs, 2, p, named_nparams(kind));
}

int orc_qft(double *psi_d, int n, int q0, int m, int inverse)
{
    cplx *psi = (cplx *)psi_d;
    int rc;
    if (m < 1 || q0 < 0 || q0 + m > n)
        return ORC_EINVAL;
    if (!inverse) {
        for (int j = m - 1; j >= 0; --j) {
            if ((rc = gate1(psi, n, ORC_H, q0 + j, NULL)) < 0) return rc;
            for (int k = j - 1; k >= 0; --k) {
                double phi = ORC_PI / (double)(1L << (j - k));
                if ((rc = gate2(psi, n, ORC_CP, q0 + k, q0 + j, &phi)) < 0) return rc;
            }
        }
        for (int j = 0; j < m / 2; ++j)
            if ((rc = gate2(psi, n, ORC_SWAP, q0 + j, q0 + m - 1 - j, NULL)) < 0) return rc;
    } else {
        for (int j = m / 2 - 1; j >= 0; --j)
            if ((rc = gate2(psi, n, ORC_SWAP, q0 + j, q0 + m - 1 - j, NULL)) < 0) return rc;
        for (int j = 0; j < m; ++j) {
            for (int k = 0; k < j; ++k) {
                double phi = -ORC_PI / (double)(1L << (j - k));
                if ((rc = gate2(psi, n, ORC_CP, q0 + k, q0 + j, &phi)) < 0) return rc;
            }
            if ((rc = gate1(psi, n, ORC_H, q0 + j, NULL)) < 0) return rc;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Cyclic Jacobi eigen-decomposition (classical two-sided rotations).
 * For each pair p < q with a_pq != 0 a plane rotation J(p, q, c, s) with
 * t = s/c the smaller root of t^2 + 2 theta t - 1 = 0,
 * theta = (a_qq - a_pp) / (2 a_pq), zeroes a_pq; A <- J^T A J, V <- V J.
 * Sweeps repeat until the off-diagonal mass is negligible.
 * ---------------------------------------------------------------------- */
int orc_jacobi(const double *A_in, int N, double *V, double *lam, int *sweeps_out)
{
    if (N < 1)
        return ORC_EINVAL;
    double *A = (double *)malloc(sizeof(double) * (size_t)N * N);
    if (!A)
        return ORC_ENOMEM;
    memcpy(A, A_in, sizeof(double) * (size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            V[i * N + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (long i = 0; i < (long)N * N; ++i)
        fro += A[i] * A[i];
    fro = sqrt(fro);
    int sweep = 0;
    for (; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < N; ++p)
            for (int q = 0; q < N; ++q)
                if (p != q)
                    off += A[p * N + q] * A[p * N + q];
        if (sqrt(off) <= 1e-17 * fro || off == 0.0)
            break;
        for (int p = 0; p < N - 1; ++p) {
            for (int q = p + 1; q < N; ++q) {
                double apq = A[p * N + q];
                if (apq == 0.0)
                    continue;
                double theta = (A[q * N + q] - A[p * N + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) /
                           (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                for (int k = 0; k < N; ++k) { /* A <- A J (columns p, q) */
                    double akp = A[k * N + p], akq = A[k * N + q];
                    A[k * N + p] = c * akp - s * akq;
                    A[k * N + q] = s * akp + c * akq;
                }
                for (int k = 0; k < N; ++k) { /* A <- J^T A (rows p, q) */
                    double apk = A[p * N + k], aqk = A[q * N + k];
                    A[p * N + k] = c * apk - s * aqk;
                    A[q * N + k] = s * apk + c * aqk;
                }
                A[p * N + q] = 0.0;
                A[q * N + p] = 0.0;
                for (int k = 0; k < N; ++k) { /* V <- V J */
                    double vkp = V[k * N + p], vkq = V[k * N + q];
                    V[k * N + p] = c * vkp - s * vkq;
                    V[k * N + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < N; ++i)
        lam[i] = A[i * N + i];
    /* ascending order (selection sort keeps it obvious) */
    for (int i = 0; i < N; ++i) {
        int best = i;
        for (int j = i + 1; j < N; ++j)
            if (lam[j] < lam[best])
                best = j;
        if (best != i) {
            double tmp = lam[i]; lam[i] = lam[best]; lam[best] = tmp;
            for (int k = 0; k < N; ++k) {
                double tv = V[k * N + i];
                V[k * N + i] = V[k * N + best];
                V[k * N + best] = tv;
            }
        }
    }
    free(A);
    if (sweeps_out)
        *sweeps_out = sweep;
    return ORC_OK;
}

/* Gaussian elimination with partial pivoting (textbook). */
int orc_ge_solve(const double *A_in, const double *b_in, int N, double *x)
{
    if (N < 1)
        return ORC_EINVAL;
    double *M = (double *)malloc(sizeof(double) * (size_t)N * (N + 1));
    if (!M)
        return ORC_ENOMEM;
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j)
            M[i * (N + 1) + j] = A_in[i * N + j];
        M[i * (N + 1) + N] = b_in[i];
    }
    for (int col = 0; col < N; ++col) {
        int piv = col;
        for (int r = col + 1; r < N; ++r)
            if (fabs(M[r * (N + 1) + col]) > fabs(M[piv * (N + 1) + col]))
                piv = r;
        if (M[piv * (N + 1) + col] == 0.0) {
            free(M);
            return ORC_EINVAL;
        }
        if (piv != col)
            for (int j = 0; j <= N; ++j) {
                double t = M[col * (N + 1) + j];
                M[col * (N + 1) + j] = M[piv * (N + 1) + j];
                M[piv * (N + 1) + j] = t;
            }
        for (int r = col + 1; r < N; ++r) {
            double f = M[r * (N + 1) + col] / M[col * (N + 1) + col];
            for (int j = col; j <= N; ++j)
                M[r * (N + 1) + j] -= f * M[col * (N + 1) + j];
        }
    }
    for (int i = N - 1; i >= 0; --i) {
        double s = M[i * (N + 1) + N];
        for (int j = i + 1; j < N; ++j)
            s -= M[i * (N + 1) + j] * x[j];
        x[i] = s / M[i * (N + 1) + i];
    }
    free(M);
    return ORC_OK;
}

/* Sec. III-B: n_data = log2(rows) of the expanded matrix; n_QPE from the
 * printed max(n_data + 1, ceil(log2(kappa + 1))).  Table I's printed counts
 * are reproduced only when the sign qubit is added to the QPE register and
 * the inversion ancilla to the total, so that is the reading taken. */
int orc_qubit_count(int dim, double kappa, int has_negative, int *n_data,
                    int *n_qpe, int *n_total)
{
    if (dim < 1 || !(kappa >= 1.0))
        return ORC_EINVAL;
    int nd = 0;
    while ((1 << nd) < dim)
        ++nd;
    int qk = (int)ceil(log2(kappa + 1.0));
    int nq = (nd + 1 > qk ? nd + 1 : qk) + (has_negative ? 1 : 0);
    if (n_data) *n_data = nd;
    if (n_qpe) *n_qpe = nq;
    if (n_total) *n_total = nd + nq + 1;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * HHL (Sec. III-A procedure box, Fig. 5).
 * ---------------------------------------------------------------------- */
typedef struct {
    int N, ns, dim, m, n;
    int sgn;       /* clock value read in two's complement (sign qubit)   */
    int x_off;     /* x occupies system indices x_off .. x_off + N - 1    */
    double *Ap;    /* the Hermitian system matrix, dim x dim              */
    double *bh;    /* normalised padded right-hand side                   */
    double *V;     /* eigenvectors (columns)                               */
    double *lam;   /* eigenvalues                                          */
    double beta, t, C, lambda_lo, lambda_hi, kappa;
    int j0;
} hhl_prep;

static void prep_free(hhl_prep *h)
{
    free(h->Ap); free(h->bh); free(h->V); free(h->lam);
}

/* Step 1 of the procedure box: the Hermitian system the circuit encodes.
 *   - step 1a (flag ORC_HHL_GS): A, b -> M^{-1} A, M^{-1} b (gauss_seidel),
 *     then the dilation, since M^{-1} A is not symmetric;
 *   - b_hat = b / ||b||, beta = ||b|| (of the preconditioned b with GS);
 *   - step 1b: A is padded to the next power of two, A' = A (+) I, with b
 *     zero-padded;
 *   - step 1c (flag ORC_HHL_DILATE): the padded A' is replaced by the
 *     symmetric dilation H = [[0, A'], [A'^T, 0]] (A real, so A^dagger =
 *     A^T) and the right-hand side by [b_hat; 0]; since H [0; x] = [b; 0]
 *     exactly when A x = b, x is read from the second half (x_off = size
 *     of A').  The paper lists padding (1b) before the dilation (1c); that
 *     order is kept, so a 29 x 29 A becomes 32 x 32 and then 64 x 64,
 *     the 6 data qubits of Table I's preconditioned 30-bus case.
 *   - without the flag A must be symmetric. */
/* Gauss-Seidel preconditioning (step 1a, Sec. III-B): with M = D + L, the
 * lower triangle of A including its diagonal, the system becomes
 * (M^{-1} A) x = M^{-1} b, which has the same solution.  The paper names the
 * preconditioner but gives no formula; this is the textbook left
 * Gauss-Seidel splitting.  M^{-1} A and M^{-1} b come from forward
 * substitution, one column at a time.  Returns ORC_ESINGULAR for a zero
 * diagonal entry. */
static int gauss_seidel(const double *A, const double *b, int N, double *At,
                        double *bt)
{
    for (int i = 0; i < N; ++i)
        if (A[i * N + i] == 0.0)
            return ORC_ESINGULAR;
    for (int col = 0; col <= N; ++col) {
        /* column col of A, or b for col == N */
        for (int i = 0; i < N; ++i) {
            double r = col < N ? A[i * N + col] : b[i];
            for (int k = 0; k < i; ++k)
                r -= A[i * N + k] * (col < N ? At[k * N + col] : bt[k]);
            r /= A[i * N + i];
            if (col < N)
                At[i * N + col] = r;
            else
                bt[i] = r;
        }
    }
    return ORC_OK;
}

static int hhl_system(const double *A_in, const double *b_in, int N,
                      int flags, hhl_prep *h)
{
    const int gs = (flags & ORC_HHL_GS) != 0;
    const int dilate = gs || (flags & ORC_HHL_DILATE) != 0;
    const double *A = A_in, *b = b_in;
    double *At = NULL, *bt = NULL;
    if (gs) {
        At = (double *)malloc(sizeof(double) * (size_t)N * N);
        bt = (double *)malloc(sizeof(double) * (size_t)N);
        if (!At || !bt) {
            free(At); free(bt);
            return ORC_ENOMEM;
        }
        int rc = gauss_seidel(A_in, b_in, N, At, bt);
        if (rc < 0) {
            free(At); free(bt);
            return rc;
        }
        A = At;
        b = bt;
    }
    int na = 0;
    while ((1 << na) < N)
        ++na;
    if (!dilate && na < 1)
        na = 1;
    const int pa = 1 << na;               /* size of the padded A'       */
    const int ns = dilate ? na + 1 : na;
    const int dim = 1 << ns;
    h->N = N; h->ns = ns; h->dim = dim;
    h->x_off = dilate ? pa : 0;
    if (!dilate) {
        double amax = 0.0, asym = 0.0;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                amax = fmax(amax, fabs(A[i * N + j]));
                asym = fmax(asym, fabs(A[i * N + j] - A[j * N + i]));
            }
        if (asym > 1e-12 * amax) {
            free(At); free(bt);
            return ORC_ENOTSYM;
        }
    }
    h->Ap = (double *)calloc((size_t)dim * dim, sizeof(double));
    h->bh = (double *)calloc((size_t)dim, sizeof(double));
    h->V = (double *)calloc((size_t)dim * dim, sizeof(double));
    h->lam = (double *)calloc((size_t)dim, sizeof(double));
    if (!h->Ap || !h->bh || !h->V || !h->lam) {
        free(At); free(bt);
        return ORC_ENOMEM;
    }
    for (int i = 0; i < pa; ++i)
        for (int j = 0; j < pa; ++j) {
            double a = (i < N && j < N) ? A[i * N + j] : (i == j ? 1.0 : 0.0);
            if (dilate) {
                h->Ap[i * dim + (pa + j)] = a;   /* upper right: A'        */
                h->Ap[(pa + j) * dim + i] = a;   /* lower left: A'^T       */
            } else {
                h->Ap[i * dim + j] = a;
            }
        }
    double bb = 0.0;
    for (int i = 0; i < N; ++i)
        bb += b[i] * b[i];
    h->beta = sqrt(bb);
    if (h->beta > 0.0)
        for (int i = 0; i < N; ++i)
            h->bh[i] = b[i] / h->beta;
    free(At); free(bt);
    return h->beta > 0.0 ? ORC_OK : ORC_EINVAL;
}

int orc_hhl_system(const double *A, const double *b, int N, int flags,
                   double *H, double *b_hat, int *x_off)
{
    hhl_prep h;
    memset(&h, 0, sizeof(h));
    if (N < 1 || (flags & ~(ORC_HHL_SIGNED | ORC_HHL_DILATE | ORC_HHL_GS)))
        return ORC_EINVAL;
    int rc = hhl_system(A, b, N, flags, &h);
    if (rc >= 0) {
        if (H)
            memcpy(H, h.Ap, sizeof(double) * (size_t)h.dim * h.dim);
        if (b_hat)
            memcpy(b_hat, h.bh, sizeof(double) * (size_t)h.dim);
        if (x_off)
            *x_off = h.x_off;
        rc = h.dim;
    }
    prep_free(&h);
    return rc;
}

/* Step 1 and the spectral parameters the circuit needs.
 *   - the system of hhl_system;
 *   - lambda_lo / lambda_hi: the smallest / largest eigenvalue among the
 *     eigenvectors b_hat overlaps (weight (v_i . b_hat)^2 > 1e-20).  This is
 *     "the smallest-magnitude eigenvalue of the matrix input" of step 4a once
 *     the pad block, which b_hat never reaches, is excluded.  With the sign
 *     qubit both are taken over |lambda|;
 *   - sign qubit (the n_neg qubit of Sec. III-B, flag ORC_HHL_SIGNED, implied
 *     by the dilation, whose spectrum is +-sigma): the paper only says that
 *     one qubit is added when A has negative eigenvalues.  Reading: the m
 *     clock qubits (the sign qubit among them, as in Table I's n_QPE) hold a
 *     two's-complement value.  A negative eigenvalue's phase lambda t / 2 pi
 *     wraps to 1 + lambda t / 2 pi, so its clock value c = 2^m + v decodes
 *     to v = lambda t 2^m / 2 pi < 0; magnitudes get m - 1 bits;
 *   - t (reading; the paper does not give its rule): with top = 2^m - 1
 *     (2^{m-1} - 1 with the sign qubit), when kappa <= top,
 *     j0 = floor(top / kappa) and t = 2 pi j0 / (2^m lambda_lo), so
 *     lambda_lo lands on clock value j0 and lambda_hi at most on top;
 *     otherwise t = 2 pi top / (2^m lambda_hi).  A caller-given t > 0
 *     overrides the rule.  Then j0 = max(1, round(lambda_lo t 2^m / 2 pi))
 *     and C = 2 pi j0 / (t 2^m), the eigenvalue clock value j0 stands for. */
static int hhl_prepare(const double *A, const double *b, int N, int m,
                       double t_in, int flags, hhl_prep *h)
{
    memset(h, 0, sizeof(*h));
    const int sgn = (flags & (ORC_HHL_SIGNED | ORC_HHL_DILATE | ORC_HHL_GS)) != 0;
    if (N < 1 || m < 1 || m > 20 || (sgn && m < 2) ||
        (flags & ~(ORC_HHL_SIGNED | ORC_HHL_DILATE | ORC_HHL_GS)))
        return ORC_EINVAL;
    int rc = hhl_system(A, b, N, flags, h);
    if (rc < 0) {
        prep_free(h);
        return rc;
    }
    const int dim = h->dim;
    h->m = m; h->n = h->ns + m + 1; h->sgn = sgn;
    rc = orc_jacobi(h->Ap, dim, h->V, h->lam, NULL);
    if (rc < 0) {
        prep_free(h);
        return rc;
    }
    int found = 0;
    for (int k = 0; k < dim; ++k) {
        double ov = 0.0;
        for (int i = 0; i < dim; ++i)
            ov += h->V[i * dim + k] * h->bh[i];
        if (ov * ov > 1e-20) {
            double l = sgn ? fabs(h->lam[k]) : h->lam[k];
            if (!found || l < h->lambda_lo) h->lambda_lo = l;
            if (!found || l > h->lambda_hi) h->lambda_hi = l;
            found = 1;
        }
    }
    if (!found || !(h->lambda_lo > 0.0)) {
        prep_free(h);
        return sgn ? ORC_ESINGULAR : ORC_ENOTPD;
    }
    h->kappa = h->lambda_hi / h->lambda_lo;
    const double top = (double)((1L << (sgn ? m - 1 : m)) - 1);
    const double two_m = (double)(1L << m);
    if (t_in > 0.0) {
        h->t = t_in;
    } else if (h->kappa <= top) {
        double j0 = floor(top / h->kappa);
        h->t = 2.0 * ORC_PI * j0 / (two_m * h->lambda_lo);
    } else {
        h->t = 2.0 * ORC_PI * top / (two_m * h->lambda_hi);
    }
    double jr = round(h->lambda_lo * h->t * two_m / (2.0 * ORC_PI));
    h->j0 = jr < 1.0 ? 1 : (int)jr;
    h->C = 2.0 * ORC_PI * (double)h->j0 / (h->t * two_m);
    return ORC_OK;
}

static void fill_info(const hhl_prep *h, orc_hhl_info *info)
{
    memset(info, 0, sizeof(*info));
    info->ns = h->ns; info->m = h->m; info->n = h->n; info->j0 = h->j0;
    info->beta = h->beta; info->t = h->t; info->C = h->C;
    info->lambda_lo = h->lambda_lo; info->lambda_hi = h->lambda_hi;
    info->kappa = h->kappa;
    info->x_off = h->x_off; info->sign_qubit = h->sgn;
}

int orc_hhl_params_ex(const double *A, const double *b, int N, int m, double t,
                      int flags, orc_hhl_info *info)
{
    hhl_prep h;
    int rc = hhl_prepare(A, b, N, m, t, flags, &h);
    if (rc < 0)
        return rc;
    if (info)
        fill_info(&h, info);
    prep_free(&h);
    return ORC_OK;
}

/* U_j = e^{i A' t 2^j} = V diag(e^{i phi_k}) V^T with
 * phi_k = fmod(lambda_k t 2^j, 2 pi); conj = 1 gives U_j^dagger.  Each power
 * comes straight from the eigen-decomposition. */
static void build_u(const hhl_prep *h, int j, int conj, cplx *U)
{
    const int d = h->dim;
    const double tj = h->t * (double)(1L << j);
    cplx *ph = (cplx *)malloc(sizeof(cplx) * d);
    for (int k = 0; k < d; ++k) {
        ph[k] = c_expi(fmod(h->lam[k] * tj, 2.0 * ORC_PI));
        if (conj)
            ph[k] = c_conj(ph[k]);
    }
    for (int a = 0; a < d; ++a)
        for (int bcol = 0; bcol < d; ++bcol) {
            cplx acc = c_make(0, 0);
            for (int k = 0; k < d; ++k) {
                double w = h->V[a * d + k] * h->V[bcol * d + k];
                acc = c_add(acc, c_make(w * ph[k].re, w * ph[k].im));
            }
            U[a * d + bcol] = acc;
        }
    free(ph);
}

int orc_hhl_params(const double *A, const double *b, int N, int m, double t,
                   orc_hhl_info *info)
{
    return orc_hhl_params_ex(A, b, N, m, t, 0, info);
}

int orc_hhl_solve_ex(const double *A, const double *b, int N, int m,
                     double t_in, int flags, double *psi_out, double *x_hhl,
                     double *x_hat, orc_hhl_info *info)
{
    hhl_prep h;
    int rc = hhl_prepare(A, b, N, m, t_in, flags, &h);
    if (rc < 0)
        return rc;
    const int ns = h.ns, n = h.n, d = h.dim;
    const long dim = 1L << n;
    cplx *psi = (cplx *)calloc((size_t)dim, sizeof(cplx));
    cplx *U = (cplx *)malloc(sizeof(cplx) * (size_t)d * d);
    int *q = (int *)malloc(sizeof(int) * (size_t)(ns + m + 1));
    double *theta = (double *)malloc(sizeof(double) * (size_t)(1L << m));
    if (!psi || !U || !q || !theta) {
        free(psi); free(U); free(q); free(theta); prep_free(&h);
        return ORC_ENOMEM;
    }
    /* |b> on the system register, clock and ancilla in |0> (Fig. 5 input;
     * the amplitudes are loaded directly). */
    for (int s = 0; s < d; ++s)
        psi[s] = c_make(h.bh[s], 0.0);
    /* Phase estimation: H on every clock qubit, then e^{iAt 2^j} controlled
     * by clock bit j, then the inverse QFT. */
    for (int j = 0; j < m && rc >= 0; ++j)
        rc = gate1(psi, n, ORC_H, ns + j, NULL);
    for (int j = 0; j < m && rc >= 0; ++j) {
        build_u(&h, j, 0, U);
        q[0] = ns + j;
        for (int s = 0; s < ns; ++s)
            q[1 + s] = s;
        rc = apply_matrix(psi, n, q + 1, ns, U, q[0]);
    }
    if (rc >= 0)
        rc = orc_qft((double *)psi, n, ns, m, 1);
    /* Eigenvalue inversion: clock value c decodes to v (v = c, or with the
     * sign qubit the two's-complement value, c - 2^m for c >= 2^{m-1}), which
     * stands for lambda = C v / j0; the ancilla is rotated so that its |1>
     * amplitude is C / lambda = j0 / v (clamped to [-1, 1]; v = 0 is left
     * alone).  A negative v gives a negative angle, so the amplitude keeps
     * lambda's sign. */
    theta[0] = 0.0;
    for (long c = 1; c < (1L << m); ++c) {
        long v = (h.sgn && c >= (1L << (m - 1))) ? c - (1L << m) : c;
        double a = (double)h.j0 / (double)v;
        if (a > 1.0)
            a = 1.0;
        if (a < -1.0)
            a = -1.0;
        theta[c] = 2.0 * asin(a);
    }
    for (int j = 0; j < m; ++j)
        q[1 + j] = ns + j;
    if (rc >= 0)
        rc = apply_ucry(psi, n, n - 1, q + 1, m, theta);
    /* Uncompute: QFT, the inverse controlled evolutions, H. */
    if (rc >= 0)
        rc = orc_qft((double *)psi, n, ns, m, 0);
    for (int j = m - 1; j >= 0 && rc >= 0; --j) {
        build_u(&h, j, 1, U);
        q[0] = ns + j;
        for (int s = 0; s < ns; ++s)
            q[1 + s] = s;
        rc = apply_matrix(psi, n, q + 1, ns, U, q[0]);
    }
    for (int j = 0; j < m && rc >= 0; ++j)
        rc = gate1(psi, n, ORC_H, ns + j, NULL);
    if (rc < 0) {
        free(psi); free(U); free(q); free(theta); prep_free(&h);
        return rc;
    }
    /* Step 3: read the state.  Postselect ancilla = 1, clock = 0:
     * y_s = psi[2^{n-1} + s]; x is y over s = x_off .. x_off + N - 1 (the
     * second half after the dilation). */
    const long base = 1L << (n - 1);
    const long xb = base + h.x_off;
    double p1 = 0.0, p10 = 0.0, max_imag = 0.0, leak = 0.0, re_norm = 0.0;
    for (long i = base; i < dim; ++i)
        p1 += c_abs2(psi[i]);
    for (int s = 0; s < d; ++s) {
        cplx y = psi[base + s];
        p10 += c_abs2(y);
        if (fabs(y.im) > max_imag)
            max_imag = fabs(y.im);
        if (s < h.x_off || s >= h.x_off + N)
            leak += c_abs2(y);
        else
            re_norm += y.re * y.re;
    }
    re_norm = sqrt(re_norm);
    /* Step 4: the ancilla-1 amplitude of eigen-component i is
     * C b_i / lambda_i, so ||A^{-1} b_hat|| = sqrt(P) / C and
     * x = beta * Re(y) / C (the printed |lambda_0| sqrt(P) is read as
     * sqrt(P) / |lambda_0|, with C standing for lambda_0). */
    for (int s = 0; s < N; ++s) {
        double y = psi[xb + s].re;
        if (x_hhl)
            x_hhl[s] = h.beta * y / h.C;
        if (x_hat)
            x_hat[s] = re_norm > 0.0 ? y / re_norm : 0.0;
    }
    if (psi_out)
        memcpy(psi_out, psi, sizeof(cplx) * (size_t)dim);
    if (info) {
        fill_info(&h, info);
        info->p1 = p1; info->p10 = p10; info->max_imag = max_imag;
        info->pad_leak = sqrt(leak);
        info->x_norm = h.beta * sqrt(p10) / h.C;
    }
    free(psi); free(U); free(q); free(theta); prep_free(&h);
    return ORC_OK;
}

int orc_hhl_solve(const double *A, const double *b, int N, int m, double t,
                  double *psi_out, double *x_hhl, double *x_hat,
                  orc_hhl_info *info)
{
    return orc_hhl_solve_ex(A, b, N, m, t, 0, psi_out, x_hhl, x_hat, info);
}

/* ------------------------------------------------------------------------
 * Newton-Raphson AC power flow (Sec. III), the application the paper's HHL
 * serves: each iteration solves J dx = F for the Jacobian J of the power
 * injections, either exactly (Gaussian elimination) or with HHL.
 *
 * Model: branch (f, t) with series impedance r + jx and total line charging
 * b contributes y = 1 / (r + jx) to Y_ft = Y_tf -= y and y + jb/2 to Y_ff
 * and Y_tt.  Bus i injects P_i = V_i sum_k V_k (G_ik cos d_ik + B_ik sin d_ik)
 * and Q_i = V_i sum_k V_k (G_ik sin d_ik - B_ik cos d_ik), d_ik = a_i - a_k.
 * Unknowns: the angle of every non-slack bus, then the magnitude of every
 * PQ bus (bus order).  F = [P_spec - P; Q_spec - Q] over the same buses, and
 * J = d[P; Q] / d[angles; magnitudes], so the update is x += J^{-1} F.
 * ---------------------------------------------------------------------- */
typedef struct {
    int nb;
    double *G, *B;    /* nb x nb admittance (real, imaginary)            */
    int *ang, *mag;   /* unknown index of bus i's angle / magnitude or -1 */
    int N;            /* number of unknowns                              */
} pf_model;

static void pf_free(pf_model *md)
{
    free(md->G); free(md->B); free(md->ang); free(md->mag);
}

static int pf_build(int nb, int nbr, const int *from, const int *to,
                    const double *r, const double *x, const double *bsh,
                    const int *type, pf_model *md)
{
    memset(md, 0, sizeof(*md));
    if (nb < 2 || nbr < 1)
        return ORC_EINVAL;
    md->nb = nb;
    md->G = (double *)calloc((size_t)nb * nb, sizeof(double));
    md->B = (double *)calloc((size_t)nb * nb, sizeof(double));
    md->ang = (int *)malloc(sizeof(int) * nb);
    md->mag = (int *)malloc(sizeof(int) * nb);
    if (!md->G || !md->B || !md->ang || !md->mag) {
        pf_free(md);
        return ORC_ENOMEM;
    }
    int nslack = 0;
    for (int i = 0; i < nb; ++i) {
        if (type[i] < 0 || type[i] > 2) {
            pf_free(md);
            return ORC_EINVAL;
        }
        nslack += type[i] == 0;
    }
    if (nslack != 1) {
        pf_free(md);
        return ORC_EINVAL;
    }
    for (int e = 0; e < nbr; ++e) {
        const int f = from[e], t = to[e];
        const double den = r[e] * r[e] + x[e] * x[e];
        if (f < 0 || t < 0 || f >= nb || t >= nb || f == t || !(den > 0.0)) {
            pf_free(md);
            return ORC_EINVAL;
        }
        const double g = r[e] / den, bs = -x[e] / den;   /* 1 / (r + jx) */
        md->G[f * nb + t] -= g;  md->B[f * nb + t] -= bs;
        md->G[t * nb + f] -= g;  md->B[t * nb + f] -= bs;
        md->G[f * nb + f] += g;  md->B[f * nb + f] += bs + 0.5 * bsh[e];
        md->G[t * nb + t] += g;  md->B[t * nb + t] += bs + 0.5 * bsh[e];
    }
    int N = 0;
    for (int i = 0; i < nb; ++i)
        md->ang[i] = type[i] != 0 ? N++ : -1;
    for (int i = 0; i < nb; ++i)
        md->mag[i] = type[i] == 2 ? N++ : -1;
    md->N = N;
    return ORC_OK;
}

/* Injections P, Q at every bus for magnitudes vm and angles va. */
static void pf_injections(const pf_model *md, const double *vm,
                          const double *va, double *P, double *Q)
{
    const int nb = md->nb;
    for (int i = 0; i < nb; ++i) {
        double p = 0.0, q = 0.0;
        for (int k = 0; k < nb; ++k) {
            const double g = md->G[i * nb + k], b = md->B[i * nb + k];
            if (g == 0.0 && b == 0.0)
                continue;
            const double d = va[i] - va[k];
            p += vm[k] * (g * cos(d) + b * sin(d));
            q += vm[k] * (g * sin(d) - b * cos(d));
        }
        P[i] = vm[i] * p;
        Q[i] = vm[i] * q;
    }
}

/* F (N) and, if J != NULL, the Jacobian (N x N, row-major). */
static void pf_eval(const pf_model *md, const double *vm, const double *va,
                    const double *pspec, const double *qspec, double *P,
                    double *Q, double *F, double *J)
{
    const int nb = md->nb, N = md->N;
    pf_injections(md, vm, va, P, Q);
    for (int i = 0; i < nb; ++i) {
        if (md->ang[i] >= 0)
            F[md->ang[i]] = pspec[i] - P[i];
        if (md->mag[i] >= 0)
            F[md->mag[i]] = qspec[i] - Q[i];
    }
    if (!J)
        return;
    memset(J, 0, sizeof(double) * (size_t)N * N);
    for (int i = 0; i < nb; ++i) {
        const int rp = md->ang[i], rq = md->mag[i];
        if (rp < 0 && rq < 0)
            continue;
        for (int k = 0; k < nb; ++k) {
            const double g = md->G[i * nb + k], b = md->B[i * nb + k];
            const int ca = md->ang[k], cm = md->mag[k];
            double dPa, dPm, dQa, dQm;   /* d/d angle_k, d/d magnitude_k */
            if (k == i) {
                dPa = -Q[i] - b * vm[i] * vm[i];
                dPm = P[i] / vm[i] + g * vm[i];
                dQa = P[i] - g * vm[i] * vm[i];
                dQm = Q[i] / vm[i] - b * vm[i];
            } else {
                if (g == 0.0 && b == 0.0)
                    continue;
                const double d = va[i] - va[k];
                const double c = cos(d), s = sin(d);
                dPa = vm[i] * vm[k] * (g * s - b * c);
                dPm = vm[i] * (g * c + b * s);
                dQa = -vm[i] * vm[k] * (g * c + b * s);
                dQm = vm[i] * (g * s - b * c);
            }
            if (rp >= 0 && ca >= 0) J[rp * N + ca] = dPa;
            if (rp >= 0 && cm >= 0) J[rp * N + cm] = dPm;
            if (rq >= 0 && ca >= 0) J[rq * N + ca] = dQa;
            if (rq >= 0 && cm >= 0) J[rq * N + cm] = dQm;
        }
    }
}

int orc_pf_eval(int nb, int nbr, const int *from, const int *to,
                const double *r, const double *x, const double *bsh,
                const int *type, const double *pspec, const double *qspec,
                const double *vm, const double *va, double *P, double *Q,
                double *F, double *J)
{
    pf_model md;
    int rc = pf_build(nb, nbr, from, to, r, x, bsh, type, &md);
    if (rc < 0)
        return rc;
    double *Fl = F ? F : (double *)malloc(sizeof(double) * (size_t)(md.N + 1));
    pf_eval(&md, vm, va, pspec, qspec, P, Q, Fl, J);
    if (!F)
        free(Fl);
    rc = md.N;
    pf_free(&md);
    return rc;
}

int orc_pf_newton(int nb, int nbr, const int *from, const int *to,
                  const double *r, const double *x, const double *bsh,
                  const int *type, const double *pspec, const double *qspec,
                  const double *vset, int solver, int m, int flags,
                  int max_iter, double tol, double *vm, double *va,
                  orc_pf_info *info)
{
    pf_model md;
    int rc = pf_build(nb, nbr, from, to, r, x, bsh, type, &md);
    if (rc < 0)
        return rc;
    const int N = md.N;
    double *P = (double *)malloc(sizeof(double) * nb);
    double *Q = (double *)malloc(sizeof(double) * nb);
    double *F = (double *)malloc(sizeof(double) * N);
    double *J = (double *)malloc(sizeof(double) * (size_t)N * N);
    double *dx = (double *)malloc(sizeof(double) * N);
    if (!P || !Q || !F || !J || !dx) {
        free(P); free(Q); free(F); free(J); free(dx); pf_free(&md);
        return ORC_ENOMEM;
    }
    /* flat start: set-point magnitudes at slack and PV buses, 1 elsewhere */
    for (int i = 0; i < nb; ++i) {
        vm[i] = type[i] == 2 ? 1.0 : vset[i];
        va[i] = 0.0;
    }
    if (info)
        memset(info, 0, sizeof(*info));
    int it = 0, conv = 0;
    double worst = 0.0;
    for (;; ++it) {
        pf_eval(&md, vm, va, pspec, qspec, P, Q, F, J);
        worst = 0.0;
        for (int i = 0; i < N; ++i)
            worst = fmax(worst, fabs(F[i]));
        if (info && it < ORC_PF_HISTORY)
            info->history[it] = worst;
        if (worst < tol) {
            conv = 1;
            break;
        }
        if (it >= max_iter)
            break;
        if (solver == 0)
            rc = orc_ge_solve(J, F, N, dx);
        else
            rc = orc_hhl_solve_ex(J, F, N, m, 0.0, flags, NULL, dx, NULL, NULL);
        if (rc < 0)
            break;
        for (int i = 0; i < nb; ++i) {
            if (md.ang[i] >= 0)
                va[i] += dx[md.ang[i]];
            if (md.mag[i] >= 0)
                vm[i] += dx[md.mag[i]];
        }
    }
    if (info) {
        info->iterations = it;
        info->converged = conv;
        info->mismatch = worst;
        info->n_unknowns = N;
    }
    free(P); free(Q); free(F); free(J); free(dx); pf_free(&md);
    return rc < 0 ? rc : ORC_OK;
}
