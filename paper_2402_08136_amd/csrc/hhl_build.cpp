// Host side of the HHL path: step-1 preparation, spectral parameters and the
// circuit of Fig. 5 (Zheng et al., PESGM 2024, Sec. III-A), built in double
// precision in C++ (the paper names a C++ generator as its future work,
// Sec. V, because Python circuit generation was its bottleneck, Table I).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace hhlsv {

namespace {

constexpr double kPi = 3.14159265358979323846;

inline double &at(std::vector<double> &M, int N, int i, int j) { return M[(size_t)i * N + j]; }

// Householder reduction of a symmetric matrix to tridiagonal form T with
// A = Z T Z^T (Golub & Van Loan, Sec. 8.3.1).  T and Z are dense N x N.
void tridiagonalise(std::vector<double> &T, std::vector<double> &Z, int N)
{
    Z.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) at(Z, N, i, i) = 1.0;
    std::vector<double> v(N);
    for (int k = 0; k + 2 < N; ++k) {
        const int L = N - k - 1;  // reflector acts on indices k+1..N-1
        double xn = 0.0;
        for (int j = 0; j < L; ++j) xn += at(T, N, k + 1 + j, k) * at(T, N, k + 1 + j, k);
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const double x0 = at(T, N, k + 1, k);
        const double alpha = x0 >= 0.0 ? -xn : xn;
        for (int j = 0; j < L; ++j) v[j] = at(T, N, k + 1 + j, k);
        v[0] -= alpha;
        double vn = 0.0;
        for (int j = 0; j < L; ++j) vn += v[j] * v[j];
        vn = std::sqrt(vn);
        if (vn == 0.0) continue;
        for (int j = 0; j < L; ++j) v[j] /= vn;
        // T <- H T H with H = I - 2 v v^T on the trailing indices.
        for (int i = 0; i < N; ++i) {      // columns
            double s = 0.0;
            for (int j = 0; j < L; ++j) s += at(T, N, i, k + 1 + j) * v[j];
            for (int j = 0; j < L; ++j) at(T, N, i, k + 1 + j) -= 2.0 * s * v[j];
        }
        for (int i = 0; i < N; ++i) {      // rows
            double s = 0.0;
            for (int j = 0; j < L; ++j) s += v[j] * at(T, N, k + 1 + j, i);
            for (int j = 0; j < L; ++j) at(T, N, k + 1 + j, i) -= 2.0 * s * v[j];
        }
        for (int i = 0; i < N; ++i) {      // Z <- Z H
            double s = 0.0;
            for (int j = 0; j < L; ++j) s += at(Z, N, i, k + 1 + j) * v[j];
            for (int j = 0; j < L; ++j) at(Z, N, i, k + 1 + j) -= 2.0 * s * v[j];
        }
        for (int j = 1; j < L; ++j) at(T, N, k + 1 + j, k) = at(T, N, k, k + 1 + j) = 0.0;
        at(T, N, k + 1, k) = at(T, N, k, k + 1) = alpha;
    }
}

// Rotate rows and columns p, p+1 of T (T <- G T G^T) and columns of Z.
void rotate(std::vector<double> &T, std::vector<double> &Z, int N, int p,
            double c, double s)
{
    for (int i = 0; i < N; ++i) {
        const double a = at(T, N, p, i), b = at(T, N, p + 1, i);
        at(T, N, p, i) = c * a + s * b;
        at(T, N, p + 1, i) = -s * a + c * b;
    }
    for (int i = 0; i < N; ++i) {
        const double a = at(T, N, i, p), b = at(T, N, i, p + 1);
        at(T, N, i, p) = c * a + s * b;
        at(T, N, i, p + 1) = -s * a + c * b;
    }
    for (int i = 0; i < N; ++i) {
        const double a = at(Z, N, i, p), b = at(Z, N, i, p + 1);
        at(Z, N, i, p) = c * a + s * b;
        at(Z, N, i, p + 1) = -s * a + c * b;
    }
}

// Implicit symmetric QR with Wilkinson shifts on a tridiagonal T, chasing the
// bulge with Givens rotations (Golub & Van Loan, Alg. 8.3.2/8.3.3).
bool tridiagonal_qr(std::vector<double> &T, std::vector<double> &Z, int N)
{
    const double eps = 2.220446049250313e-16;
    int hi = N - 1, iters = 0;
    while (hi > 0) {
        if (std::fabs(at(T, N, hi, hi - 1)) <=
            eps * (std::fabs(at(T, N, hi, hi)) + std::fabs(at(T, N, hi - 1, hi - 1)))) {
            at(T, N, hi, hi - 1) = at(T, N, hi - 1, hi) = 0.0;
            --hi;
            continue;
        }
        if (++iters > 60 * N) return false;
        int lo = hi - 1;
        while (lo > 0 && std::fabs(at(T, N, lo, lo - 1)) >
                             eps * (std::fabs(at(T, N, lo, lo)) + std::fabs(at(T, N, lo - 1, lo - 1))))
            --lo;
        if (lo > 0) at(T, N, lo, lo - 1) = at(T, N, lo - 1, lo) = 0.0;
        // Wilkinson shift from the trailing 2x2 block.
        const double a = at(T, N, hi - 1, hi - 1), b = at(T, N, hi, hi - 1), c = at(T, N, hi, hi);
        const double d = 0.5 * (a - c);
        const double mu = c - b * b / (d + (d >= 0 ? 1.0 : -1.0) * std::hypot(d, b));
        double x = at(T, N, lo, lo) - mu, z = at(T, N, lo + 1, lo);
        for (int p = lo; p < hi; ++p) {
            if (p > lo) {
                x = at(T, N, p, p - 1);
                z = at(T, N, p + 1, p - 1);
            }
            const double r = std::hypot(x, z);
            const double cs = r == 0.0 ? 1.0 : x / r;
            const double sn = r == 0.0 ? 0.0 : z / r;
            rotate(T, Z, N, p, cs, sn);
            if (p > lo) at(T, N, p + 1, p - 1) = at(T, N, p - 1, p + 1) = 0.0;
        }
    }
    return true;
}

int ceil_log2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

}  // namespace

bool sym_eig(const std::vector<double> &A, int N, std::vector<double> &w,
             std::vector<double> &V)
{
    std::vector<double> T = A, Z;
    tridiagonalise(T, Z, N);
    if (!tridiagonal_qr(T, Z, N)) return false;
    std::vector<int> order(N);
    for (int i = 0; i < N; ++i) order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](int p, int q) { return at(T, N, p, p) < at(T, N, q, q); });
    w.resize(N);
    V.assign((size_t)N * N, 0.0);
    for (int k = 0; k < N; ++k) {
        w[k] = at(T, N, order[k], order[k]);
        for (int i = 0; i < N; ++i) V[(size_t)i * N + k] = at(Z, N, i, order[k]);
    }
    return true;
}

namespace {

void add(Circuit &c, int kind, std::vector<int> q, std::vector<double> p = {})
{
    Gate g;
    g.kind = kind;
    g.qubits = std::move(q);
    g.params = std::move(p);
    c.gates.push_back(std::move(g));
}

// |b> preparation for a real unit vector a (2^ns entries) from |0>: one
// uniformly controlled RY per system qubit, top qubit first.  On qubit q the
// rotation for higher-bit value v splits the weight of the block
// [v 2^{q+1}, (v+1) 2^{q+1}) between its halves; on qubit 0 the angle is
// signed (atan2 of the two amplitudes), which carries the signs of b
// (uniformly controlled rotations, Mottonen et al. 2004).
void add_state_prep(Circuit &c, const std::vector<double> &a, int ns)
{
    for (int q = ns - 1; q >= 0; --q) {
        const int r = ns - 1 - q;                // controls q+1..ns-1
        std::vector<double> theta((size_t)1 << r);
        const size_t half = (size_t)1 << q;
        for (size_t v = 0; v < theta.size(); ++v) {
            const size_t base = v << (q + 1);
            if (q == 0) {
                theta[v] = 2.0 * std::atan2(a[base + 1], a[base]);
            } else {
                double lo = 0.0, hi = 0.0;
                for (size_t i = 0; i < half; ++i) {
                    lo += a[base + i] * a[base + i];
                    hi += a[base + half + i] * a[base + half + i];
                }
                theta[v] = 2.0 * std::atan2(std::sqrt(hi), std::sqrt(lo));
            }
        }
        std::vector<int> qs{q};
        for (int l = 0; l < r; ++l) qs.push_back(q + 1 + l);
        add(c, SV_GATE_UCRY, qs, theta);
    }
}

// QFT on clock qubits q0..q0+m-1 as H / controlled-phase / SWAP gates, with
// QFT|x> = 2^{-m/2} sum_y e^{+2 pi i x y / 2^m}|y>; inverse = reversed order,
// negated phases.
void add_qft(Circuit &c, int q0, int m, bool inverse)
{
    std::vector<Gate> seq;
    for (int j = m - 1; j >= 0; --j) {
        seq.push_back(Gate{SV_GATE_H, {q0 + j}, {}});
        for (int k = j - 1; k >= 0; --k)
            seq.push_back(Gate{SV_GATE_CP, {q0 + k, q0 + j}, {kPi / double(1L << (j - k))}});
    }
    for (int j = 0; j < m / 2; ++j)
        seq.push_back(Gate{SV_GATE_SWAP, {q0 + j, q0 + m - 1 - j}, {}});
    if (inverse) {
        std::reverse(seq.begin(), seq.end());
        for (auto &g : seq)
            if (g.kind == SV_GATE_CP) g.params[0] = -g.params[0];
    }
    for (auto &g : seq) c.gates.push_back(std::move(g));
}

// e^{+i A t 2^j} (or its inverse) from A = V diag(w) V^T, each power taken
// directly from the eigenvalues (phase reduced mod 2 pi in double).
std::vector<double> evolution(const std::vector<double> &w, const std::vector<double> &V,
                              int D, double tj, bool inverse)
{
    std::vector<double> cs(D), sn(D);
    for (int k = 0; k < D; ++k) {
        const double ph = std::fmod(w[k] * tj, 2.0 * kPi);
        cs[k] = std::cos(ph);
        sn[k] = inverse ? -std::sin(ph) : std::sin(ph);
    }
    std::vector<double> U((size_t)2 * D * D);
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < D; ++k) {
                const double vv = V[(size_t)a * D + k] * V[(size_t)b * D + k];
                re += vv * cs[k];
                im += vv * sn[k];
            }
            U[2 * ((size_t)a * D + b)] = re;
            U[2 * ((size_t)a * D + b) + 1] = im;
        }
    return U;
}

}  // namespace

}  // namespace hhlsv

using namespace hhlsv;

extern "C" sv_status sv_qubit_estimate(int dim, double kappa, int has_negative,
                                       int *n_data, int *n_qpe, int *n_total)
{
    if (dim < 1 || !(kappa >= 1.0) || !std::isfinite(kappa))
        return fail(SV_ERR_INVALID, "sv_qubit_estimate: need dim >= 1 and finite kappa >= 1");
    const int nd = ceil_log2(dim);
    const int qk = (int)std::ceil(std::log2(kappa + 1.0));
    const int nq = std::max(nd + 1, qk) + (has_negative ? 1 : 0);
    if (n_data) *n_data = nd;
    if (n_qpe) *n_qpe = nq;
    if (n_total) *n_total = nd + nq + 1;
    return SV_OK;
}

extern "C" sv_status circuit_build_hhl(const double *A, const double *b, int dim,
                                       int clock_bits, double t, sv_circuit **out)
{
    if (!out) return fail(SV_ERR_INVALID, "circuit_build_hhl: out is NULL");
    *out = nullptr;
    if (!A || !b) return fail(SV_ERR_INVALID, "circuit_build_hhl: A or b is NULL");
    if (dim < 1 || dim > (1 << 16)) return fail(SV_ERR_INVALID, "circuit_build_hhl: dim out of range");
    const int m = clock_bits;
    if (m < 1 || m > 16) return fail(SV_ERR_INVALID, "circuit_build_hhl: clock_bits must be in [1, 16]");
    const int ns = std::max(1, ceil_log2(dim));
    const int n = ns + m + 1;
    if (n > kMaxQubits) return fail(SV_ERR_INVALID, "circuit_build_hhl: more than 34 qubits");
    if (ns > kMaxDenseQubits) return fail(SV_ERR_INVALID, "circuit_build_hhl: system register wider than 12 qubits");
    if (!std::isfinite(t)) return fail(SV_ERR_INVALID, "circuit_build_hhl: t is not finite");

    // Step 1: symmetry (the Hermitian case), ||b||, pad to 2^ns with a unit
    // diagonal and zero entries of b.
    double amax = 0.0, asym = 0.0;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            const double aij = A[(size_t)i * dim + j];
            if (!std::isfinite(aij)) return fail(SV_ERR_INVALID, "circuit_build_hhl: A has non-finite entries");
            amax = std::max(amax, std::fabs(aij));
            asym = std::max(asym, std::fabs(aij - A[(size_t)j * dim + i]));
        }
    if (asym > 1e-12 * amax) return fail(SV_ERR_NOT_SYMMETRIC, "circuit_build_hhl: A is not symmetric");
    double bb = 0.0;
    for (int i = 0; i < dim; ++i) {
        if (!std::isfinite(b[i])) return fail(SV_ERR_INVALID, "circuit_build_hhl: b has non-finite entries");
        bb += b[i] * b[i];
    }
    const double beta = std::sqrt(bb);
    if (!(beta > 0.0)) return fail(SV_ERR_INVALID, "circuit_build_hhl: b is zero");
    const int D = 1 << ns;
    std::vector<double> Ap((size_t)D * D, 0.0), bh(D, 0.0);
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j)
            Ap[(size_t)i * D + j] = (i < dim && j < dim) ? A[(size_t)i * dim + j] : (i == j ? 1.0 : 0.0);
    for (int i = 0; i < dim; ++i) bh[i] = b[i] / beta;

    // Spectral parameters.
    std::vector<double> w, V;
    if (!sym_eig(Ap, D, w, V)) return fail(SV_ERR_INVALID, "circuit_build_hhl: eigensolver did not converge");
    bool any = false;
    double lo = 0.0, hi = 0.0;
    for (int k = 0; k < D; ++k) {
        double ov = 0.0;
        for (int i = 0; i < D; ++i) ov += V[(size_t)i * D + k] * bh[i];
        if (ov * ov > 1e-20) {
            if (!any || w[k] < lo) lo = w[k];
            if (!any || w[k] > hi) hi = w[k];
            any = true;
        }
    }
    if (!any || !(lo > 0.0))
        return fail(SV_ERR_NOT_POSDEF, "circuit_build_hhl: A is not positive definite on the span of b");
    const double kappa = hi / lo;
    const double two_m = std::ldexp(1.0, m);
    const double top = two_m - 1.0;
    double tt = t;
    if (!(tt > 0.0)) {
        if (kappa <= top) {
            const double j0f = std::floor(top / kappa);
            tt = 2.0 * kPi * j0f / (two_m * lo);
        } else {
            tt = 2.0 * kPi * top / (two_m * hi);
        }
    }
    const double jr = std::round(lo * tt * two_m / (2.0 * kPi));
    const int j0 = jr < 1.0 ? 1 : (int)jr;
    const double C = 2.0 * kPi * j0 / (tt * two_m);

    auto *sc = new (std::nothrow) sv_circuit;
    if (!sc) return fail(SV_ERR_OOM, "circuit_build_hhl: out of host memory");
    Circuit &c = sc->c;
    c.n = n;
    HHLParams &h = c.hhl;
    h.is_hhl = true;
    h.dim = dim; h.ns = ns; h.m = m; h.j0 = j0;
    h.t = tt; h.C = C; h.lambda_lo = lo; h.lambda_hi = hi; h.kappa = kappa; h.b_norm = beta;
    {
        int nd, nq, nt;
        sv_qubit_estimate(D, std::max(1.0, kappa), 0, &nd, &nq, &nt);
        h.n_qpe_est = nq;
    }

    std::vector<int> sys(ns);
    for (int s = 0; s < ns; ++s) sys[s] = s;
    auto ctrl_sys = [&](int ctl) {
        std::vector<int> q{ctl};
        q.insert(q.end(), sys.begin(), sys.end());
        return q;
    };
    // |b> on the system register.
    add_state_prep(c, bh, ns);
    // Phase estimation with controlled e^{iAt 2^j}.
    for (int j = 0; j < m; ++j) add(c, SV_GATE_H, {ns + j});
    for (int j = 0; j < m; ++j)
        add(c, SV_GATE_CDENSE, ctrl_sys(ns + j), evolution(w, V, D, tt * std::ldexp(1.0, j), false));
    add_qft(c, ns, m, true);
    // Eigenvalue inversion: clock value c stands for lambda = C c / j0, and
    // the ancilla's |1> amplitude becomes C / lambda = j0 / c (clamped).
    {
        std::vector<double> theta((size_t)1 << m);
        theta[0] = 0.0;
        for (size_t cv = 1; cv < theta.size(); ++cv)
            theta[cv] = 2.0 * std::asin(std::min(1.0, double(j0) / double(cv)));
        std::vector<int> q{n - 1};
        for (int j = 0; j < m; ++j) q.push_back(ns + j);
        add(c, SV_GATE_UCRY, q, theta);
    }
    // Uncompute.
    add_qft(c, ns, m, false);
    for (int j = m - 1; j >= 0; --j)
        add(c, SV_GATE_CDENSE, ctrl_sys(ns + j), evolution(w, V, D, tt * std::ldexp(1.0, j), true));
    for (int j = 0; j < m; ++j) add(c, SV_GATE_H, {ns + j});
    *out = sc;
    return SV_OK;
}
