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

// Householder tridiagonalisation of a symmetric matrix held in its upper
// triangle (row-major, destroyed): A = Q T Q^T, T = tridiag(e, d, e).  Each
// step k forms the reflector I - 2 v v^T that zeroes row k beyond k+1, then
// p = A22 v (symmetric product from the upper triangle), w = p - (v.p) v and
// A22 -= 2 (v w^T + w v^T) on the upper triangle only.  Q is accumulated
// backwards (Q = H_0 (H_1 (... H_{N-3}))), so each reflector touches only the
// trailing block; the result is returned transposed, Zt = Q^T (rows are the
// columns of Q), ready for the row rotations of the QR sweeps.
//
// This and the QR sweeps below are built twice, with AVX2 and for the
// baseline ISA, and the loader picks the AVX2 copy where the CPU has it.
// AVX2 alone brings no fused multiply-add, so both copies round every
// operation alike and give the same bits.  (A clone for a whole CPU
// generation, such as arch=haswell, also asks for RDRND, which virtual
// machines may hide; then the baseline copy would always run.)
__attribute__((target_clones("avx2", "default")))
void tridiagonalise(std::vector<double> &A, int N, std::vector<double> &d, std::vector<double> &e,
                    std::vector<double> &Zt)
{
    d.assign(N, 0.0);
    e.assign(N > 1 ? N - 1 : 0, 0.0);
    std::vector<double> vs((size_t)N * N, 0.0);   // reflector k in row k, entries k+1..N-1
    std::vector<char> used(N, 0);
    std::vector<double> p(N), w(N);
    for (int k = 0; k + 2 < N; ++k) {
        const int L = N - k - 1, o = k + 1;
        double *v = &vs[(size_t)k * N + o];       // v[0..L)
        const double *row = &A[(size_t)k * N + o];
        double xn = 0.0;
        for (int j = 0; j < L; ++j) xn += row[j] * row[j];
        xn = std::sqrt(xn);
        const double alpha = row[0] >= 0.0 ? -xn : xn;
        e[k] = alpha;
        if (xn == 0.0) { e[k] = 0.0; continue; }
        for (int j = 0; j < L; ++j) v[j] = row[j];
        v[0] -= alpha;
        double vn = 0.0;
        for (int j = 0; j < L; ++j) vn += v[j] * v[j];
        vn = std::sqrt(vn);
        if (vn == 0.0) continue;
        const double inv = 1.0 / vn;
        for (int j = 0; j < L; ++j) v[j] *= inv;
        used[k] = 1;
        // p = A22 v from the upper triangle: row i contributes its diagonal,
        // a dot product with v[i+1..] to p[i] and an axpy into p[i+1..].
        std::fill(p.begin(), p.begin() + L, 0.0);
        for (int i = 0; i < L; ++i) {
            const double *ri = &A[(size_t)(o + i) * N + o];
            const double vi = v[i];
            double acc = ri[i] * vi;
            for (int j = i + 1; j < L; ++j) {
                acc += ri[j] * v[j];
                p[j] += ri[j] * vi;
            }
            p[i] += acc;
        }
        double kv = 0.0;
        for (int i = 0; i < L; ++i) kv += v[i] * p[i];
        for (int i = 0; i < L; ++i) w[i] = p[i] - kv * v[i];
        for (int i = 0; i < L; ++i) {
            double *ri = &A[(size_t)(o + i) * N + o];
            const double vi = 2.0 * v[i], wi = 2.0 * w[i];
            for (int j = i; j < L; ++j) ri[j] -= vi * w[j] + wi * v[j];
        }
    }
    for (int k = 0; k < N; ++k) d[k] = A[(size_t)k * N + k];
    if (N >= 2) e[N - 2] = A[(size_t)(N - 2) * N + N - 1];
    // Q = H_0 H_1 ... H_{N-3}, accumulated from the last reflector: M <- H_k M
    // changes rows and columns k+1.. of M only.
    std::vector<double> Q((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) Q[(size_t)i * N + i] = 1.0;
    std::vector<double> s(N);
    for (int k = N - 3; k >= 0; --k) {
        if (!used[k]) continue;
        const int L = N - k - 1, o = k + 1;
        const double *v = &vs[(size_t)k * N + o];
        std::fill(s.begin(), s.begin() + L, 0.0);
        for (int i = 0; i < L; ++i) {           // s = v^T M22
            const double *ri = &Q[(size_t)(o + i) * N + o];
            const double vi = v[i];
            for (int j = 0; j < L; ++j) s[j] += vi * ri[j];
        }
        for (int i = 0; i < L; ++i) {           // M22 -= 2 v s^T
            double *ri = &Q[(size_t)(o + i) * N + o];
            const double vi = 2.0 * v[i];
            for (int j = 0; j < L; ++j) ri[j] -= vi * s[j];
        }
    }
    Zt.resize((size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Zt[(size_t)j * N + i] = Q[(size_t)i * N + j];
}

// Implicit symmetric QR with Wilkinson shifts on T = tridiag(e, d, e)
// (Golub & Van Loan, Alg. 8.3.2): each step chases a bulge down the active
// block with Givens rotations G(p, p+1) = [[c, s], [-s, c]], T <- G T G^T,
// applied to d / e in O(1) and to the rows p, p+1 of Z^T in O(N).
__attribute__((target_clones("avx2", "default")))
bool tridiagonal_qr(std::vector<double> &d, std::vector<double> &e, std::vector<double> &Zt, int N)
{
    const double eps = 2.220446049250313e-16;
    int hi = N - 1, iters = 0;
    while (hi > 0) {
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi]) + std::fabs(d[hi - 1]))) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        if (++iters > 60 * N) return false;
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo]) + std::fabs(d[lo - 1]))) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        const double a = d[hi - 1], b = e[hi - 1], c = d[hi];
        const double dd = 0.5 * (a - c);
        const double mu = c - b * b / (dd + (dd >= 0 ? 1.0 : -1.0) * std::hypot(dd, b));
        double x = d[lo] - mu, z = e[lo], bulge = 0.0;
        for (int p = lo; p < hi; ++p) {
            if (p > lo) {
                x = e[p - 1];
                z = bulge;
            }
            const double r = std::hypot(x, z);
            const double cs = r == 0.0 ? 1.0 : x / r;
            const double sn = r == 0.0 ? 0.0 : z / r;
            if (p > lo) e[p - 1] = r;
            const double a0 = d[p], b0 = e[p], d1 = d[p + 1];
            d[p] = cs * cs * a0 + 2.0 * cs * sn * b0 + sn * sn * d1;
            d[p + 1] = sn * sn * a0 - 2.0 * cs * sn * b0 + cs * cs * d1;
            e[p] = cs * sn * (d1 - a0) + (cs * cs - sn * sn) * b0;
            if (p + 1 < hi) {
                bulge = sn * e[p + 1];
                e[p + 1] = cs * e[p + 1];
            }
            double *zp = &Zt[(size_t)p * N], *zq = &Zt[(size_t)(p + 1) * N];
            for (int i = 0; i < N; ++i) {
                const double u = zp[i], v = zq[i];
                zp[i] = cs * u + sn * v;
                zq[i] = -sn * u + cs * v;
            }
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
    std::vector<double> T = A, d, e, Zt;
    tridiagonalise(T, N, d, e, Zt);
    if (!tridiagonal_qr(d, e, Zt, N)) return false;
    std::vector<int> order(N);
    for (int i = 0; i < N; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int p, int q) { return d[p] < d[q]; });
    w.resize(N);
    V.assign((size_t)N * N, 0.0);
    for (int k = 0; k < N; ++k) {
        w[k] = d[order[k]];
        const double *z = &Zt[(size_t)order[k] * N];
        for (int i = 0; i < N; ++i) V[(size_t)i * N + k] = z[i];
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

}  // namespace

// e^{+iAt 2^j} (or its inverse) from A' = V diag(w) V^T, each power taken
// directly from the eigenvalues with the phase reduced mod 2 pi in double:
// U[a][b] = sum_k V[a][k] V[b][k] e^{+-i phi_k}.  U is symmetric, so only
// b >= a is accumulated (rows of Vt are contiguous: AXPY over b) and mirrored.
std::vector<double> evolution_params(const Spectral &sp, int j, bool inverse)
{
    return evolution_params_pow(sp, std::ldexp(1.0, j), inverse);
}

std::vector<double> evolution_params_pow(const Spectral &sp, double p, bool inverse)
{
    const int D = sp.D;
    const double tj = sp.t * p;
    std::vector<double> cs(D), sn(D);
    for (int k = 0; k < D; ++k) {
        const double ph = std::fmod(sp.w[k] * tj, 2.0 * kPi);
        cs[k] = std::cos(ph);
        sn[k] = inverse ? -std::sin(ph) : std::sin(ph);
    }
    std::vector<double> re((size_t)D * D, 0.0), im((size_t)D * D, 0.0);
    for (int a = 0; a < D; ++a) {
        double *ra = &re[(size_t)a * D], *ia = &im[(size_t)a * D];
        for (int k = 0; k < D; ++k) {
            const double *vk = &sp.Vt[(size_t)k * D];
            const double fc = vk[a] * cs[k], fs = vk[a] * sn[k];
            for (int b = a; b < D; ++b) {
                ra[b] += fc * vk[b];
                ia[b] += fs * vk[b];
            }
        }
    }
    std::vector<double> U((size_t)2 * D * D);
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            const size_t src = a <= b ? (size_t)a * D + b : (size_t)b * D + a;
            U[2 * ((size_t)a * D + b)] = re[src];
            U[2 * ((size_t)a * D + b) + 1] = im[src];
        }
    return U;
}

void materialize(Gate &g, const HHLParams &h)
{
    if (!gate_deferred(g) || !h.spec) return;
    if (g.kind == SV_GATE_MUX2 || g.kind == SV_GATE_MUX3) {
        const std::vector<int> js = gate_evo_js(g);
        for (int v = 1; v < (1 << (int)js.size()); ++v) {
            double p = 0.0;   // sum of 2^j over the controls set in v, lowest first
            for (size_t l = 0; l < js.size(); ++l)
                if ((v >> l) & 1) p += std::ldexp(1.0, js[l]);
            const std::vector<double> u = evolution_params_pow(*h.spec, p, g.evo_inv);
            g.params.insert(g.params.end(), u.begin(), u.end());
        }
        return;
    }
    g.params = evolution_params(*h.spec, g.evo_j, g.evo_inv);
}

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

namespace {

// Step 1a with the Gauss-Seidel splitting A = (D + L) + U: the system becomes
// (D + L)^{-1} A x = (D + L)^{-1} b.  Rows of X = (D + L)^{-1} [A | b] by
// forward substitution, X_i = (row_i - sum_{k<i} a_ik X_k) / a_ii, each
// update an AXPY over a contiguous row.  False on a zero diagonal entry.
bool gauss_seidel_precondition(const double *A, const double *b, int dim, std::vector<double> &At,
                               std::vector<double> &bt)
{
    const size_t w = (size_t)dim + 1;  // [A | b]
    std::vector<double> X((size_t)dim * w);
    for (int i = 0; i < dim; ++i) {
        const double d = A[(size_t)i * dim + i];
        if (d == 0.0) return false;
        double *xi = &X[(size_t)i * w];
        for (int j = 0; j < dim; ++j) xi[j] = A[(size_t)i * dim + j];
        xi[dim] = b[i];
        for (int k = 0; k < i; ++k) {
            const double l = A[(size_t)i * dim + k];
            if (l == 0.0) continue;
            const double *xk = &X[(size_t)k * w];
            for (size_t j = 0; j < w; ++j) xi[j] -= l * xk[j];
        }
        const double inv = 1.0 / d;
        for (size_t j = 0; j < w; ++j) xi[j] *= inv;
    }
    At.assign((size_t)dim * dim, 0.0);
    bt.assign(dim, 0.0);
    for (int i = 0; i < dim; ++i) {
        for (int j = 0; j < dim; ++j) At[(size_t)i * dim + j] = X[(size_t)i * w + j];
        bt[i] = X[(size_t)i * w + dim];
    }
    return true;
}

}  // namespace

extern "C" sv_status circuit_build_hhl(const double *A, const double *b, int dim,
                                       int clock_bits, double t, sv_circuit **out)
{
    return circuit_build_hhl_ex(A, b, dim, clock_bits, t, 0, out);
}

extern "C" sv_status circuit_build_hhl_ex(const double *A, const double *b, int dim,
                                          int clock_bits, double t, int flags, sv_circuit **out)
{
    if (!out) return fail(SV_ERR_INVALID, "circuit_build_hhl: out is NULL");
    *out = nullptr;
    if (!A || !b) return fail(SV_ERR_INVALID, "circuit_build_hhl: A or b is NULL");
    if (dim < 1 || dim > (1 << 16)) return fail(SV_ERR_INVALID, "circuit_build_hhl: dim out of range");
    const int m = clock_bits;
    if (m < 1 || m > 16) return fail(SV_ERR_INVALID, "circuit_build_hhl: clock_bits must be in [1, 16]");
    if (!std::isfinite(t)) return fail(SV_ERR_INVALID, "circuit_build_hhl: t is not finite");
    if (flags & ~(SV_HHL_DEVICE_EVOLUTIONS | SV_HHL_SIGNED | SV_HHL_DILATE | SV_HHL_AUTO | SV_HHL_GAUSS_SEIDEL))
        return fail(SV_ERR_INVALID, "circuit_build_hhl_ex: unknown flags");
    std::vector<double> Ags, bgs;
    if (flags & SV_HHL_GAUSS_SEIDEL) {
        for (int i = 0; i < dim; ++i)
            if (!std::isfinite(A[(size_t)i * dim + i]) || !std::isfinite(b[i]))
                return fail(SV_ERR_INVALID, "circuit_build_hhl: non-finite input");
        if (!gauss_seidel_precondition(A, b, dim, Ags, bgs))
            return fail(SV_ERR_SINGULAR, "circuit_build_hhl: Gauss-Seidel needs a nonzero diagonal");
        A = Ags.data();
        b = bgs.data();
        flags |= SV_HHL_DILATE;
    }

    // Step 1: inspect A (finite, symmetric?) and b.
    double amax = 0.0, asym = 0.0;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            const double aij = A[(size_t)i * dim + j];
            if (!std::isfinite(aij)) return fail(SV_ERR_INVALID, "circuit_build_hhl: A has non-finite entries");
            amax = std::max(amax, std::fabs(aij));
            asym = std::max(asym, std::fabs(aij - A[(size_t)j * dim + i]));
        }
    const bool symmetric = asym <= 1e-12 * amax;
    const bool autoflags = (flags & SV_HHL_AUTO) != 0;
    const bool dilate = (flags & SV_HHL_DILATE) || (autoflags && !symmetric);
    bool sgn = dilate || (flags & SV_HHL_SIGNED);
    if (!dilate && !symmetric) return fail(SV_ERR_NOT_SYMMETRIC, "circuit_build_hhl: A is not symmetric");
    double bb = 0.0;
    for (int i = 0; i < dim; ++i) {
        if (!std::isfinite(b[i])) return fail(SV_ERR_INVALID, "circuit_build_hhl: b has non-finite entries");
        bb += b[i] * b[i];
    }
    const double beta = std::sqrt(bb);
    if (!(beta > 0.0)) return fail(SV_ERR_INVALID, "circuit_build_hhl: b is zero");

    // Step 1b: pad to a power of two with a unit diagonal and zero entries
    // of b; step 1c: replace the padded A' by [[0, A'], [A'^T, 0]] and b by
    // [b; 0], so that x comes out in the second half.
    const int na = dilate ? ceil_log2(dim) : std::max(1, ceil_log2(dim));
    const int ns = dilate ? na + 1 : na;
    const int n = ns + m + 1;
    if (n > kMaxQubits) return fail(SV_ERR_INVALID, "circuit_build_hhl: more than 34 qubits");
    if (ns > kMaxDenseQubits) return fail(SV_ERR_INVALID, "circuit_build_hhl: system register wider than 12 qubits");
    const int P = 1 << na;
    const int D = 1 << ns;
    std::vector<double> Ap((size_t)D * D, 0.0), bh(D, 0.0);
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            const double a = (i < dim && j < dim) ? A[(size_t)i * dim + j] : (i == j ? 1.0 : 0.0);
            if (dilate) {
                Ap[(size_t)i * D + P + j] = a;
                Ap[(size_t)(P + j) * D + i] = a;
            } else {
                Ap[(size_t)i * D + j] = a;
            }
        }
    for (int i = 0; i < dim; ++i) bh[i] = b[i] / beta;

    // Spectral parameters over the eigenvectors b reaches (|lambda| with the
    // sign qubit, whose clock spends one bit on the sign).
    std::vector<double> w, V;
    if (!sym_eig(Ap, D, w, V)) return fail(SV_ERR_INVALID, "circuit_build_hhl: eigensolver did not converge");
    std::vector<char> reached(D, 0);
    bool any = false;
    double lo = 0.0, hi = 0.0, wmin = 0.0;
    for (int k = 0; k < D; ++k) {
        double ov = 0.0;
        for (int i = 0; i < D; ++i) ov += V[(size_t)i * D + k] * bh[i];
        if (ov * ov > 1e-20) {
            reached[k] = 1;
            if (!any || w[k] < wmin) wmin = w[k];
            any = true;
        }
    }
    if (!any) return fail(SV_ERR_INVALID, "circuit_build_hhl: b reaches no eigenvector");
    if (autoflags && wmin <= 0.0) sgn = true;
    bool first = true;
    for (int k = 0; k < D; ++k) {
        if (!reached[k]) continue;
        const double l = sgn ? std::fabs(w[k]) : w[k];
        if (first || l < lo) lo = l;
        if (first || l > hi) hi = l;
        first = false;
    }
    if (sgn && m < 2) return fail(SV_ERR_INVALID, "circuit_build_hhl: the sign qubit needs clock_bits >= 2");
    if (sgn && !(lo > 0.0))
        return fail(SV_ERR_SINGULAR, "circuit_build_hhl: b reaches a zero eigenvalue");
    if (!(lo > 0.0))
        return fail(SV_ERR_NOT_POSDEF, "circuit_build_hhl: A is not positive definite on the span of b");
    const double kappa = hi / lo;
    const double two_m = std::ldexp(1.0, m);
    const double top = std::ldexp(1.0, sgn ? m - 1 : m) - 1.0;
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
    h.x_off = dilate ? P : 0;
    h.sign_qubit = sgn;
    h.dilated = dilate;
    h.preconditioned = (flags & SV_HHL_GAUSS_SEIDEL) != 0;
    {
        int nd, nq, nt;
        sv_qubit_estimate(D, std::max(1.0, kappa), sgn ? 1 : 0, &nd, &nq, &nt);
        h.n_qpe_est = nq;
    }
    {
        auto sp = std::make_shared<Spectral>();
        sp->D = D;
        sp->w = w;
        sp->t = tt;
        sp->Vt.resize((size_t)D * D);
        for (int k = 0; k < D; ++k)
            for (int i = 0; i < D; ++i) sp->Vt[(size_t)k * D + i] = V[(size_t)i * D + k];
        h.spec = sp;
    }
    const bool defer = (flags & SV_HHL_DEVICE_EVOLUTIONS) != 0;
    auto evo = [&](int ctl, int j, bool inverse) {
        Gate g;
        g.kind = SV_GATE_CDENSE;
        g.qubits = {ctl};
        for (int q = 0; q < ns; ++q) g.qubits.push_back(q);
        g.evo_j = j;
        g.evo_inv = inverse;
        if (!defer) g.params = evolution_params(*h.spec, j, inverse);
        c.gates.push_back(std::move(g));
    };

    // |b> on the system register.
    add_state_prep(c, bh, ns);
    // Phase estimation with controlled e^{iAt 2^j}.
    for (int j = 0; j < m; ++j) add(c, SV_GATE_H, {ns + j});
    for (int j = 0; j < m; ++j) evo(ns + j, j, false);
    add_qft(c, ns, m, true);
    // Eigenvalue inversion: clock value c decodes to v (c itself, or its
    // two's-complement value with the sign qubit) standing for
    // lambda = C v / j0, and the ancilla's |1> amplitude becomes
    // C / lambda = j0 / v, clamped to [-1, 1].
    {
        std::vector<double> theta((size_t)1 << m);
        theta[0] = 0.0;
        const long long half = 1ll << (m - 1);
        for (size_t cv = 1; cv < theta.size(); ++cv) {
            const long long v = (sgn && (long long)cv >= half) ? (long long)cv - 2 * half : (long long)cv;
            const double a = std::max(-1.0, std::min(1.0, double(j0) / double(v)));
            theta[cv] = 2.0 * std::asin(a);
        }
        std::vector<int> q{n - 1};
        for (int j = 0; j < m; ++j) q.push_back(ns + j);
        add(c, SV_GATE_UCRY, q, theta);
    }
    // Uncompute.
    add_qft(c, ns, m, false);
    for (int j = m - 1; j >= 0; --j) evo(ns + j, j, true);
    for (int j = 0; j < m; ++j) add(c, SV_GATE_H, {ns + j});
    *out = sc;
    return SV_OK;
}
