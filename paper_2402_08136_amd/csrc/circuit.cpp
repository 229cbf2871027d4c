// Circuit IR, its ABI calls, and the gate-fusion pass.
//
// Gate fusion follows the idea of Sec. II-C / Fig. 4 (Zheng et al., PESGM
// 2024): several gates are replaced by one gate, which cuts the number of
// state-vector sweeps.  The paper's four strategies (1q-1q, 1q into 2q from
// either side, 2q-2q) are the k_max = 2 case of the greedy pass below, which
// merges into one dense 2^k x 2^k gate any run of gates whose joint qubit
// set stays within k_max qubits.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.hpp"

namespace hhlsv {

namespace {
thread_local std::string g_last_error;
constexpr double kSqrtHalf = 0.70710678118654752440;
}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

sv_status fail(sv_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

int gate_nparams_named(int kind)
{
    switch (kind) {
    case SV_GATE_H: case SV_GATE_X: case SV_GATE_CX: case SV_GATE_SWAP: return 0;
    case SV_GATE_RY: case SV_GATE_RZ: case SV_GATE_P: case SV_GATE_CP: return 1;
    case SV_GATE_U3: return 3;
    default: return -1;
    }
}

bool gate_is_diagonal(int kind)
{
    return kind == SV_GATE_RZ || kind == SV_GATE_P || kind == SV_GATE_CP || kind == SV_GATE_DIAG;
}

static int gate_width(int kind)
{
    switch (kind) {
    case SV_GATE_H: case SV_GATE_X: case SV_GATE_RY: case SV_GATE_RZ:
    case SV_GATE_P: case SV_GATE_U3: return 1;
    case SV_GATE_CX: case SV_GATE_CP: case SV_GATE_SWAP: return 2;
    default: return -1;
    }
}

sv_status validate_gate(int n, int kind, const int *qubits, int nq,
                        const double *params, int nparams)
{
    if (kind < SV_GATE_H || kind > SV_GATE_MUX3)
        return fail(SV_ERR_INVALID, "circuit_add_gate: unknown gate kind");
    if (nq < 1 || !qubits) return fail(SV_ERR_INVALID, "circuit_add_gate: no qubits");
    if (nparams < 0 || (nparams > 0 && !params))
        return fail(SV_ERR_INVALID, "circuit_add_gate: bad params");
    for (int i = 0; i < nq; ++i) {
        if (qubits[i] < 0 || qubits[i] >= n) return fail(SV_ERR_INVALID, "circuit_add_gate: qubit out of range");
        for (int j = 0; j < i; ++j)
            if (qubits[i] == qubits[j]) return fail(SV_ERR_INVALID, "circuit_add_gate: repeated qubit");
    }
    for (int i = 0; i < nparams; ++i)
        if (!std::isfinite(params[i])) return fail(SV_ERR_INVALID, "circuit_add_gate: non-finite parameter");
    const int w = gate_width(kind);
    if (w > 0) {
        if (nq != w) return fail(SV_ERR_INVALID, "circuit_add_gate: wrong number of qubits for gate kind");
        if (nparams != gate_nparams_named(kind))
            return fail(SV_ERR_INVALID, "circuit_add_gate: wrong number of params for gate kind");
        return SV_OK;
    }
    if (kind == SV_GATE_DENSE || kind == SV_GATE_DIAG) {
        if (nq > kMaxDenseQubits) return fail(SV_ERR_INVALID, "circuit_add_gate: gate wider than 12 qubits");
        const long need = kind == SV_GATE_DENSE ? 2L << (2 * nq) : 2L << nq;
        if (nparams != need) return fail(SV_ERR_INVALID, "circuit_add_gate: params must hold the complex matrix");
        return SV_OK;
    }
    if (kind == SV_GATE_CDENSE) {
        const int k = nq - 1;
        if (k < 1 || k > kMaxDenseQubits) return fail(SV_ERR_INVALID, "circuit_add_gate: CDENSE needs 1..12 targets");
        if (nparams != (2L << (2 * k))) return fail(SV_ERR_INVALID, "circuit_add_gate: params must hold the complex matrix");
        return SV_OK;
    }
    if (kind == SV_GATE_MUX2 || kind == SV_GATE_MUX3) {
        const int r = kind == SV_GATE_MUX2 ? 2 : 3, k = nq - r;
        if (k < 1 || k > kMaxDenseQubits) return fail(SV_ERR_INVALID, "circuit_add_gate: MUX needs 1..12 targets");
        if (nparams != ((1L << r) - 1) * (2L << (2 * k)))
            return fail(SV_ERR_INVALID, "circuit_add_gate: MUX params must hold 2^r - 1 complex matrices");
        return SV_OK;
    }
    // UCRY
    const int r = nq - 1;
    if (r > kMaxUcryControls) return fail(SV_ERR_INVALID, "circuit_add_gate: UCRY with more than 20 controls");
    if (nparams != (1L << r)) return fail(SV_ERR_INVALID, "circuit_add_gate: UCRY needs 2^r angles");
    return SV_OK;
}

std::vector<cd> gate_matrix(const Gate &g)
{
    const auto &p = g.params;
    switch (g.kind) {
    case SV_GATE_H:
        return {cd(kSqrtHalf, 0), cd(kSqrtHalf, 0), cd(kSqrtHalf, 0), cd(-kSqrtHalf, 0)};
    case SV_GATE_X:
        return {0.0, 1.0, 1.0, 0.0};
    case SV_GATE_RY: {
        const double c = std::cos(0.5 * p[0]), s = std::sin(0.5 * p[0]);
        return {c, -s, s, c};
    }
    case SV_GATE_U3: {
        const double c = std::cos(0.5 * p[0]), s = std::sin(0.5 * p[0]);
        return {cd(c, 0), -std::polar(s, p[2]), std::polar(s, p[1]), std::polar(c, p[1] + p[2])};
    }
    case SV_GATE_CX: {  // list (control, target): index r = bit_c + 2 bit_t
        std::vector<cd> M(16, 0.0);
        M[0 * 4 + 0] = M[2 * 4 + 2] = 1.0;
        M[1 * 4 + 3] = M[3 * 4 + 1] = 1.0;
        return M;
    }
    case SV_GATE_SWAP: {
        std::vector<cd> M(16, 0.0);
        M[0 * 4 + 0] = M[3 * 4 + 3] = 1.0;
        M[1 * 4 + 2] = M[2 * 4 + 1] = 1.0;
        return M;
    }
    case SV_GATE_DENSE: {
        std::vector<cd> M(p.size() / 2);
        for (size_t i = 0; i < M.size(); ++i) M[i] = cd(p[2 * i], p[2 * i + 1]);
        return M;
    }
    case SV_GATE_CDENSE: {  // block-diag(I, U) over (c, targets): r = bit_c + 2 r_t
        const int k = (int)g.qubits.size() - 1;
        const size_t K = (size_t)1 << k, D = 2 * K;
        std::vector<cd> M(D * D, 0.0);
        for (size_t r = 0; r < K; ++r) {
            M[(2 * r) * D + 2 * r] = 1.0;
            for (size_t c = 0; c < K; ++c)
                M[(2 * r + 1) * D + (2 * c + 1)] = cd(p[2 * (r * K + c)], p[2 * (r * K + c) + 1]);
        }
        return M;
    }
    case SV_GATE_MUX2:
    case SV_GATE_MUX3: {  // block-diag(I, U_1, ..) over (controls, targets): r = v + V r_t
        const size_t V = (size_t)1 << gate_controls(g);
        const int k = (int)g.qubits.size() - gate_controls(g);
        const size_t K = (size_t)1 << k, D = V * K;
        std::vector<cd> M(D * D, 0.0);
        for (size_t r = 0; r < K; ++r) {
            M[(V * r) * D + V * r] = 1.0;
            for (size_t v = 1; v < V; ++v)
                for (size_t c = 0; c < K; ++c) {
                    const size_t at = 2 * ((v - 1) * K * K + r * K + c);
                    M[(V * r + v) * D + (V * c + v)] = cd(p[at], p[at + 1]);
                }
        }
        return M;
    }
    case SV_GATE_UCRY: {  // over (t, c...): r = bit_t + 2 v
        const int rr = (int)g.qubits.size() - 1;
        const size_t V = (size_t)1 << rr, D = 2 * V;
        std::vector<cd> M(D * D, 0.0);
        for (size_t v = 0; v < V; ++v) {
            const double c = std::cos(0.5 * p[v]), s = std::sin(0.5 * p[v]);
            M[(2 * v) * D + 2 * v] = c;
            M[(2 * v) * D + 2 * v + 1] = -s;
            M[(2 * v + 1) * D + 2 * v] = s;
            M[(2 * v + 1) * D + 2 * v + 1] = c;
        }
        return M;
    }
    default: {  // diagonal kinds
        std::vector<cd> d = gate_diagonal(g);
        std::vector<cd> M(d.size() * d.size(), 0.0);
        for (size_t i = 0; i < d.size(); ++i) M[i * d.size() + i] = d[i];
        return M;
    }
    }
}

std::vector<cd> gate_diagonal(const Gate &g)
{
    const auto &p = g.params;
    switch (g.kind) {
    case SV_GATE_RZ: return {std::polar(1.0, -0.5 * p[0]), std::polar(1.0, 0.5 * p[0])};
    case SV_GATE_P: return {1.0, std::polar(1.0, p[0])};
    case SV_GATE_CP: return {1.0, 1.0, 1.0, std::polar(1.0, p[0])};
    case SV_GATE_DIAG: {
        std::vector<cd> d(p.size() / 2);
        for (size_t i = 0; i < d.size(); ++i) d[i] = cd(p[2 * i], p[2 * i + 1]);
        return d;
    }
    default: return {};
    }
}

namespace {

// ---------------------------------------------------------------- fusion --
struct Block {
    std::vector<int> qubits;     // sorted
    std::vector<cd> M;           // dense: 2^k x 2^k over sorted qubits
    std::vector<cd> dv;          // a merged diagonal block: its 2^k entries (M unused)
    bool diag = true;
    bool open = true;            // false: a gate too wide to fuse, kept as is
    bool alive = true;
    Gate orig;                   // for closed blocks
};

// Embed a matrix over qubit list gq (index sum_l bit(gq_l) 2^l) into the
// sorted qubit set U: identity on U \ gq.
std::vector<cd> embed(const std::vector<cd> &G, const std::vector<int> &gq,
                      const std::vector<int> &U)
{
    const int u = (int)U.size();
    const size_t D = (size_t)1 << u;
    const size_t K = (size_t)1 << gq.size();
    std::vector<int> pos(gq.size());
    size_t gmask = 0;
    for (size_t l = 0; l < gq.size(); ++l) {
        pos[l] = (int)(std::find(U.begin(), U.end(), gq[l]) - U.begin());
        gmask |= (size_t)1 << pos[l];
    }
    auto sub = [&](size_t R) {
        size_t r = 0;
        for (size_t l = 0; l < gq.size(); ++l) r |= ((R >> pos[l]) & 1) << l;
        return r;
    };
    std::vector<cd> E(D * D, 0.0);
    for (size_t R = 0; R < D; ++R)
        for (size_t Cc = 0; Cc < D; ++Cc)
            if ((R & ~gmask) == (Cc & ~gmask)) E[R * D + Cc] = G[sub(R) * K + sub(Cc)];
    return E;
}

// C = A B for D x D complex matrices, row by row: C[i][.] += A[i][k] B[k][.]
// for k in increasing order, skipping zero A[i][k].  The complex product is
// written out in real arithmetic, (ar br - ai bi, ar bi + ai br), which is
// what std::complex computes for finite operands, so that the row update
// vectorises; built for AVX2 (no fused multiply-add, so the same bits) and
// for the baseline ISA.
__attribute__((target_clones("avx2", "default")))
void matmul_rows(const double *A, const double *B, double *C, size_t D)
{
    for (size_t i = 0; i < D; ++i) {
        double *c = C + 2 * i * D;
        for (size_t k = 0; k < D; ++k) {
            const double ar = A[2 * (i * D + k)], ai = A[2 * (i * D + k) + 1];
            if (ar == 0.0 && ai == 0.0) continue;
            const double *b = B + 2 * k * D;
            for (size_t j = 0; j < D; ++j) {
                const double br = b[2 * j], bi = b[2 * j + 1];
                c[2 * j] += ar * br - ai * bi;
                c[2 * j + 1] += ar * bi + ai * br;
            }
        }
    }
}

std::vector<cd> matmul(const std::vector<cd> &A, const std::vector<cd> &B, size_t D)
{
    std::vector<cd> C(D * D, 0.0);
    matmul_rows(reinterpret_cast<const double *>(A.data()), reinterpret_cast<const double *>(B.data()),
                reinterpret_cast<double *>(C.data()), D);
    return C;
}

std::vector<int> unite(const std::vector<int> &a, const std::vector<int> &b)
{
    std::vector<int> u = a;
    u.insert(u.end(), b.begin(), b.end());
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    return u;
}

// Blocks examined, most recent first, for a merge with a disjoint block.
constexpr int kDisjointLookback = 32;

// Second pass over the fused blocks: a block that shares no qubit with a
// later block, and that no block in between touches, commutes up to it; the
// two become one block on the union of their qubits while that stays within
// k_max (a layer of one-qubit gates on distinct qubits becomes one sweep).
// Done after the overlap merges so that it never takes a gate away from a
// block that shares its qubits.
void merge_disjoint(std::vector<Block> &blocks, int n, int k_max)
{
    std::vector<int> last(n, -1);
    for (int j = 0; j < (int)blocks.size(); ++j) {
        Block &bj = blocks[j];
        if (!bj.alive) continue;
        if (bj.open) {
            int seen = 0;
            for (int i = j - 1; i >= 0 && seen < kDisjointLookback && (int)bj.qubits.size() < k_max; --i) {
                Block &bi = blocks[i];
                if (!bi.alive) continue;
                ++seen;
                if (!bi.open || (int)(bi.qubits.size() + bj.qubits.size()) > k_max) continue;
                bool ok = true;
                for (int q : bi.qubits)
                    ok = ok && last[q] == i && !std::binary_search(bj.qubits.begin(), bj.qubits.end(), q);
                if (!ok) continue;
                const std::vector<int> U = unite(bi.qubits, bj.qubits);
                const size_t D = (size_t)1 << U.size();
                bj.M = matmul(embed(bj.M, bj.qubits, U), embed(bi.M, bi.qubits, U), D);
                bj.diag = bj.diag && bi.diag;
                bj.qubits = U;
                bi.alive = false;
                for (int q : bi.qubits) last[q] = j;
            }
        }
        for (int q : bj.qubits) last[q] = j;
    }
}

// Third pass: diagonal blocks merge with each other past everything they
// commute with, up to kDiagFuseMax qubits (beyond k_max: a diagonal costs
// one sweep whatever its width, its table 2^k entries).  The inverse QFT's
// controlled phases, for instance, come out of the first passes as runs of
// 5-qubit diagonals on the clock register between its Hadamards.
constexpr int kDiagFuseMax = 10;
constexpr int kDiagLookback = 64;

// Whether a diagonal operator on the sorted qubits dq commutes with block b:
// b is diagonal, or every qubit it shares with dq is one b only reads as a
// control (a controlled dense gate's control, a uniformly controlled
// rotation's controls: both are block-diagonal in those qubits' basis).
bool diag_commutes(const std::vector<int> &dq, const Block &b)
{
    if (b.open ? b.diag : gate_is_diagonal(b.orig.kind)) return true;
    std::vector<int> moved = b.qubits;   // qubits b does not act on diagonally
    if (!b.open && b.orig.kind == SV_GATE_CDENSE) moved.assign(b.orig.qubits.begin() + 1, b.orig.qubits.end());
    if (!b.open && b.orig.kind == SV_GATE_UCRY) moved.assign(1, b.orig.qubits[0]);
    for (int q : moved)
        if (std::binary_search(dq.begin(), dq.end(), q)) return false;
    return true;
}

// The diagonal entries of an open diagonal block (index bit l = qubits[l]).
std::vector<cd> diag_entries(const Block &b)
{
    if (!b.dv.empty()) return b.dv;
    const size_t D = (size_t)1 << b.qubits.size();
    std::vector<cd> d(D);
    for (size_t i = 0; i < D; ++i) d[i] = b.M[i * D + i];
    return d;
}

void merge_diagonals(std::vector<Block> &blocks)
{
    for (int j = 0; j < (int)blocks.size(); ++j) {
        Block &bj = blocks[j];
        if (!bj.alive || !bj.open || !bj.diag) continue;
        int seen = 0;
        for (int i = j - 1; i >= 0 && seen < kDiagLookback; --i) {
            Block &bi = blocks[i];
            if (!bi.alive) continue;
            ++seen;
            if (bi.open && bi.diag) {
                const std::vector<int> U = unite(bi.qubits, bj.qubits);
                if ((int)U.size() <= kDiagFuseMax) {
                    // bj commutes with every block between: apply it right
                    // after bi, i.e. multiply the two diagonals entry by entry
                    const std::vector<cd> di = diag_entries(bi), dj = diag_entries(bj);
                    // position in U of each qubit of a block, found once
                    auto positions = [&](const std::vector<int> &qs) {
                        std::vector<int> pos(qs.size());
                        for (size_t l = 0; l < qs.size(); ++l)
                            pos[l] = (int)(std::find(U.begin(), U.end(), qs[l]) - U.begin());
                        return pos;
                    };
                    const std::vector<int> pi = positions(bi.qubits), pj = positions(bj.qubits);
                    auto index_in = [](const std::vector<int> &pos, size_t R) {
                        size_t r = 0;
                        for (size_t l = 0; l < pos.size(); ++l) r |= ((R >> pos[l]) & 1) << l;
                        return r;
                    };
                    std::vector<cd> d((size_t)1 << U.size());
                    for (size_t R = 0; R < d.size(); ++R) d[R] = dj[index_in(pj, R)] * di[index_in(pi, R)];
                    bi.dv = std::move(d);
                    bi.M.clear();
                    bi.qubits = U;
                    bj.alive = false;
                    break;
                }
            }
            if (!diag_commutes(bj.qubits, bi)) break;
        }
    }
}

// Last pass: up to three controlled dense gates in a row on the same
// targets (the controlled e^{iAt 2^j} of phase estimation) become one MUX3
// or MUX2 gate: one sweep instead of three or two, over the 7/8 or 3/4 of
// the state where some control is 1 instead of three or two halves.  Up to
// kMuxMaxTargets targets.
constexpr int kMuxMaxTargets = 6;

// The MUX gate of the controlled gates gs (applied in that order, same
// targets, distinct controls, all deferred evolutions or none): control l
// is gs[l]'s, and U_v is the product of the gates set in v, later gates on
// the left; for evolutions e^{iAt p_v} from the eigen-decomposition.
Gate make_mux(const std::vector<const Gate *> &gs, const HHLParams &h)
{
    const int r = (int)gs.size();
    Gate m;
    m.kind = r == 2 ? SV_GATE_MUX2 : SV_GATE_MUX3;
    for (const Gate *g : gs) m.qubits.push_back(g->qubits[0]);
    m.qubits.insert(m.qubits.end(), gs[0]->qubits.begin() + 1, gs[0]->qubits.end());
    bool evolutions = h.spec != nullptr;
    for (const Gate *g : gs) evolutions = evolutions && g->evo_j >= 0 && g->evo_inv == gs[0]->evo_inv;
    if (evolutions) {
        m.evo_j = gs[0]->evo_j;
        m.evo_j2 = gs[1]->evo_j;
        if (r == 3) m.evo_j3 = gs[2]->evo_j;
        m.evo_inv = gs[0]->evo_inv;
        // deferred: the device builds the tables; eager: the same tables on
        // the host (materialize), so both forms hold the same matrices
        if (!gate_deferred(*gs[0])) materialize(m, h);
        return m;
    }
    const size_t K = (size_t)1 << (gs[0]->qubits.size() - 1);
    std::vector<std::vector<cd>> u(r, std::vector<cd>(K * K));
    for (int l = 0; l < r; ++l)
        for (size_t i = 0; i < K * K; ++i) u[l][i] = cd(gs[l]->params[2 * i], gs[l]->params[2 * i + 1]);
    for (int v = 1; v < (1 << r); ++v) {
        std::vector<cd> P;
        for (int l = 0; l < r; ++l)
            if ((v >> l) & 1) P = P.empty() ? u[l] : matmul(u[l], P, K);
        for (const cd &x : P) {
            m.params.push_back(x.real());
            m.params.push_back(x.imag());
        }
    }
    return m;
}

void merge_controlled_runs(std::vector<Block> &blocks, const HHLParams &h)
{
    std::vector<int> run;   // live candidate blocks in a row, mergeable with each other
    auto flush = [&]() {
        size_t at = 0;
        while (run.size() - at >= 2) {
            const size_t take = std::min<size_t>(3, run.size() - at);
            std::vector<const Gate *> gs;
            for (size_t l = 0; l < take; ++l) gs.push_back(&blocks[run[at + l]].orig);
            Gate m = make_mux(gs, h);
            Block &b0 = blocks[run[at]];
            for (size_t l = 1; l < take; ++l) {
                b0.qubits = unite(b0.qubits, blocks[run[at + l]].qubits);
                blocks[run[at + l]].alive = false;
            }
            b0.orig = std::move(m);
            at += take;
        }
        run.clear();
    };
    for (int j = 0; j < (int)blocks.size(); ++j) {
        Block &bj = blocks[j];
        if (!bj.alive) continue;
        const Gate &b = bj.orig;
        const int nt = (int)b.qubits.size() - 1;
        const bool cand = !bj.open && b.kind == SV_GATE_CDENSE && nt >= 2 && nt <= kMuxMaxTargets;
        bool joins = cand && !run.empty();
        if (joins) {
            const Gate &a = blocks[run[0]].orig;
            joins = a.qubits.size() == b.qubits.size() &&
                    std::equal(a.qubits.begin() + 1, a.qubits.end(), b.qubits.begin() + 1) &&
                    gate_deferred(a) == gate_deferred(b) && a.evo_inv == b.evo_inv;
            for (int ri : run) joins = joins && blocks[ri].orig.qubits[0] != b.qubits[0];
        }
        if (!joins) flush();
        if (cand) run.push_back(j);
    }
    flush();
}

int fused_width(const Gate &g)
{
    return (int)g.qubits.size();
}

}  // namespace

}  // namespace hhlsv

using namespace hhlsv;

extern "C" const char *sv_last_error(void) { return g_last_error.c_str(); }

extern "C" sv_status circuit_create(int n_qubits, sv_circuit **out)
{
    if (!out) return fail(SV_ERR_INVALID, "circuit_create: out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > kMaxQubits) return fail(SV_ERR_INVALID, "circuit_create: n must be in [1, 34]");
    auto *c = new (std::nothrow) sv_circuit;
    if (!c) return fail(SV_ERR_OOM, "circuit_create: out of host memory");
    c->c.n = n_qubits;
    *out = c;
    return SV_OK;
}

extern "C" sv_status circuit_add_gate(sv_circuit *c, int kind, const int *qubits, int nq,
                                      const double *params, int nparams)
{
    if (!c) return fail(SV_ERR_INVALID, "circuit_add_gate: circuit is NULL");
    sv_status st = validate_gate(c->c.n, kind, qubits, nq, params, nparams);
    if (st != SV_OK) return st;
    {
        std::lock_guard<std::mutex> lk(c->c.dev_mu);
        if (!c->c.dev.empty())
            return fail(SV_ERR_INVALID, "circuit_add_gate: circuit already applied; it is read-only now");
    }
    Gate g;
    g.kind = kind;
    g.qubits.assign(qubits, qubits + nq);
    if (nparams) g.params.assign(params, params + nparams);
    c->c.gates.push_back(std::move(g));
    return SV_OK;
}

extern "C" sv_status circuit_info(const sv_circuit *c, sv_hhl_info *out)
{
    if (!c || !out) return fail(SV_ERR_INVALID, "circuit_info: NULL argument");
    std::memset(out, 0, sizeof(*out));
    const HHLParams &h = c->c.hhl;
    out->n_total = c->c.n;
    out->n_gates = (int)c->c.gates.size();
    if (h.is_hhl) {
        out->n_sys = h.ns;
        out->n_clock = h.m;
        out->n_qpe_est = h.n_qpe_est;
        out->dim = h.dim;
        out->j0 = h.j0;
        out->t = h.t;
        out->C = h.C;
        out->lambda_lo = h.lambda_lo;
        out->lambda_hi = h.lambda_hi;
        out->kappa = h.kappa;
        out->b_norm = h.b_norm;
        out->x_offset = h.x_off;
        out->sign_qubit = h.sign_qubit ? 1 : 0;
        out->dilated = h.dilated ? 1 : 0;
        out->preconditioned = h.preconditioned ? 1 : 0;
    }
    return SV_OK;
}

extern "C" sv_status circuit_shape(const sv_circuit *c, int *n_qubits, int *n_gates)
{
    if (!c) return fail(SV_ERR_INVALID, "circuit_shape: NULL circuit");
    if (n_qubits) *n_qubits = c->c.n;
    if (n_gates) *n_gates = (int)c->c.gates.size();
    return SV_OK;
}

extern "C" sv_status circuit_serialize(const sv_circuit *c, void *buf, size_t *len)
{
    if (!c || !len) return fail(SV_ERR_INVALID, "circuit_serialize: NULL argument");
    size_t need = 8;
    for (const auto &g : c->c.gates) {
        size_t np = g.params.size();
        if (gate_deferred(g))
            np = (size_t)gate_matrices(g) * ((size_t)2 << (2 * (g.qubits.size() - gate_controls(g))));
        need += 12 + 4 * g.qubits.size() + 8 * np;
    }
    if (!buf) {
        *len = need;
        return SV_OK;
    }
    if (*len < need) {
        *len = need;
        return fail(SV_ERR_INVALID, "circuit_serialize: buffer too small");
    }
    char *p = static_cast<char *>(buf);
    auto put32 = [&](int32_t v) { std::memcpy(p, &v, 4); p += 4; };
    put32(c->c.n);
    put32((int32_t)c->c.gates.size());
    for (const auto &g0 : c->c.gates) {
        Gate tmp;
        if (gate_deferred(g0)) {
            tmp = g0;
            materialize(tmp, c->c.hhl);
        }
        const Gate &g = gate_deferred(g0) ? tmp : g0;
        put32(g.kind);
        put32((int32_t)g.qubits.size());
        put32((int32_t)g.params.size());
        for (int q : g.qubits) put32(q);
        std::memcpy(p, g.params.data(), 8 * g.params.size());
        p += 8 * g.params.size();
    }
    *len = need;
    return SV_OK;
}

extern "C" sv_status fuse(const sv_circuit *in, int k_max, sv_circuit **out)
{
    if (!in || !out) return fail(SV_ERR_INVALID, "fuse: NULL argument");
    *out = nullptr;
    if (k_max < 1 || k_max > 5) return fail(SV_ERR_INVALID, "fuse: k_max must be in [1, 5]");
    const int n = in->c.n;
    // SWAP gates become a relabelling of the qubits instead of a sweep: the
    // gates after a swap are applied with its two qubits exchanged (an exact
    // permutation of the amplitudes).  Whatever permutation remains at the
    // end is undone by swaps, so the fused circuit leaves every amplitude
    // where the input circuit does; in HHL the inverse QFT's swap layer and
    // the QFT's cancel, and no swap is left.
    std::vector<Gate> gates;
    gates.reserve(in->c.gates.size());
    {
        std::vector<int> phys(n);   // logical qubit -> where its data is
        for (int q = 0; q < n; ++q) phys[q] = q;
        for (const Gate &g : in->c.gates) {
            if (g.kind == SV_GATE_SWAP) {
                std::swap(phys[g.qubits[0]], phys[g.qubits[1]]);
                continue;
            }
            Gate r = g;
            for (int &q : r.qubits) q = phys[q];
            gates.push_back(std::move(r));
        }
        std::vector<int> logical(n);   // data position -> logical qubit
        for (int q = 0; q < n; ++q) logical[phys[q]] = q;
        for (int p = 0; p < n; ++p) {
            while (logical[p] != p) {
                // move logical qubit logical[p] home to position logical[p]
                const int q = logical[p];
                Gate sw;
                sw.kind = SV_GATE_SWAP;
                sw.qubits = {p, q};
                gates.push_back(sw);
                std::swap(logical[p], logical[q]);
            }
        }
    }
    std::vector<Block> blocks;
    blocks.reserve(gates.size());
    std::vector<int> last(n, -1);

    for (const Gate &g0 : gates) {
        const int w = fused_width(g0);
        Gate tmp;
        if (w <= k_max && gate_deferred(g0)) {  // merged on the host: build its matrix here
            tmp = g0;
            materialize(tmp, in->c.hhl);
        }
        const Gate &g = (w <= k_max && gate_deferred(g0)) ? tmp : g0;
        if (w > k_max) {
            Block b;
            b.qubits = g.qubits;
            std::sort(b.qubits.begin(), b.qubits.end());
            b.open = false;
            b.diag = false;
            b.orig = g;
            blocks.push_back(std::move(b));
            for (int q : g.qubits) last[q] = (int)blocks.size() - 1;
            continue;
        }
        std::vector<int> S = g.qubits;
        std::sort(S.begin(), S.end());
        // Candidate blocks: open blocks that are the last block on every one
        // of their qubits and on at least one qubit of g.  Such a block can
        // move past everything after it, so it may be merged with g.
        std::vector<int> cand;
        for (int q : S) {
            const int bi = last[q];
            if (bi < 0 || !blocks[bi].open) continue;
            if (std::find(cand.begin(), cand.end(), bi) != cand.end()) continue;
            bool frontier = true;
            for (int bq : blocks[bi].qubits) frontier = frontier && last[bq] == bi;
            if (frontier) cand.push_back(bi);
        }
        std::vector<int> chosen;
        {
            std::vector<int> U = S;
            for (int bi : cand) U = unite(U, blocks[bi].qubits);
            if ((int)U.size() <= k_max) {
                chosen = cand;
            } else {
                int best = -1;
                size_t best_w = 0;
                for (int bi : cand) {
                    const auto u = unite(S, blocks[bi].qubits);
                    if ((int)u.size() <= k_max && u.size() > best_w) {
                        best = bi;
                        best_w = u.size();
                    }
                }
                if (best >= 0) chosen.push_back(best);
            }
        }
        Block nb;
        nb.qubits = S;
        for (int bi : chosen) nb.qubits = unite(nb.qubits, blocks[bi].qubits);
        const size_t D = (size_t)1 << nb.qubits.size();
        // M = E_g E_{b_last} ... E_{b_first}; the first factor is taken as
        // is rather than multiplied into the identity (a product that could
        // only change the sign of zero entries)
        std::vector<cd> M;
        nb.diag = gate_is_diagonal(g.kind);
        for (int bi : chosen) {  // disjoint, so their order does not matter
            std::vector<cd> E = embed(blocks[bi].M, blocks[bi].qubits, nb.qubits);
            M = M.empty() ? std::move(E) : matmul(E, M, D);
            nb.diag = nb.diag && blocks[bi].diag;
            blocks[bi].alive = false;
        }
        std::vector<cd> E = embed(gate_matrix(g), g.qubits, nb.qubits);
        M = M.empty() ? std::move(E) : matmul(E, M, D);
        nb.M = std::move(M);
        blocks.push_back(std::move(nb));
        for (int q : blocks.back().qubits) last[q] = (int)blocks.size() - 1;
    }

    merge_disjoint(blocks, n, k_max);
    merge_diagonals(blocks);
    merge_controlled_runs(blocks, in->c.hhl);

    auto *oc = new (std::nothrow) sv_circuit;
    if (!oc) return fail(SV_ERR_OOM, "fuse: out of host memory");
    oc->c.n = n;
    oc->c.hhl = in->c.hhl;
    for (auto &b : blocks) {
        if (!b.alive) continue;
        if (!b.open) {
            oc->c.gates.push_back(b.orig);
            continue;
        }
        Gate g;
        g.qubits = b.qubits;
        const size_t D = (size_t)1 << b.qubits.size();
        if (b.diag) {
            g.kind = SV_GATE_DIAG;
            g.params.resize(2 * D);
            const std::vector<cd> d = diag_entries(b);
            for (size_t i = 0; i < D; ++i) {
                g.params[2 * i] = d[i].real();
                g.params[2 * i + 1] = d[i].imag();
            }
        } else {
            g.kind = SV_GATE_DENSE;
            g.params.resize(2 * D * D);
            for (size_t i = 0; i < D * D; ++i) {
                g.params[2 * i] = b.M[i].real();
                g.params[2 * i + 1] = b.M[i].imag();
            }
        }
        oc->c.gates.push_back(std::move(g));
    }
    *out = oc;
    return SV_OK;
}

extern "C" sv_status circuit_destroy(sv_circuit *c)
{
    delete c;
    return SV_OK;
}
