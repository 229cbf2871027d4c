// Newton-Raphson AC power flow with HHL as the linear solver: the power-flow
// application the HHL path serves (Zheng et al., PESGM 2024, Sec. III).  The
// Jacobian system of every iteration is handed to the HHL circuit builder
// (dilated or Gauss-Seidel preconditioned, since the Jacobian is not
// symmetric), run on the GPU and read back by postselection.
//
// Model, in complex form: bus admittance Y from the branch list (series
// y = 1/(r + jx), line charging jb/2 at both ends), bus injections
// S = diag(V) conj(Y V).  With I = Y V and E = diag(V / |V|):
//   dS/d angle     = j diag(V) conj(diag(I) - Y diag(V))
//   dS/d magnitude = diag(V) conj(Y E) + conj(diag(I)) E
// (derivatives of S with respect to the polar coordinates of V).  Unknowns:
// angles of the non-slack buses, then magnitudes of the PQ buses, in bus
// order; mismatch F = [P_spec - P; Q_spec - Q] over the same buses; the
// update is x += J^{-1} F with J the derivative of [P; Q].
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace hhlsv {
namespace {

using cplx = std::complex<double>;

struct PFModel {
    int nb = 0, N = 0;
    std::vector<cplx> Y;        // nb x nb, row-major
    std::vector<int> ang, mag;  // unknown index of bus i's angle / magnitude, or -1
};

sv_status build_model(int nb, int nbr, const int *from, const int *to, const double *r, const double *x,
                      const double *bsh, const int *type, PFModel &md)
{
    if (nb < 2 || nbr < 1) return fail(SV_ERR_INVALID, "power flow: need at least 2 buses and 1 branch");
    if (!from || !to || !r || !x || !bsh || !type) return fail(SV_ERR_INVALID, "power flow: NULL array");
    int nslack = 0;
    for (int i = 0; i < nb; ++i) {
        if (type[i] < 0 || type[i] > 2) return fail(SV_ERR_INVALID, "power flow: bus type must be 0, 1 or 2");
        nslack += type[i] == 0;
    }
    if (nslack != 1) return fail(SV_ERR_INVALID, "power flow: exactly one slack bus is required");
    md.nb = nb;
    md.Y.assign((size_t)nb * nb, cplx(0, 0));
    for (int e = 0; e < nbr; ++e) {
        const int f = from[e], t = to[e];
        if (f < 0 || t < 0 || f >= nb || t >= nb || f == t)
            return fail(SV_ERR_INVALID, "power flow: branch endpoints out of range");
        const cplx z(r[e], x[e]);
        if (!(std::norm(z) > 0.0) || !std::isfinite(std::norm(z)) || !std::isfinite(bsh[e]))
            return fail(SV_ERR_INVALID, "power flow: branch impedance must be finite and nonzero");
        const cplx y = 1.0 / z, half(0.0, 0.5 * bsh[e]);
        md.Y[(size_t)f * nb + f] += y + half;
        md.Y[(size_t)t * nb + t] += y + half;
        md.Y[(size_t)f * nb + t] -= y;
        md.Y[(size_t)t * nb + f] -= y;
    }
    md.ang.assign(nb, -1);
    md.mag.assign(nb, -1);
    int N = 0;
    for (int i = 0; i < nb; ++i)
        if (type[i] != 0) md.ang[i] = N++;
    for (int i = 0; i < nb; ++i)
        if (type[i] == 2) md.mag[i] = N++;
    md.N = N;
    return SV_OK;
}

// F (N) and optionally J (N x N); P, Q (nb) receive the injections.
void evaluate(const PFModel &md, const double *vm, const double *va, const double *pspec, const double *qspec,
              double *P, double *Q, double *F, double *J)
{
    const int nb = md.nb, N = md.N;
    std::vector<cplx> V(nb), I(nb, cplx(0, 0));
    for (int i = 0; i < nb; ++i) V[i] = std::polar(vm[i], va[i]);
    for (int i = 0; i < nb; ++i)
        for (int k = 0; k < nb; ++k) I[i] += md.Y[(size_t)i * nb + k] * V[k];
    for (int i = 0; i < nb; ++i) {
        const cplx S = V[i] * std::conj(I[i]);
        P[i] = S.real();
        Q[i] = S.imag();
        if (md.ang[i] >= 0) F[md.ang[i]] = pspec[i] - P[i];
        if (md.mag[i] >= 0) F[md.mag[i]] = qspec[i] - Q[i];
    }
    if (!J) return;
    std::memset(J, 0, sizeof(double) * (size_t)N * N);
    for (int i = 0; i < nb; ++i) {
        const int rp = md.ang[i], rq = md.mag[i];
        if (rp < 0 && rq < 0) continue;
        for (int k = 0; k < nb; ++k) {
            const cplx yik = md.Y[(size_t)i * nb + k];
            if (k != i && yik == cplx(0, 0)) continue;
            const cplx ek = V[k] / vm[k];
            // column k of dS/d angle and dS/d magnitude, row i
            cplx dsa = cplx(0, 1) * V[i] * std::conj(-yik * V[k]);
            cplx dsm = V[i] * std::conj(yik * ek);
            if (k == i) {
                dsa += cplx(0, 1) * V[i] * std::conj(I[i]);
                dsm += std::conj(I[i]) * ek;
            }
            const int ca = md.ang[k], cm = md.mag[k];
            if (rp >= 0 && ca >= 0) J[(size_t)rp * N + ca] = dsa.real();
            if (rp >= 0 && cm >= 0) J[(size_t)rp * N + cm] = dsm.real();
            if (rq >= 0 && ca >= 0) J[(size_t)rq * N + ca] = dsa.imag();
            if (rq >= 0 && cm >= 0) J[(size_t)rq * N + cm] = dsm.imag();
        }
    }
}

}  // namespace
}  // namespace hhlsv

using namespace hhlsv;

extern "C" sv_status pf_mismatch_jacobian(int n_bus, int n_branch, const int *from, const int *to, const double *r,
                                          const double *x, const double *b_charging, const int *bus_type,
                                          const double *p_spec, const double *q_spec, const double *vm,
                                          const double *va, double *P, double *Q, double *F, double *J,
                                          int *n_unknowns)
{
    PFModel md;
    sv_status st = build_model(n_bus, n_branch, from, to, r, x, b_charging, bus_type, md);
    if (st != SV_OK) return st;
    if (n_unknowns) *n_unknowns = md.N;
    if (!F && !J && !P && !Q) return SV_OK;
    if (!p_spec || !q_spec || !vm || !va) return fail(SV_ERR_INVALID, "pf_mismatch_jacobian: NULL input");
    std::vector<double> Pl(n_bus), Ql(n_bus), Fl(md.N);
    evaluate(md, vm, va, p_spec, q_spec, P ? P : Pl.data(), Q ? Q : Ql.data(), F ? F : Fl.data(), J);
    return SV_OK;
}

extern "C" sv_status pf_newton_hhl(int n_bus, int n_branch, const int *from, const int *to, const double *r,
                                   const double *x, const double *b_charging, const int *bus_type,
                                   const double *p_spec, const double *q_spec, const double *v_set, int clock_bits,
                                   int hhl_flags, sv_dtype dtype, int k_max, int max_iter, double tol, double *vm,
                                   double *va, pf_info *info)
{
    if (!p_spec || !q_spec || !v_set || !vm || !va) return fail(SV_ERR_INVALID, "pf_newton_hhl: NULL argument");
    if (max_iter < 0 || max_iter > 1000 || !(tol > 0.0))
        return fail(SV_ERR_INVALID, "pf_newton_hhl: max_iter in [0, 1000] and tol > 0");
    if (k_max < 0 || k_max > 5) return fail(SV_ERR_INVALID, "pf_newton_hhl: k_max in [0, 5]");
    if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_ERR_INVALID, "pf_newton_hhl: bad dtype");
    const int allowed = SV_HHL_DEVICE_EVOLUTIONS | SV_HHL_DILATE | SV_HHL_AUTO | SV_HHL_GAUSS_SEIDEL;
    if (hhl_flags & ~allowed) return fail(SV_ERR_INVALID, "pf_newton_hhl: HHL flags");
    // the Jacobian is not symmetric: without a choice, dilate
    if (!(hhl_flags & (SV_HHL_DILATE | SV_HHL_AUTO | SV_HHL_GAUSS_SEIDEL))) hhl_flags |= SV_HHL_DILATE;
    PFModel md;
    sv_status st = build_model(n_bus, n_branch, from, to, r, x, b_charging, bus_type, md);
    if (st != SV_OK) return st;
    const int nb = n_bus, N = md.N;
    if (info) std::memset(info, 0, sizeof(*info));
    for (int i = 0; i < nb; ++i) {
        vm[i] = bus_type[i] == 2 ? 1.0 : v_set[i];   // flat start
        va[i] = 0.0;
    }
    std::vector<double> P(nb), Q(nb), F(N), J((size_t)N * N), xh(N);
    sv_state *state = nullptr;
    int state_n = 0;
    double hhl_s = 0.0, worst = 0.0;
    int it = 0;
    bool conv = false;
    for (;; ++it) {
        evaluate(md, vm, va, p_spec, q_spec, P.data(), Q.data(), F.data(), J.data());
        worst = 0.0;
        for (double f : F) worst = std::max(worst, std::fabs(f));
        if (info && it < PF_HISTORY) info->history[it] = worst;
        if (worst < tol) {
            conv = true;
            break;
        }
        if (it >= max_iter) break;
        const auto t0 = std::chrono::steady_clock::now();
        sv_circuit *c = nullptr, *run = nullptr;
        st = circuit_build_hhl_ex(J.data(), F.data(), N, clock_bits, 0.0, hhl_flags, &c);
        if (st == SV_OK && k_max > 0) st = fuse(c, k_max, &run);
        int n = 0;
        if (st == SV_OK) st = circuit_shape(c, &n, nullptr);
        if (st == SV_OK && n != state_n) {
            sv_destroy(state);
            state = nullptr;
            st = sv_create(n, dtype, &state);
            state_n = st == SV_OK ? n : 0;
        } else if (st == SV_OK) {
            st = sv_reset(state);
        }
        sv_solution_info si;
        if (st == SV_OK) st = sv_apply(state, run ? run : c);
        if (st == SV_OK) st = sv_postselect_solution(state, c, xh.data(), N, &si);
        if (run) circuit_destroy(run);
        if (c) circuit_destroy(c);
        hhl_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (st != SV_OK) break;
        for (int i = 0; i < nb; ++i) {
            if (md.ang[i] >= 0) va[i] += si.scale * xh[md.ang[i]];
            if (md.mag[i] >= 0) vm[i] += si.scale * xh[md.mag[i]];
        }
    }
    sv_destroy(state);
    if (info) {
        info->iterations = it;
        info->converged = conv ? 1 : 0;
        info->n_unknowns = N;
        info->mismatch = worst;
        info->hhl_seconds = hhl_s;
    }
    return st;
}
