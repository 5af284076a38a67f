// Analytic Verlet-buffer estimate (Sec. 5 "Effective pair list buffering" and
// the appendix's upper bound on the energy drift from missed pairs).
//
// Over a list lifetime t a free particle of mass m is displaced by a Gaussian
// of variance kB T t^2 / m per dimension, so a pair's distance changes with
// sigma^2 = kB T t^2 (1/m_a + 1/m_b).  A pair starting beyond r_l = r_c + r_b
// and ending inside r_c is missed; expanding the potential (shifted to zero at
// r_c) to second order at r_c and taking r_0^2 ~ (r_l + sigma)^2 gives, per
// type-a particle and type-b neighbours of density rho_b,
//   dV = 4 pi (r_l+sigma)^2 rho_b { V'/2 [r_b sigma G(x) - (r_b^2+sigma^2) E(x)]
//                                 + V''/6 [sigma (r_b^2 + 2 sigma^2) G(x) - r_b (r_b^2 + 3 sigma^2) E(x)] },
// x = r_b/sigma, G the unit normal density, E(x) = erfc(x/sqrt 2)/2.  The
// factor 2 sigma^2 is what the underlying integral gives (the printed form
// has sigma^2).  Drift per particle = 1/2 sum_a N_a sum_b |dV_ab| / (N nstlist dt),
// displacement time t = (nstlist - 1) dt.
#include <cmath>

#include "internal.h"

namespace mxn {

namespace {

constexpr double kB = 0.0083144626;   // kJ mol^-1 K^-1

void derivs(const nb_buffer_query &q, int a, int b, double &v1, double &v2) {
    const double rc = q.rc, beta = q.beta;
    const double c6 = q.c6c12[2 * (a * q.ntypes + b)], c12 = q.c6c12[2 * (a * q.ntypes + b) + 1];
    v1 = -12.0 * c12 / std::pow(rc, 13) + 6.0 * c6 / std::pow(rc, 7);
    v2 = 156.0 * c12 / std::pow(rc, 14) - 42.0 * c6 / std::pow(rc, 8);
    const double qq = q.coulomb_f * q.charge[a] * q.charge[b];
    const double br = beta * rc;
    const double g = 2.0 * beta / std::sqrt(M_PI) * std::exp(-br * br);
    v1 += qq * (-std::erfc(br) / (rc * rc) - g / rc);
    v2 += qq * (2.0 * std::erfc(br) / (rc * rc * rc) + g * (2.0 / (rc * rc) + 2.0 * beta * beta));
}

}  // namespace

double analytic_drift(const nb_buffer_query &q, double rb) {
    const double t = (q.nstlist - 1) * q.dt;
    double total = 0.0, ntot = 0.0;
    for (int a = 0; a < q.ntypes; ++a) ntot += q.count[a];
    for (int a = 0; a < q.ntypes; ++a)
        for (int b = 0; b < q.ntypes; ++b) {
            const double sig = std::sqrt(kB * q.T * t * t * (1.0 / q.mass[a] + 1.0 / q.mass[b]));
            if (!(sig > 0.0)) continue;
            double v1, v2;
            derivs(q, a, b, v1, v2);
            const double x = rb / sig;
            const double G = std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI);
            const double E = 0.5 * std::erfc(x / std::sqrt(2.0));
            const double first = 0.5 * v1 * (rb * sig * G - (rb * rb + sig * sig) * E);
            const double second =
                v2 / 6.0 * (sig * (rb * rb + 2.0 * sig * sig) * G - rb * (rb * rb + 3.0 * sig * sig) * E);
            const double rl = q.rc + rb;
            const double dv = 4.0 * M_PI * (rl + sig) * (rl + sig) * (q.count[b] / q.volume) * (first + second);
            total += 0.5 * q.count[a] * std::fabs(dv);
        }
    return total / (ntot * q.nstlist * q.dt);
}

int analytic_buffer(const nb_buffer_query &q, double *rb_out, double *drift_out) {
    constexpr double kGrid = 0.0005, kMax = 2.0;
    for (int k = 0; k * kGrid <= kMax + 1e-12; ++k) {
        const double rb = k * kGrid;
        const double d = analytic_drift(q, rb);
        if (d <= q.target) {
            *rb_out = rb;
            if (drift_out) *drift_out = d;
            return NB_OK;
        }
    }
    return fail(NB_ERR_ARG, "nb_buffer_estimate: no buffer up to 2 nm meets the drift target");
}

int validate_query(const nb_buffer_query *q) {
    if (!q || !q->mass || !q->charge || !q->c6c12 || !q->count) return fail(NB_ERR_ARG, "nb_buffer_estimate: null");
    if (q->ntypes < 1 || q->nstlist < 1 || !(q->dt > 0) || !(q->T > 0) || !(q->volume > 0) || !(q->rc > 0) ||
        !(q->beta >= 0) || !(q->target > 0))
        return fail(NB_ERR_ARG, "nb_buffer_estimate: parameter out of range");
    for (int a = 0; a < q->ntypes; ++a)
        if (!(q->mass[a] > 0) || !(q->count[a] >= 0)) return fail(NB_ERR_ARG, "nb_buffer_estimate: bad mass/count");
    return NB_OK;
}

}  // namespace mxn
