// Lubricant model and Moes line-contact constants shared by the line-contact
// kernels (assembly, adjoint partial derivatives).
//
// Roelands pressure-viscosity law and Dowson-Higginson density (paper
// appendix, dimensionless with the Hertzian pressure p_h), Moes line-contact
// parameters alpha-bar = L sqrt(M / 2 pi), lambda-bar = 3 pi^2 / (8 M^2)
// (Sec. 3.3).
#pragma once
#include "common.h"

namespace pq {

namespace lub {
constexpr double ALPHA = 1.7e-8;  // pressure-viscosity coefficient [1/Pa]
constexpr double P0R = 1.98e8;    // Roelands reference pressure [Pa]
constexpr double ZR = 0.68;       // Roelands pressure-viscosity index
constexpr double RHO_A = 0.59e9;  // Dowson-Higginson constants [Pa]
constexpr double RHO_B = 1.34;
}  // namespace lub

struct LineConst {
    double lam, ph;  // lambda-bar and the Hertzian pressure p_h [Pa]
};

PQ_DEV LineConst line_const(double M, double L)
{
    LineConst c;
    const double abar = L * sqrt(M / (2.0 * M_PI));
    c.lam = 3.0 * M_PI * M_PI / (8.0 * M * M);
    c.ph = abar / lub::ALPHA;
    return c;
}

// Node quantities of the Reynolds operator at pressure P and film H:
// rho, eps = rho H^3 / (eta lam), rho*H and their derivatives with respect to
// the node pressure (at fixed H) and the node film.
struct NodeState {
    double rho, drho, eps, rH, eP, eH, drhoH;
};

PQ_DEV NodeState node_state(double Pm, double Hm, const LineConst& lc)
{
    using namespace lub;
    NodeState q;
    const double s = lc.ph / P0R;
    const double base = 1.0 + s * Pm;
    const double cc = ALPHA * P0R / ZR;
    const double lneta = cc * (-1.0 + pow(base, ZR));
    const double dlneta = cc * ZR * pow(base, ZR - 1.0) * s;
    const double den = RHO_A + lc.ph * Pm;
    q.rho = (RHO_A + RHO_B * lc.ph * Pm) / den;
    q.drho = (RHO_B * lc.ph * den - (RHO_A + RHO_B * lc.ph * Pm) * lc.ph) / (den * den);
    const double lam_eta = exp(lneta) * lc.lam;
    q.eps = q.rho * Hm * Hm * Hm / lam_eta;
    q.rH = q.rho * Hm;
    q.eP = q.drho * Hm * Hm * Hm / lam_eta - q.eps * dlneta;
    q.eH = 3.0 * q.rho * Hm * Hm / lam_eta;
    q.drhoH = q.drho * Hm;
    return q;
}

// van Leer limiter psi(d-, d+) = 2 d+ d- / (d+ + d-) where the slopes have the
// same sign, else 0; pa = d psi / d d+, pb = d psi / d d-.
PQ_DEV void van_leer(double dm, double dp, double& psi, double& pa, double& pb)
{
    if (dm * dp > 0.0) {
        const double den = dp + dm;
        psi = 2.0 * dp * dm / den;
        pa = 2.0 * dm * dm / (den * den);
        pb = 2.0 * dp * dp / (den * den);
    } else {
        psi = pa = pb = 0.0;
    }
}

// Limiter coefficients (pa, pb) used in the Newton matrix only (the residual
// always uses psi itself): mode 0 the exact derivatives of psi; mode 1 the
// ratio frozen at the current iterate, psi = phi(r) D- with r = D+/D- and
// phi(r) = 2r/(1+r) held fixed (eqs. 64-65 take r from the old film), so
// only D- moves: pa = 0, pb = phi; mode 2 the first-order upwind flux
// (pa = pb = 0).
PQ_DEV void limiter_jacobian(int mode, double dm, double dp, double& pa, double& pb)
{
    if (mode == 0) {
        double psi;
        van_leer(dm, dp, psi, pa, pb);
        return;
    }
    pa = 0.0;
    pb = (mode == 1 && dm * dp > 0.0) ? 2.0 * dp / (dm + dp) : 0.0;
}

// Convective slope psi of the face value (rho H)_{i+1/2} = (rho H)_i + psi/2
// and the coefficients (pa, pb) of the Newton matrix: conv 0 the van Leer
// slope with limiter_jacobian(limjac); conv 1 the kappa-scheme (Sec. 3.3,
// eqs. 56-59) psi = (1+kappa)/2 D+ + (1-kappa)/2 D-, linear, whose exact
// coefficients are used for limjac 0 and 1 (limjac 2: first-order flux).
PQ_DEV void convective_slope(int conv, double kappa, int limjac, double dm, double dp,
                             double& psi, double& pa, double& pb)
{
    if (conv == 1) {
        psi = 0.5 * (1.0 + kappa) * dp + 0.5 * (1.0 - kappa) * dm;
        pa = limjac == 2 ? 0.0 : 0.5 * (1.0 + kappa);
        pb = limjac == 2 ? 0.0 : 0.5 * (1.0 - kappa);
        return;
    }
    van_leer(dm, dp, psi, pa, pb);
    limiter_jacobian(limjac, dm, dp, pa, pb);
}

// Partials of the slope only (the Newton-matrix coefficients pa = d/dD+,
// pb = d/dD-): limiter_jacobian(limjac) for van Leer, the kappa-scheme's
// constants for conv 1 (zero with limjac 2, the first-order matrix).
PQ_DEV void slope_partials(int conv, double kappa, int limjac, double dm, double dp, double& pa,
                           double& pb)
{
    double psi;
    convective_slope(conv, kappa, limjac, dm, dp, psi, pa, pb);
}

}  // namespace pq
