// qrfs_plan.cpp -- host-side choice of the Cartesian sampling
// hyper-parameters (Sec. 4.3): pitch df = 0.25 / L0 by default, and N from
// the saturation of the radial integral of the filtered PSD.
#include <cmath>

#include "qrfs.h"
#include "qrfs_internal.hpp"

namespace qrfs {
qrfs_status api_fail(qrfs_status s, const char* fmt, ...);
qrfs_status api_ok();
}  // namespace qrfs

namespace {

// f W(f) F(f)^2 (von Karman), F the signed filter of Eq. 7
double radial(double c, double r0, double L0, const qrfs_aperture* ap, double f) {
    if (f <= 0.0) return 0.0;
    const double w = c * std::pow(r0, -5.0 / 3.0) * std::pow(f * f + 1.0 / (L0 * L0), -11.0 / 6.0);
    double F = 1.0;
    if (ap) {
        const double pi = 3.141592653589793;
        double num = ap->D * std::cyl_bessel_j(1.0, pi * ap->D * f);
        if (ap->d > 0.0) num -= ap->d * std::cyl_bessel_j(1.0, pi * ap->d * f);
        F = 2.0 * num / (pi * (ap->D * ap->D - ap->d * ap->d) * f);
    }
    return f * w * F * F;
}

// 5-point Gauss-Legendre rule on [a, b]
double gauss5(double c, double r0, double L0, const qrfs_aperture* ap, double a, double b) {
    static const double x[5] = {-0.9061798459386640, -0.5384693101056831, 0.0,
                                0.5384693101056831, 0.9061798459386640};
    static const double w[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                                0.4786286704993665, 0.2369268850561891};
    const double m = 0.5 * (a + b), h = 0.5 * (b - a);
    double s = 0.0;
    for (int i = 0; i < 5; ++i) s += w[i] * radial(c, r0, L0, ap, m + h * x[i]);
    return s * h;
}

}  // namespace

extern "C" qrfs_status qrfs_choose_cartesian(const qrfs_psd* psd, const qrfs_aperture* ap,
                                             double df, double eps, int32_t* N, double* df_out,
                                             double* sigma2) {
    using qrfs::api_fail;
    if (!psd) return api_fail(QRFS_ERR_INVALID_ARG, "psd is NULL");
    if (!N || !df_out) return api_fail(QRFS_ERR_INVALID_ARG, "N and df_out are required");
    if (psd->model == QRFS_PSD_KOLMOGOROV)
        return api_fail(QRFS_ERR_UNSUPPORTED, "the radial integral of the Kolmogorov PSD diverges");
    if (psd->model != QRFS_PSD_VON_KARMAN)
        return api_fail(QRFS_ERR_INVALID_ARG, "unknown PSD model %d", psd->model);
    if (!(psd->r0 > 0.0) || !(psd->L0 > 0.0))
        return api_fail(QRFS_ERR_INVALID_ARG, "r0 and L0 must be > 0");
    if (!(eps > 0.0) || !(eps < 1.0)) return api_fail(QRFS_ERR_INVALID_ARG, "eps must be in (0, 1)");
    if (ap && (!(ap->D > 0.0) || !(ap->d >= 0.0) || !(ap->d < ap->D)))
        return api_fail(QRFS_ERR_INVALID_ARG, "aperture needs 0 <= d < D");
    if (!(df > 0.0)) df = 0.25 / psd->L0;
    if (!(psd->wavelength >= 0.0) || !std::isfinite(psd->wavelength))
        return api_fail(QRFS_ERR_INVALID_ARG, "wavelength must be >= 0");
    const double c = qrfs::psd_constant(psd->c, psd->wavelength);
    // far enough that the increments left out hold < 1e-6 of the variance
    const double x_max = ap ? 200.0 / ap->D : 2000.0 / psd->L0;
    const double steps = std::ceil(x_max / df);
    if (steps > 2147483647.0) return api_fail(QRFS_ERR_INVALID_ARG, "df too small");
    const int64_t n_max = (int64_t)steps;
    double total = 0.0;
    for (int64_t n = 1; n <= n_max; ++n)
        total += gauss5(c, psd->r0, psd->L0, ap, (double)(n - 1) * df, (double)n * df);
    int64_t nstar = 1;
    for (int64_t n = n_max; n >= 1; --n)
        if (gauss5(c, psd->r0, psd->L0, ap, (double)(n - 1) * df, (double)n * df) >= eps * total) {
            nstar = n;
            break;
        }
    if (nstar == n_max)
        return api_fail(QRFS_ERR_NOT_CONVERGED,
                        "increments still >= eps g(inf) at the integration limit %g (eps %g)",
                        x_max, eps);
    *N = (int32_t)(2 * nstar);
    *df_out = df;
    if (sigma2) *sigma2 = 2.0 * 3.141592653589793 * total;
    return qrfs::api_ok();
}
