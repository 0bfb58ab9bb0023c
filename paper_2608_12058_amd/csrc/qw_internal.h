// Internal declarations shared by the host and HIP translation units of libqwexp.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace qw {

// --- host coefficient setup (qw_coeffs.cpp) -------------------------------
int bessel_cutoff(double x);
int bessel_miller(double a, int mmax, double *J);
int cf_real(const double *c, int M, int m, double *p, double *lam_out);
// method 0 = Chebyshev, 1 = CF.  alpha gets alpha_0..alpha_K.
int coefficients(double a, double tol, int method, std::vector<double> &alpha, int *K_out, double *err_out);

// --- error reporting (qw_api.hip) -----------------------------------------
void set_error(const std::string &msg);

}  // namespace qw
