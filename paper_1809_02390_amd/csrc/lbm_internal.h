// Internal declarations shared by the host map and the HIP translation unit.
#pragma once

#include <cstddef>

#include "lbm.h"

namespace lbm {

double critical_temperature(double a, double b, double r_gas);
int maxwell(double tr, double a, double b, double r_gas, double* rho_g, double* rho_l, double* p0);
int interface_constants(double tr, double a, double b, double r_gas, double* c_sigma, double* c_w);
int sigma_paper(double width, double tr, double a, double b, double r_gas, double* sigma);
int validate(const lbm_params* p, char* msg, size_t len);
int derive(const lbm_params* p, lbm_derived* out, char* msg, size_t len);
int param_jacobian(const lbm_params* p, double* jac, char* msg, size_t len);

}  // namespace lbm
