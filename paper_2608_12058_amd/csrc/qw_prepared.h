// Action calls on energy tables that are already on the device, for
// integrators that apply many exponentials exp(-i t (alpha H_P + beta sum_j X_j))
// with the same couplings (defined in qw_action.hip).
#pragma once

#include "qw_device.h"
#include "qwexp.h"

namespace qw {

// Device tables of one (h, J) set and, for an action call, the factor alpha by
// which the energies are scaled.
struct Prepared {
    EnergyTables T;
    double escale;
};

// Uploads (h, J) into the workspace (qw_workspace_bytes layout), builds the
// pair table and returns min / max of E over all 2^n states (one read-back).
template <typename R>
qw_status prepare_energy(int n, const double *h, const double *J, void *workspace, size_t ws_bytes, void *stream,
                         EnergyTables *T, double *emin, double *emax);

// psi_out = exp(-i t (alpha H_P + beta sum_j X_j)) psi_in with the prepared
// tables; the shift and bound follow from alpha, [emin, emax] and beta without
// a read-back, and the norm monitor stays off.
template <typename R>
qw_status scaled_action(int n, const double *h, const double *J, const EnergyTables &T, double alpha, double emin,
                        double emax, double beta, double t, const void *psi_in, void *psi_out, double tol,
                        void *workspace, size_t ws_bytes, void *stream, qw_info *info);

}  // namespace qw
