// Host-only tables of the path propagation (no HIP types).
#pragma once

namespace quapi_host {
bool hermitian_ok(int M, const double* H);
void propagator(int M, const double* H, double dt, double* U);
int eta_columns(double ohmic_alpha, double ohmic_wc, int n_peaks, const double* peaks,
                double beta, double dt, int K, double* eta);
}  // namespace quapi_host
