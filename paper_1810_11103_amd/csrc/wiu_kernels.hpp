// Kernel launch interface of libwenoiu (internal to the library).
#pragma once

#include "wiu_device.hpp"

namespace wiu {

// Arguments of one direction sweep (see sweep_kernel).
struct SweepArgs {
  Dims d;
  const double* U;                      // state the fluxes are built from
  const double* M;                      // metrics (with tag)
  const unsigned long long* lam_xi;     // raw line maxima (bit patterns)
  const unsigned long long* lam_eta;
  double gamma, alpha, eps;
  int ppm;
  int mode;                             // 0 write R^xi, 1 dU/dt, 2 RK stage
  double* Rxi;                          // R^xi (written in mode 0, read otherwise)
  double* out;                          // dU/dt or the new RK stage state
  const double* U0;                     // RK base state U^n
  const double* dt;                     // device scalar time step
  double ca, cb;                        // out = ca U0 + cb (U + dt L)
  int* status;
};

hipError_t launch_sweep(int scheme, int dir, const SweepArgs& a, hipStream_t st);
hipError_t launch_wave_max(const Dims& d, const double* U, const double* M, double gam, unsigned long long* lx,
                           unsigned long long* le, unsigned long long* cfl, int* status, hipStream_t st);
hipError_t launch_metrics(const Dims& d, int scheme, const double* x, const double* y, double* M, double* T,
                          int* status, hipStream_t st);
hipError_t launch_cfl_dt(const unsigned long long* cfl_max, double cfl, double* dt, hipStream_t st);
hipError_t launch_lambda_out(const Dims& d, double alpha, const unsigned long long* lx, const unsigned long long* le,
                             double* ox, double* oe, hipStream_t st);
hipError_t launch_set_tag(const Dims& d, int scheme, double* M, hipStream_t st);
hipError_t launch_zero_header(int* p, int n, hipStream_t st);

}  // namespace wiu
