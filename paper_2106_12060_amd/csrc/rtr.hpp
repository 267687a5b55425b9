// Launch interface of the trust-region solver's small kernels.
#pragma once
#include "common.hpp"

namespace srp {

constexpr int kRtrK = 16;        // largest k of the trust-region solver
constexpr int kRtrMaxDots = 6;   // inner products per launch

struct RtrLinSide {
  double* out = nullptr;
  const double* A = nullptr;
  double a = 0.0;
  const double* C = nullptr;
  double c = 0.0;
  const double* K = nullptr;   // k x k, null = identity
  int d = 0;
  int lda = 0, ldc = 0;        // row strides of A and C (0 = k)
};
struct RtrLinArgs {
  RtrLinSide side[2];
  int k = 0;
};
int rtr_lin(const RtrLinArgs& a, int nb, hipStream_t st);

struct RtrDotArgs {
  const double* X[kRtrMaxDots][2] = {};
  const double* Y[kRtrMaxDots][2] = {};
  int d[2] = {0, 0};
  int nb = 1, k = 0, np = 0;
  double* out = nullptr;   // device, np values
};
int rtr_dots(const RtrDotArgs& a, hipStream_t st);

struct RtrSylvArgs {
  const double* Q[2] = {};
  const double* lam[2] = {};
  const double* C[2] = {};
  double* S[2] = {};
  int k = 0;
};
int rtr_sylv(const RtrSylvArgs& a, int nb, hipStream_t st);

struct RtrTrialArgs {
  const double* E[2] = {};   // (B_b Z_b)^T (Z_b / 2 + eta_b): E + E^T = Z^T B Z + Z^T B eta + eta^T B Z
  const double* F[2] = {};   // eta_b^T B_b eta_b
  const double* X0[4] = {};     // the four parts of (Z_0 + eta_0)^T K (Z_1 + eta_1)
  const double* mu = nullptr;
  double cost_scale = 1.0;
  double* Lit[2] = {};
  double* out = nullptr;     // f+, breakdown flag
  int nb = 1, k = 0;
};
int rtr_trial(const RtrTrialArgs& a, hipStream_t st);

}  // namespace srp
