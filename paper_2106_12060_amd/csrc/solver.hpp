// Device-side state of one Riemannian CG solve and the step kernels that
// advance it.  See solver_kernels.hip for the mathematics.
#pragma once
#include "common.hpp"

namespace srp {

constexpr int KMAX = 32;       // largest k the step kernels support
constexpr int KK_STRIDE = KMAX * KMAX;

// k x k matrices kept per side in SolverState::kk, each KMAX*KMAX doubles.
enum KKSlot { KK_LINVT = 0, KK_S = 1, KK_PHI = 2, KK_ROT = 3, KK_EIG = 4, KK_NSLOTS = 5 };

struct SolverCtrl {
  double t;        // accepted step along the retraction curve
  double t_guess;  // centre of the next line search
  double f;        // cost at the current iterate
  double gg;       // <grad, grad>_M at the current iterate
  double gg_old;
  double df0;      // <grad, xi>_M for the current direction
  double beta;
  double tol;
  int done;        // 1: stop (converged, failed or out of iterations)
  int status;      // SRP_OK / SRP_ENOCONV / SRP_ENOTSPD
  int iter;
  int max_iter;
  int restart;     // next direction is -grad
  int ls_fail;     // consecutive line-search failures
  int fixed_step;  // 1: take t = 1 without a line search (the qf start)
  int eig_ok;      // KK_EIG holds the eigenvectors of the previous P
};

// One block of the (product) manifold: St_B(k, d) with B = A^T A + lam I.
struct SideView {
  int d;
  double lam;
  double* U;      // d x k iterate
  double* Ks;     // A^T A U
  double* Kc;     // cost products: CCA A^T A_other U_other; FDA S_B U
  double* xi;     // d x k search direction
  double* gold;   // d x k previous Riemannian gradient
  const double* J;  // pass output d x jld (Js at column js_off, Jc at jc_off)
  int jld, js_off, jc_off;
  const double* Jc_sep;  // FDA: S_B xi, d x k (then J's jc block is unused)
  double* Z;      // d x 2k: [E | B U]
  double* Wz;     // d x 2k: M^-1 Z
};

struct ProbView {
  int nb;         // 1 (FDA) or 2 (CCA)
  int k;
  int lda_cost;   // 1: cost -1/2 tr(W^T S_B W N); 0: CCA cross cost
  SideView s[2];
  const double* mu;   // device, k weights
  SolverCtrl* ctrl;
  double* kk;         // [2][KK_NSLOTS][KMAX*KMAX]
  double* part;       // partial k x k products
  int part_slices;    // row-slice workgroups per side used for partials
  double eig_tol2;    // Jacobi stop of the direction step: off^2 <= eig_tol2 diag^2
};

// k-wide inner products over row slices:
// out[y][z][a*k+i][b*k+j] = sum over rows r of slice z of L_a[r][i] R_b[r][j]
// for side y.
struct PartialSide {
  int d, nl, nr;
  const double* lp[4]; int lld[4];
  const double* rp[6]; int rld[6];
};
struct PartialArgs {
  int k, slices, nb;
  PartialSide side[2];
  double* out;            // [side][slices][nl*k][nr*k]
  int64_t side_stride;
  const SolverCtrl* ctrl;
};
// The partial products of a step for view p: kind 0 the line search's, 1
// the direction's, 2 the finish's.
void fill_partial_args(const ProbView& p, int kind, PartialArgs* a);

// Grouped launches (the serving engine's ticks): one launch runs a step for
// up to kGroupMax solves, each read from a device array of ProbView (or
// PartialArgs) at index idx[z]; aux carries a per-solve launch parameter.
constexpr int kGroupMax = 16;
struct GroupSel {
  int n;
  int idx[kGroupMax];
  int aux[kGroupMax];
};
int launch_partials_g(const PartialArgs* ga, const GroupSel& sel, int max_slices, int64_t max_nlnr,
                      hipStream_t st);
int ctrl_ls_shape(int k, int nb, size_t* lds);   // returns the trial count (< 1: k too large)
size_t ctrl_dir_lds(int k, int nb);
int launch_ctrl_ls_g(const ProbView* v, const GroupSel& sel, size_t lds, int kc, hipStream_t st);
int launch_update_g(const ProbView* v, const GroupSel& sel, int refresh, int dmax, int kc, hipStream_t st);
int launch_ctrl_dir_g(const ProbView* v, const GroupSel& sel, size_t lds, int kc, hipStream_t st);
int launch_combine_g(const ProbView* v, const GroupSel& sel, int64_t max_dk, int kc, hipStream_t st);

// Launchers (solver_kernels.hip).
int launch_ls_partials(const ProbView& p, hipStream_t st);
int launch_ctrl_ls(const ProbView& p, hipStream_t st);
int launch_update(const ProbView& p, int refresh, hipStream_t st);
int launch_dir_partials(const ProbView& p, hipStream_t st);
int launch_ctrl_dir(const ProbView& p, hipStream_t st);
int launch_combine(const ProbView& p, hipStream_t st);
int launch_final_partials(const ProbView& p, hipStream_t st);
int launch_ctrl_final(const ProbView& p, double* sigma_out, hipStream_t st);
int launch_apply_rot(const ProbView& p, hipStream_t st);
int launch_sign_fix(const ProbView& p, hipStream_t st);
int launch_gauss_fill(double* p, int64_t count, uint64_t seed, hipStream_t st);
int launch_ctrl_init(SolverCtrl* c, double tol, int max_iter, hipStream_t st);
int launch_set_fixed_step(SolverCtrl* c, int on, hipStream_t st);
size_t partial_bytes(int k, int dmax);
// Exact sketched solves (warm start): Cholesky-QR factor B = L^-T of a
// q x q block Gram (q <= 64; *flag = 1 on breakdown), written with leading
// dimension cholqr_block(q) (16, 32 or 64; B must hold its square), and the
// Rayleigh-Ritz eigenvectors of a symmetric q x q block (top k, descending).
int cholqr_block(int q);
int launch_cholqr_factor(const double* G, int q, double* B, int* flag, hipStream_t st);
int launch_rr_eig(const double* G, int q, int k, double* Q, double* ev, hipStream_t st);
int partial_slices(int dmax);

}  // namespace srp
