// Host-side launchers of the gfx950 kernels (defined in fft.hip, gemm.hip, cg.hip).
#pragma once
#include "basis.hpp"
#include "common.hpp"

namespace stern {

// Geometry of the pruned 3-D FFT of one system.
// Sphere coefficients are stored per vector in "column order": the plane waves
// grouped by x-pencil column (n_y, n_z), n_x ascending inside a column, padded
// to npw_pad. Pencil data after the x pass is [vec][ix][ncol_pad].
struct FftGeom {
  int N;
  int npw;
  int npw_pad;
  int ncol;
  int ncol_pad;
  int nza;                  // number of active n_z lines of the yz plane
  const int* col_start;     // [ncol_pad] first sphere index of the column
  const int* col_len;       // [ncol_pad] number of n_x values (0 for padding)
  const int* col_xmin;      // [ncol_pad] smallest n_x of the column
  const int* col_pos;       // [ncol] iy * N + iz of the column in a yz plane
  const int* zl;            // [nza] iz of the active lines
  const int* ycol;          // [N][nza] pencil column of (iy, zl[f]), -1 outside the sphere's disk
  int zact_lo, zact_hi;     // active lines are iz <= zact_lo or iz >= zact_hi
  int n_cu;                 // compute units of the device (persistent launches)
  const double* g2h;        // [npw_pad] |G|^2 / 2 in column order (0 for padding)
  const Z64* tw64;          // [N] exp(-2 pi i m / N)
  const Z32* tw32;
  // device count of the live vectors, or null: a launch sized for nvec vectors then covers only
  // the first *live of them (the active list shrinks on the device between host polls)
  const int* live = nullptr;
};

// columns per workgroup in the x-pencil passes: 32 FP32 or 16 FP64 columns, about the same
// bytes per workgroup; the basis pads the column count to kColPad (basis.hpp), a multiple of both
template <class T>
constexpr int col_block() {
  return sizeof(T) == 4 ? 32 : 16;
}
static_assert(kColPad % 32 == 0 && kColPad % 16 == 0, "column padding must hold whole column blocks");

bool fft_size_supported(int N);
size_t plane_lds_bytes(int N, int elem_bytes);
// LDS of the FP64 RHS / psi_v(r) / dn plane kernels (full plane, or the compact layout when that does not fit)
size_t plane_fp64_lds(int N, int nza);

// x pass, inverse: sphere coefficients of vectors vidx[b] (b < nvec) -> pencils.
template <class T>
void launch_xinv(const FftGeom& g, const Z<T>* sph, const int* vidx, int nvec, Z<T>* pen, hipStream_t st);
// x pass, forward + output mode:
//   mode 0: out = pencil transform
//   mode 1: out = pencil transform + (|G|^2/2 - eps[vec]) * pin        (H apply without KB)
//   mode 2: out = scale * pencil transform
template <class T>
void launch_xfwd(const FftGeom& g, const Z<T>* pen, const int* vidx, int nvec, Z<T>* out, int mode,
                 const Z<T>* pin, const double* eps, double scale, hipStream_t st);
// yz planes of the H apply: inverse, multiply by v_r (pre-scaled by 1/N^3), forward; in place.
template <class T>
void launch_plane_vloc(const FftGeom& g, Z<T>* pen, const int* vidx, int nvec, const T* v_r, hipStream_t st);
// same operation, compact-LDS wave-local kernel; vt = V_loc as [x][z][y]
template <class T>
void launch_plane_hw(const FftGeom& g, Z<T>* pen, const int* vidx, int nvec, const T* vt, bool prefetch,
                     hipStream_t st);
size_t plane_hw_lds(int N, int nza, bool fp64);  // its LDS bytes per workgroup
// yz planes of the right-hand sides of a batch of bands [v0, v0 + nb) x fields [i0, i0 + npert), solve
// s = (i - i0) nb + (v - v0) (band[s], pert[s] give the same): pencils[s] = forward planes of
// psi_r[v] * dv[i].
void launch_plane_rhs(const FftGeom& g, const Z64* psi_r, const double* dv, int v0, int nb, int i0, int npert,
                      const int* band, const int* pert, Z64* pen, hipStream_t st);
// yz planes, inverse to a full real-space grid: out[vec] = [N][N][N] complex.
void launch_plane_full_inv(const FftGeom& g, const Z64* pen, int nvec, Z64* out, hipStream_t st);
// dn[pert_out[p]] = scale * Re sum_{b < nb} conj(psi_r[band0 + b]) * x_r[p * nb + b], from pencils.
void launch_plane_dn(const FftGeom& g, const Z64* pen, const Z64* psi_r, int band0, int nb, int npert,
                     const int* pert_out, double scale, double* dn, hipStream_t st);

// C[n][m] = sum_k conj(A[m][k]) X[xidx[n]][k]; partial sums per K split.
// A: [M_pad][K] (M_pad multiple of 64), X rows of length ldx, K multiple of 8.
void launch_zgemm_reduce(const Z64* A, int M_pad, const Z64* X, int ldx, const int* xidx, int ncols, int K,
                         Z64* cpart, int nsplit, hipStream_t st);
// C[n][m] = scale * sum_s cpart[s][n][m]
void launch_sum_parts(const Z64* cpart, int nsplit, int ncols, int M_pad, double scale, Z64* C, hipStream_t st);
// Y[yidx[n]][k] += sum_m A[m][k] C[n][m], k < K (multiple of 64).
void launch_zgemm_expand(const Z64* A, int M_pad, const Z64* C, Z64* Y, int ldy, const int* yidx, int ncols, int K,
                         hipStream_t st);
// split-K factor for a reduce of ncols columns aiming at `target` workgroups (<= 0: default)
int choose_nsplit(int M_pad, int ncols, int K, int target);

// ---- CG vector kernels; one workgroup per solve s = act[b] ----
struct CgState {
  Z64 *x, *r, *p, *q, *z, *b;  // [nbatch][npw_pad]
  double *bb, *rz, *rr;        // [nbatch]
  int* flag;                   // 0 active, 1 recurrence-converged, 2 done (true residual accepted)
  int* iters;
  double* tres;                // true relative residual
  const double* eps;           // [nbatch] eps of the band of each solve
  const double* invT;          // [nbatch] 1 / T_v of the band of each solve
  const double* g2h;           // [npw_pad]
  const float* kprec;          // [nbatch][npw_pad] learned diagonal preconditioner, or null for Teter
  int npw_pad;
};
void launch_cg_init(const CgState& s, const int* act, int n, bool keep, hipStream_t st);
// r = b - A x + i u x for a guess x (A x in q, or q32 when not null); rejects guesses with ||r|| >= ||b||;
// with tol2 >= 0, marks a guess with ||r||^2 <= tol2 ||b||^2 converged (flag 2)
void launch_guess_resid(const CgState& s, const int* act, int n, const Z32* q32, int* rejected, hipStream_t st,
                        double u = 0.0, double tol2 = -1.0);
void launch_to32(const Z64* x, Z32* y, size_t n, hipStream_t st);
void launch_cg_init2(const CgState& s, const int* act, int n, hipStream_t st);
void launch_cg_alpha(const CgState& s, const int* act, int n, double tol2, hipStream_t st);
void launch_cg_beta(const CgState& s, const int* act, int n, hipStream_t st);
void launch_copy_rows(const Z64* src, Z64* dst, int ld, const int* act, int n, hipStream_t st);
void launch_true_resid(const CgState& s, const int* act, int n, double tol, hipStream_t st);
void launch_cg_restart(const CgState& s, const int* act, int n, hipStream_t st);
// Conjugate orthogonal CG for (P_c (H - eps) P_c - i u) x = b (response at imaginary frequency):
// negk [npw_pad] the index of -G of each coefficient; rzi [nbatch] the imaginary parts of the
// per-solve (r, z)_J (real parts in CgState::rz). start: p = z, rho = (r, z)_J for the solves with
// flag `from` (0 or 3), flag -> 0. alpha: q = P_c (H - eps) P_c p given. true: z = P_c x and
// q = P_c (H - eps) P_c x given, flag 1 -> 2 (accepted) or 3 (restart from the true residual).
void launch_cocg_start(const CgState& s, const int* negk, double* rzi, const int* act, int n, int from,
                       hipStream_t st);
void launch_cocg_alpha(const CgState& s, const int* negk, const double* rzi, double u, const int* act, int n,
                       double tol2, hipStream_t st);
void launch_cocg_beta(const CgState& s, const int* negk, double* rzi, const int* act, int n, hipStream_t st);
void launch_cocg_true(const CgState& s, double u, const int* act, int n, double tol, hipStream_t st);
// permutations between canonical and column order: out[v][perm[k]] = in[v][k] (scatter) or gather
void launch_permute(const Z64* in, int ld_in, Z64* out, int ld_out, const int* perm, int npw, int nvec, bool scatter,
                    hipStream_t st);
void launch_fill_zero(Z64* p, size_t n, hipStream_t st);
void launch_set_flag(int* flag, const int* list, int n, int value, hipStream_t st);
void launch_ri_to_complex(const double* in, Z64* out, size_t n, hipStream_t st);
// out = in + 0 i; out = scale Re(in) (grid fields of the PDEP potentials)
void launch_real_to_z(const double* in, Z64* out, size_t n, hipStream_t st);
void launch_z_real(const Z64* in, double scale, double* out, size_t n, hipStream_t st);
// whether the full-plane FP64 forward transform of an N^3 grid fits in `lds` bytes of LDS
bool plane_full_fwd_fits(int N, size_t lds);

// ---- learned initial guess (coarse-grid 3-D conv net, learn.hip) ----
constexpr int kNetChannels = 16;
constexpr int kNetInputs = 5;  // live input channels: Re, Im psi_v; Re, Im b / |b|; eps_v
constexpr int kNetLayers = 3;
constexpr int kNetLayerParams = kNetChannels * 27 * kNetChannels + kNetChannels;  // weights + bias
int net_ldp(int Nc);  // per-solve point stride of the activations (multiple of 16)
// preconditioner head: knots of the scale on u = log2(|G|^2 / 2T_v), features, parameters
constexpr int kPrecKnots = 8;
constexpr double kPrecU0 = -6.0;
constexpr double kPrecDu = 2.0;
constexpr int kPrecIn = kNetChannels + 2;
constexpr int kPrecParams = kPrecKnots * kPrecIn + kPrecKnots;
void launch_pool(const __bf16* act, const double* eps, const double* invT, float* f, int Nc, int nsolve,
                 hipStream_t st);
void launch_prec_coef(const float* head, const float* f, float* coef, int n, hipStream_t st);
void launch_prec_build(const float* coef, const float* f, const double* g2h, float* K, int npw_pad, int n,
                       hipStream_t st);
void launch_prec_apply(const float* K, const Z64* R0, const int* idx, Z64* out, int npw_pad, int n, hipStream_t st);
void launch_prec_grad(const Z64* P, const Z64* R0, const Z64* E0, const int* idx, const float* coef, const float* f,
                      const double* g2h, int npw, int npw_pad, float* gc, float* loss, int n, hipStream_t st);
void launch_head_grad(const float* gc, const float* f, int n, float* grad, hipStream_t st);
void launch_gather_rows(Z64* dst, const Z64* src, const int* rows, int ld, int n, bool sub, hipStream_t st);
void launch_gather_f32(float* dst, const float* src, const int* rows, int ld, int n, hipStream_t st);
void launch_conv3(const __bf16* in, const __bf16* W, const float* bias, void* out, int Nc, int nsolve, int act,
                  bool out_f32, hipStream_t st);
// weight and bias gradients of a layer into grad (kNetLayerParams floats); part holds
// conv3_wgrad_parts(Nc) x kNetLayerParams floats of per-tile partials
int conv3_wgrad_parts(int Nc);
void launch_conv3_wgrad(const __bf16* in, const float* gout, float* part, float* grad, int Nc, int nsolve,
                        hipStream_t st);
void launch_relu_bwd(float* g, const __bf16* act, size_t n, hipStream_t st);
void launch_f32_to_bf16(const float* a, __bf16* b, size_t n, hipStream_t st);
void launch_flip_weights(const float* W, __bf16* Wt, hipStream_t st);
void launch_loss(const float* out, const float* tgt, float* gout, float* loss, int Nc, int nsolve, hipStream_t st);
void launch_adam(float* w, float* m, float* v, const float* g, int n, float lr, int step, float scale,
                 hipStream_t st);
void launch_pack_input(const Z64* psi_c, const Z64* b_c, const int* band, const double* eps, const double* bnorm2,
                       __bf16* out, int Nc, int nsolve, hipStream_t st);
void launch_pack_band(const Z64* psi_c, const double* eps, __bf16* out, int Nc, int nband, hipStream_t st);
void launch_pack_target(const Z64* x_c, const double* bnorm2, float* tgt, int Nc, int nsolve, hipStream_t st);
void launch_unpack_output(const float* out, const double* bnorm2, Z64* x_c, int Nc, int nsolve, hipStream_t st);
// yz planes, forward: full complex planes in[vec][ix][iy][iz] -> pencils (for the coarse grid)
void launch_plane_full_fwd(const FftGeom& g, const Z64* in, int nvec, Z64* pen, hipStream_t st);

// ---- mixed precision (FP32 vectors, BF16 MFMA GEMMs, FP64 scalars) ----
struct Cg32State {
  Z32 *d, *r, *p, *q, *z;      // [nbatch][npw_pad]
  double *rz, *rr0, *beta;     // [nbatch]; beta = (r, z) new / old, set with rz by the alpha step
  int* flag;                   // inner: 0 active, 1 reached the inner tolerance, 2 nothing to do
  int* iters;
  const double* invT;
  const double* g2h;
  const float* kprec;  // as in CgState
  int npw_pad;
};
void launch_cg32_init(const Cg32State& s, const Z64* r64, const int* act, int n, hipStream_t st);
void launch_cg32_init2(const Cg32State& s, const int* act, int n, hipStream_t st);
void launch_cg32_alpha(const Cg32State& s, const int* act, int n, double tol2, hipStream_t st,
                       const int* live = nullptr);
// in-place stable compaction of the active list: rows s = list[i], i < *count, with flag[s] == 0 keep
// their order at the front and *count becomes their number (one workgroup)
void launch_compact(int* list, int* count, const int* flag, hipStream_t st);
void launch_cg32_beta(const Cg32State& s, const int* act, int n, hipStream_t st, const int* live = nullptr);
void launch_set_int(int* p, int v, hipStream_t st);  // *p = v (device), as a kernel
void launch_add_d(Z64* x, const Z32* d, int ld, const int* act, int n, hipStream_t st);
void launch_outer_resid(const CgState& s, const int* act, int n, double tol, hipStream_t st);
void launch_row_norm2(const Z64* y, int ld, int n, double* out, hipStream_t st);
void launch_outer_init(const CgState& s, const int* act, int n, double cut, hipStream_t st);
void launch_fill_zero32(Z32* p, size_t n, hipStream_t st);

int choose_nsplit_bf16(int M_pad, int ncols, int K, int target);
// hi/lo BF16 split of complex rows A [M][K] into [M][2K] and transposed [K][2M] layouts
void launch_split_bf16(const Z64* A, int M, int K, __bf16* hi, __bf16* lo, __bf16* thi, __bf16* tlo, hipStream_t st);
// the same into rows [row0, row0 + M) of a split matrix of Mt rows (row layout skipped when hi is null)
void launch_split_bf16_rows(const Z64* A, int M, int K, int row0, int Mt, __bf16* hi, __bf16* lo, __bf16* thi,
                            __bf16* tlo, hipStream_t st);
// coefficients of the projected (H - eps) p over the stacked rows [P_c KB (Ma); Psi (Mb)]:
// rows a: D <beta_a|p>; rows Ma + b: -<psi_b|q_loc>, q_loc the local part of (H - eps) p
void launch_sum_proj32(const Z32* cp_a, int ns_a, const Z32* cp_b, int ns_b, int ncols, int Ma, int Mb, float D,
                       __bf16* Cs, hipStream_t st, const int* live = nullptr);
// C[n][m] partial = sum_k conj(A[m][k]) X[xidx[n]][k] (BF16 split operands, FP32 accumulation)
// live (optional, device): only the first *live of the ncols columns are computed (ncols still
// sets the grid and the strides of the partials and of C)
void launch_reduce_bf16(const __bf16* Ahi, const __bf16* Alo, int M_pad, const Z32* X, int ldx, const int* xidx,
                        int ncols, int K, Z32* cpart, int nsplit, hipStream_t st, const int* live = nullptr);
void launch_sum_parts32(const Z32* cpart, int nsplit, int ncols, int M_pad, float scale, __bf16* Cs,
                        hipStream_t st, const int* live = nullptr);
// Y[yidx[n]][k] += sum_m A[m][k] C[n][m] from the transposed split copy of A (blocked
// layout, as k_split_rows writes it) and C as launch_sum_parts32 / launch_sum_proj32 write it;
// variant 0: 256 x 128 tiles of 8 waves, 1: 128 x 128 tiles of 16 waves, 2: 128 x 128 tiles of 8 waves.
// With P: Y is not written, P[s] = (Y[s] + A C) + beta[s] P[s] for s = yidx[n] instead.
void launch_expand_bf16(const __bf16* ATh, const __bf16* ATl, int M_pad, const __bf16* Cs, Z32* Y, int ldy,
                        const int* yidx, int ncols, int K, int variant, hipStream_t st, Z32* P = nullptr,
                        const double* beta = nullptr, const int* live = nullptr);

// ---- TDDFT Liouville apply and its block solve (tddft.hip, cg.hip) ----
// rho[e] = scale sum_v conj(psi_r[v]) a_r[e nb + v] on full N^3 grids (n3 points each)
void launch_band_density(const Z64* psi_r, const Z64* a_r, int n_exc, int nb, size_t n3, double scale, Z64* rho,
                         hipStream_t st);
// c[n][k] *= fac / g2h[k] for nvec rows of K coefficients, zero where g2h = 0
void launch_coulomb(Z64* c, const double* g2h, int K, int nvec, double fac, hipStream_t st);
// out[e nb + v] = v_r[e] psi_r[v] - alpha acc[e nb + v] (acc may be null) on full grids (n_exc nb <= 65535 rows)
void launch_grid_mul(const Z64* v_r, const Z64* psi_r, int n_exc, int nb, size_t n3, const Z64* acc, double alpha,
                     Z64* out, hipStream_t st);
// out[w] = scale conj(psi_r[w]) psi_r[v] for w < nb
void launch_pair_density(const Z64* psi_r, int v, int nb, size_t n3, double scale, Z64* out, hipStream_t st);
// proj[r][a] = N^-3 sum_j w[a][j] rho[r][j] for n real potentials w and nrows complex grids rho
void launch_scr_proj(const Z64* rho, const double* w, int n, int nrows, size_t n3, Z64* proj, hipStream_t st);
// tau[r] += sum_a w[a] c[a] proj[r][a]
void launch_scr_add(Z64* tau, const double* w, const Z64* proj, const double* c, int n, int nrows, size_t n3,
                    hipStream_t st);
// acc[e nb + v] = sum_{w < nb} tau[w] a_r[e nb + w] for e < n_exc
void launch_exch_acc(const Z64* tau, const Z64* a_r, int n_exc, int nb, int v, size_t n3, Z64* acc, hipStream_t st);
void launch_add(Z64* y, const Z64* x, size_t n, hipStream_t st);
// per-row conj(a) . b; y[row] += c[row / nb] x[row]; p[row] = z[row] + c[row / nb] p[row];
// z = Teter K_v r with T_v of band row mod nb
void launch_row_dot(const Z64* a, const Z64* b, int ld, int nrows, Z64* out, hipStream_t st);
void launch_blk_axpy(Z64* y, const Z64* x, const Z64* c, int nb, int ld, int nrows, hipStream_t st);
void launch_blk_xpby(Z64* p, const Z64* z, const Z64* c, int nb, int ld, int nrows, hipStream_t st);
void launch_teter_rows(const Z64* r, Z64* z, const double* g2h, const double* invT, int nb, int ld, int nrows,
                       hipStream_t st);
void launch_blk_scale(Z64* y, const Z64* c, int nb, int ld, int nrows, hipStream_t st);  // y[row] *= c[row / nb]

}  // namespace stern
