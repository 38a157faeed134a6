/*
 * stern.h - C ABI of the MI355X (gfx950) Sternheimer chi0 library.
 *
 * The library evaluates the static density response dn = chi0 dV of a set of
 * occupied Kohn-Sham-like states without empty states, the route that
 * Sec. II.A of the WEST paper (arXiv 2607.14025) uses inside its PDEP
 * diagonalisation of chi0 (eq. pdep): for every occupied band v and field dV_i
 *
 *     P_c (H - eps_v) P_c x_{v,i} = -P_c dV_i psi_v,      P_c = 1 - sum_v |psi_v><psi_v|
 *     dn_i(r) = 4 Re sum_v conj(psi_v(r)) x_{v,i}(r)       (2 spin x 2 c.c.)
 *
 * solved by projected preconditioned CG (Teter-Payne-Allan diagonal) from zero.
 * The same solves serve the steps around it: the mixed-precision and learned
 * starts, the response at imaginary frequency and warm starts (stern_opts), the
 * PDEP Davidson on chi-bar0 (Sec. II.A, eq. pdep), and the TDDFT/BSE Liouville
 * superoperator of Sec. II.C.1 (eq. bse_tddft) with its Z-vector solves, its
 * Davidson for excitation energies and its Lanczos spectra.
 *
 * Model Hamiltonian (input stand-in for the ground-state code of the paper's
 * workflow, Sec. II): cubic cell of edge L (bohr), Gamma point, plane waves
 * G = 2 pi n / L with |G|^2 <= ecut_ry (bohr^-2);
 *   H = |G|^2/2 + V_loc + D sum_a |beta_a><beta_a|,
 *   V_loc(q) = A (2 pi s^2)^{3/2} / Omega exp(-s^2 |q|^2 / 2) sum_a exp(-i q.R_a),
 *   beta_a(G) = Omega^{-1/2} exp(-w^2 |G|^2 / 2) exp(-i G.R_a).
 *
 * Conventions shared by every entry point:
 *   - Coefficient order ("canonical order"): the plane waves sorted by |n|^2,
 *     then n_x, n_y, n_z ascending. stern_basis_info() returns the triples.
 *   - Complex arrays are interleaved (re, im) doubles.
 *   - Real-space arrays are [n][N][N][N] doubles indexed [ix][iy][iz] with iz
 *     fastest, at r = L (ix, iy, iz) / N; N is the FFT grid of the system.
 *   - psi(r) = Omega^{-1/2} sum_G c_G exp(i G.r); dn is in electrons / bohr^3.
 *   - Every call is synchronous with respect to the caller: when it returns,
 *     outputs are written (host) or the work is complete on the stream (device).
 *   - The caller owns every pointer it passes; the library copies what it keeps.
 *   - Errors: a negative return code; stern_last_error() gives the message of
 *     the last failing call on the calling thread. Nothing throws across the ABI.
 */
#ifndef STERN_H
#define STERN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define STERN_OK 0
#define STERN_WARN_NOT_CONVERGED 1   /* dn written; some solves missed tol (see stats) */
#define STERN_ERR_INVALID_ARG (-1)
#define STERN_ERR_STATE (-2)          /* e.g. apply before set_occupied */
#define STERN_ERR_OOM (-3)
#define STERN_ERR_HIP (-4)
#define STERN_ERR_UNSUPPORTED (-6)    /* e.g. FFT size not of the form 2^a 3^b <= 128 */

/* precision of the solver: plain FP64 PCG, or FP32 FFTs + split-BF16 MFMA
   GEMMs inside an FP64 defect-correction loop (FP64 scalars, FP64 true residual) */
#define STERN_FP64 0
#define STERN_MIXED 1

/* initial guess: zero, or the learned guess of a trained stern_model */
#define STERN_GUESS_ZERO 0
#define STERN_GUESS_LEARNED 1    /* learned x0 and learned diagonal preconditioner */
#define STERN_GUESS_LEARNED_K 2  /* learned diagonal preconditioner only, x0 = 0 */
/* warm start: every solve (v, i) starts from the solution of the same (v, i) kept by an earlier
   call with keep_solutions set (same n_pert and band range, and no set_occupied since; else
   STERN_ERR_STATE). The FP64 residual of the start decides: a start already within tol is a
   converged solve with no iteration, one with ||r|| >= ||b|| is replaced by zero. For sequences
   of related calls on the same fields: a frequency sweep of the response at i u, or a tighter
   tolerance after a loose one. FP64, mixed and imaginary-frequency solves. */
#define STERN_GUESS_PREVIOUS 3

/* where pointer arguments live */
#define STERN_MEM_HOST 0
#define STERN_MEM_DEVICE 1

typedef struct stern_system stern_system;

/* One cell. pos: [n_atoms][3] bohr, copied. fft_n = 0 selects the smallest
 * 2^a 3^b >= 2 (floor(2 sqrt(ecut) L / 2 pi) + 1) + 1, which holds the 4 ecut
 * sphere so that every grid product is exact in the basis. */
typedef struct {
  double L;
  double ecut_ry;
  int n_atoms;
  const double* pos;
  double vloc_amp;    /* A, Ha (e.g. -2) */
  double vloc_sigma;  /* s, bohr (e.g. 1) */
  double kb_D;        /* D, Ha (e.g. +1) */
  double kb_width;    /* w (e.g. 1) */
  int fft_n;
} stern_cell;

/* device: HIP ordinal; stream: hipStream_t to run on (NULL = default stream).
 * dev_alloc / dev_free (both or neither; NULL = hipMalloc / hipFree): the
 * caller's device allocator, e.g. a framework's caching allocator. The library
 * takes every device buffer of the system from dev_alloc(bytes, alloc_ctx),
 * which must return memory on `device` aligned to at least 256 bytes, or NULL
 * (the call then fails with STERN_ERR_OOM); it hands each one back with
 * dev_free(ptr, alloc_ctx) once the work that used it has completed (it
 * synchronises the device first), at the latest in stern_free. The callbacks
 * may run on any thread that calls into the library for this system,
 * including the worker threads of stern_apply_chi0_many. */
typedef struct {
  int device;
  void* stream;
  void* (*dev_alloc)(size_t bytes, void* ctx);
  void (*dev_free)(void* ptr, void* ctx);
  void* alloc_ctx;
} stern_runtime;

typedef struct {
  double tol;          /* relative FP64 true residual ||b - A x|| / ||b|| to accept */
  int max_iter;        /* CG iterations per solve (0 = 1000) */
  int precision;       /* STERN_FP64 or STERN_MIXED */
  int guess;           /* STERN_GUESS_ZERO, _LEARNED, _LEARNED_K (these two need model) or _PREVIOUS */
  int mem_kind;        /* STERN_MEM_HOST or STERN_MEM_DEVICE for dv_r / dn_r */
  int band_begin;      /* solve bands [band_begin, band_end); band_end <= 0 means n_occ.
                          P_c always uses every occupied band; dn is the partial sum. */
  int band_end;
  int max_batch;       /* solves held in flight at once (0 = choose from free memory) */
  int check_every;     /* iterations between convergence checks and active-set compaction
                          (0 = 1: every iteration; converged solves stop costing work at once) */
  /* optional per-solve outputs for a list of (band, perturbation) pairs:
     sample_pairs[2k] = v, sample_pairs[2k+1] = i; sample_x receives
     n_sample x n_pw complex solutions in canonical order (host memory). */
  int n_sample;
  const int* sample_pairs;
  double* sample_x;
  /* nonzero: time every kernel launch with HIP events on the library's stream
     and report per-class totals in stern_stats (adds one event pair per launch) */
  int profile;
  /* STERN_MIXED only: relative tolerance of each FP32/BF16 inner solve (0 = 1e-4)
     and the number of FP64 defect-correction steps before the solves still above
     tol fall back to FP64 PCG from zero (0 = 8) */
  double inner_tol;
  int max_outer;
  /* nonzero: capture one CG iteration (all its launches) into a hipGraph after
     every active-set compaction and replay it check_every times (ignored when
     profile != 0) */
  int use_graph;
  /* trained stern_model for STERN_GUESS_LEARNED / _LEARNED_K (not owned) */
  const struct stern_model* model;
  /* STERN_MIXED only: operator of the inner solve, one of STERN_INNER_* (0 = projected) */
  int inner_op;
  /* u >= 0: the response at imaginary frequency i u (Sec. II.A: the self-energy is evaluated at
     many frequencies, Lanczos chains and full frequency, which need chi0 beyond zero frequency).
     u > 0 solves (P_c (H - eps_v) P_c - i u) x = -P_c dV_i psi_v by conjugate orthogonal CG with
     the bilinear form sum_G a(-G) b(G), in which the shifted operator is symmetric, and returns
     dn_i = 4 Re sum_v conj(psi_v) x_{v,i}: for a real field the two frequency terms of chi0(i u)
     are complex conjugates of each other, so one shifted solve per pair gives the real chi0(i u).
     FP64 with Teter's preconditioner, from zero or from kept solutions (STERN_GUESS_PREVIOUS),
     STERN_ERR_UNSUPPORTED otherwise; 0 = the static response. */
  double omega_imag;
  /* nonzero: keep the solutions x of every (v, i) of this call on the device (n_pert x bands x
     n_pw complex FP64, owned by the system until the next keeping call, set_occupied or
     stern_free) as the starts of a later STERN_GUESS_PREVIOUS call */
  int keep_solutions;
} stern_opts;

/* Inner operators of the mixed solve (stern_opts.inner_op). The FP64 outer
   residual always uses P_c (H - eps_v) P_c, so the choice changes only how many
   inner iterations a solve takes and what each costs, never which solutions
   are accepted.
   PROJECTED: q = P_c (H - eps_v) p and z = P_c K r; the projection of z and
     the direction update p = P_c z + beta p share one split-BF16 GEMM pair.
   SHIFTED: H - eps_v + alpha P_v (alpha = twice the occupied band width, at
     least 0.01 Ha; Baroni et al., Rev. Mod. Phys. 73, 515 (2001)) and z = K r;
     fewer GEMMs per iteration, but with Teter's K, which does not commute with
     P_v, more than twice the iterations on the mid cell. */
#define STERN_INNER_PROJECTED 0
#define STERN_INNER_SHIFTED 1

/* kernel classes of the per-launch profile */
#define STERN_K_XINV 0        /* x pencils, inverse (sphere -> pencils) */
#define STERN_K_PLANE_H 1     /* yz planes of the H apply (inverse, x V_loc, forward) */
#define STERN_K_XFWD 2        /* x pencils, forward (pencils -> sphere, + kinetic - eps) */
#define STERN_K_PC_REDUCE 3   /* C = Psi^H Y partial sums (MFMA) */
#define STERN_K_PC_EXPAND 4   /* Y -= Psi C (MFMA) */
#define STERN_K_KB_REDUCE 5   /* P = B^H p (MFMA) */
#define STERN_K_KB_EXPAND 6   /* w += B D P (MFMA) */
#define STERN_K_SUM_PARTS 7   /* split-K partial sums */
#define STERN_K_CG 8          /* fused CG vector updates and FP64 dots */
#define STERN_K_RHS 9         /* yz planes of dV psi_v (right-hand side) */
#define STERN_K_DN 10         /* yz planes of the density response accumulation */
#define STERN_K_OTHER 11
#define STERN_K_PLANE_H32 12  /* FP32 yz planes of the mixed inner H apply */
#define STERN_K_X32 13        /* FP32 x pencils (both directions) */
#define STERN_K_GEMM_BF16 14  /* split-BF16 MFMA GEMMs (KB and P_c) */
#define STERN_K_CG32 15       /* FP32 CG updates with FP64 dots */
#define STERN_K_NET 16        /* learned guess and K: coarse-grid transforms, BF16 MFMA convolutions, head */
#define STERN_NKERNEL 17

typedef struct {
  int n_solves;        /* (band, perturbation) pairs solved */
  int n_converged;     /* pairs with FP64 true relative residual <= tol */
  int n_fallback;      /* pairs re-solved by Teter FP64 PCG from zero: mixed, after max_outer steps;
                          learned guess, after missing tol with the learned start and K */
  int n_restarts;      /* PCG restarts from the FP64 true residual */
  int n_guess_rejected;/* learned guesses rejected (non-finite, or residual >= ||b||): started from zero */
  long long total_iters;
  int max_iters;
  double wall_s;       /* wall time of the call */
  double max_true_resid;
  int* iters;          /* optional caller array [n_solves] (pair order: i major, v minor) */
  double* resid;       /* optional caller array [n_solves] */
  /* filled when opts->profile != 0, per STERN_K_* class: launches, summed
     event time (ms), and the algorithmic HBM bytes / real flops of those
     launches (the minimum the operation must move or compute) */
  long long kernel_launches[STERN_NKERNEL];
  double kernel_ms[STERN_NKERNEL];
  double kernel_bytes[STERN_NKERNEL];
  double kernel_flops[STERN_NKERNEL];
} stern_stats;

/* Plane-wave basis of the wave functions (the representation of Sec. II, whose
 * cost N_pw enters the N_occ^2 x N_PDEP x N_pw count of Sec. II.A).
 * Host only, no GPU needed: basis size, FFT grid and (if miller != NULL) the
 * [n_pw][3] Miller triples in canonical order. */
int stern_basis_info(const stern_cell* cell, int* n_pw, int* fft_n, int32_t* miller);

/* The Hamiltonian of eq. ks for one cell (Sec. II: the ground-state code
 * supplies it; here the model above stands in for it). Builds the basis, V_loc
 * on the grid and the projectors on the GPU. *out receives a system the caller
 * releases with stern_free. Returns STERN_ERR_INVALID_ARG for a bad cell or
 * runtime, STERN_ERR_UNSUPPORTED for grids other than 2^a 3^b in [8, 128] or
 * whose plane kernels do not fit in LDS, STERN_ERR_OOM / _HIP on device errors. */
int stern_init_system(const stern_cell* cell, const stern_runtime* rt, stern_system** out);

/* Sizes of the system's basis (Sec. II): plane waves, FFT grid N, cell volume
 * Omega (bohr^3). Any output pointer may be NULL. Host only. */
int stern_query(const stern_system* sys, int* n_pw, int* fft_n, double* omega);

/* The Miller triples n (G = 2 pi n / L) of the system's canonical order, as
 * [n_pw][3] int32 into caller memory: the order every coefficient array of
 * this ABI uses (psi, sample_x, apply_h / apply_pc rows). Host only. */
int stern_get_miller(const stern_system* sys, int32_t* miller);

/* The occupied Kohn-Sham states psi_v and energies eps_v of eq. ks, the input
 * of the density response of Sec. II.A. psi [n_occ][n_pw] complex in canonical
 * order (orthonormal), eps [n_occ] Ha, both host (mem_kind = STERN_MEM_HOST) or
 * both device pointers; copied. Replaces earlier states. Errors:
 * STERN_ERR_INVALID_ARG, STERN_ERR_OOM, STERN_ERR_HIP. */
int stern_set_occupied(stern_system* sys, int n_occ, const double* psi, const double* eps, int mem_kind);

/* The density response chi0 dV that PDEP iterates on (Sec. II.A, eq. pdep):
 * one Sternheimer solve per (band, field), then dn = 4 Re sum_v psi_v* x_v.
 * dn_r[i] = chi0 dv_r[i] for i < n_pert, summed over bands [band_begin, band_end).
 * dv_r, dn_r: [n_pert][N][N][N] real, host or device per opts->mem_kind.
 * Returns STERN_OK, STERN_WARN_NOT_CONVERGED, or an error. stats may be NULL. */
int stern_apply_chi0(stern_system* sys, int n_pert, const double* dv_r, double* dn_r,
                     const stern_opts* opts, stern_stats* stats);

/* Sec. III.A treats images and bands as independent units of work; this
 * batches independent cells in one call.
 * Batched apply over n_sys independent cells of uneven size (e.g. different L,
 * atom counts, bands and grids): dn_r[k] = chi0_k dv_r[k] for each system k,
 * with n_pert[k] fields. The systems are spread over concurrent HIP streams
 * (one per worker thread, default priority), each system keeping its own
 * workspace and per-solve convergence masks; opts applies to every system.
 * Every system must have had set_occupied; no system may appear twice.
 * stats (may be NULL) accumulates over all systems (iters/resid arrays are
 * ignored). Returns the first error, else STERN_WARN_NOT_CONVERGED if any
 * solve missed tol, else STERN_OK. Synchronous: all work is complete on return. */
int stern_apply_chi0_many(int n_sys, stern_system* const* sys, const int* n_pert, const double* const* dv_r,
                          double* const* dn_r, const stern_opts* opts, stern_stats* stats);

/* ---- PDEP: the eigenpairs of the symmetrised response (Sec. II.A, eq. pdep) ----
 * chi-bar0 = v^{1/2} chi0 v^{1/2}, v^{1/2}(G) = sqrt(4 pi) / |G|, acts on real
 * potentials band-limited to |G|^2 < ecut_pot (G != 0: the long-range G = 0 part
 * is the separate term of eq. pdep). A block Davidson iteration finds its n_eig
 * lowest (most negative) eigenvalues lambda_a and eigenpotentials phi_a; every
 * product chi-bar0 phi is one stern_apply_chi0 over a block of trial potentials
 * (so with the chi0 options' precision, guess and tolerance). Converged pairs stay
 * in the basis but add no new directions. The projected eigenproblem is solved on
 * the host. Grids whose full FP64 yz plane does not fit in LDS (108^3, 128^3) are
 * refused with STERN_ERR_UNSUPPORTED. */
typedef struct {
  int n_eig;            /* eigenpairs wanted (> 0) */
  int block;            /* trial potentials per chi0 apply (0 = n_eig) */
  int max_basis;        /* basis size before a restart from the Ritz vectors (0 = 4 n_eig) */
  int max_iter;         /* Davidson iterations (0 = 50) */
  double tol;           /* converged when ||chi-bar0 phi - lambda phi|| <= tol |lambda| (0 = 1e-6) */
  double ecut_pot_ry;   /* sphere of the potentials, |G|^2 < ecut_pot (0 = ecut / 4) */
  unsigned long long seed;  /* seeded random start */
  const stern_opts* chi0;   /* options of every chi0 apply (mem_kind, band range, samples and
                               profile are ignored) */
} stern_pdep_opts;

typedef struct {
  int iterations;       /* Davidson iterations */
  int n_converged;      /* of the n_eig wanted pairs */
  int chi0_calls;       /* stern_apply_chi0 calls */
  int basis_dim;        /* real dimension of the potential space (2 x half-space G count) */
  long long total_solves;   /* Sternheimer solves over all chi0 calls */
  long long total_cg_iters;
  double max_rel_resid; /* max_a ||chi-bar0 phi_a - lambda_a phi_a|| / |lambda_a| */
  double wall_s;
} stern_pdep_stats;

/* The potential sphere of stern_pdep_davidson: n_g nonzero G with |G|^2 < ecut_pot
 * (0 = ecut / 4), both G and -G, in canonical order; miller (optional) receives
 * their [n_g][3] Miller triples. Host only. */
int stern_pdep_basis(const stern_system* sys, double ecut_pot_ry, int* n_g, int32_t* miller);
/* eig [n_eig] receives the eigenvalues in ascending order; vec (optional, host)
 * [n_eig][n_g] complex coefficients phi_a(G) over stern_pdep_basis's list
 * (phi(-G) = conj phi(G), sum_G |phi(G)|^2 = 1). Needs set_occupied. Returns
 * STERN_OK, STERN_WARN_NOT_CONVERGED (max_iter reached or the basis exhausted),
 * STERN_ERR_STATE when a chi0 apply leaves a solve above its tolerance, or an
 * error. Synchronous. */
int stern_pdep_davidson(stern_system* sys, const stern_pdep_opts* opts, double* eig, double* vec,
                        stern_pdep_stats* stats);

/* The eigenpotentials of stern_pdep_davidson on the grid, w_a(r) = sum_G v^{1/2}(G) phi_a(G) e^{i G.r}
 * (real; v^{1/2}(G) = sqrt(4 pi) / |G|), for n coefficient rows vec [n][n_g] over the basis of
 * ecut_pot_ry (0 = ecut / 4) as stern_pdep_davidson writes them; w [n][N^3] in the grid order of
 * the fields of stern_apply_chi0, host or device per mem_kind. With c_a = lambda_a / (1 - lambda_a)
 * they are the screening of stern_liouville_set_screening (BSE's W, eq. tau). Synchronous. */
int stern_pdep_potentials(stern_system* sys, int n, const double* vec, double ecut_pot_ry, double* w, int mem_kind);

/* ---- learned initial guess and diagonal preconditioner ----
 * A small 3-D convolutional net (3 periodic 3x3x3 layers, 16 channels, ReLU,
 * BF16 weights, FP32 accumulation) on the coarse (N/2)^3 grid, which holds the
 * wave-function sphere exactly. Input channels per (v, i): psi_v(r), the
 * right-hand side b_{v,i}(r) / ||b|| (the sphere part of -P_c dV_i psi_v) and
 * eps_v; output: x0(r) / ||b||, mapped back to the sphere and projected by
 * P_c. A linear head on the grid-averaged second hidden layer of the same net
 * evaluated on (psi_v, 0, eps_v) (one evaluation per band, shared by every
 * field), plus eps_v and T_v, gives 8 knot values z_k on u = log2(|G|^2 / 2 T_v)
 * in [-6, 8]; band v's diagonal preconditioner is
 * K(G) = Teter(G) softplus(z(u)) / ln 2, positive, equal to Teter when the head
 * is zero. STERN_GUESS_LEARNED uses x0 and K, STERN_GUESS_LEARNED_K only K
 * (x0 = 0): a defect-correction inner solve runs to a tolerance relative to its
 * own right-hand side, so there a guess saves little and K carries the gain.
 * The net is fitted to the solutions the plain FP64 path produces (relative L2
 * of x0); then the head to the error left after the guess, minimising
 * ||P_c (K o r0) - e0||^2 / ||e0||^2 with r0 = b - A x0 and e0 = x* - x0.
 * The FP64 true residual still judges every solve: a guess that is non-finite
 * or whose residual is not below ||b|| is dropped (the solve starts from zero),
 * and a solve that misses tol with the learned start and K is re-solved by
 * Teter-preconditioned FP64 PCG from zero (counted in n_fallback).
 * Needs an even grid N with N/2 >= 2 nmax + 1 (STERN_ERR_UNSUPPORTED otherwise). */
typedef struct stern_model stern_model;

typedef struct {
  int epochs;          /* passes over the training solves for the net (0 = 4) */
  int batch;           /* solves per Adam step (0 = 16) */
  double lr;           /* Adam learning rate of the net (0 = 1e-3) */
  int max_solves;      /* cap on training solves, drawn at random (0 = 4096) */
  double tol;          /* tolerance of the FP64 solves that make the targets (0 = 1e-8) */
  unsigned long long seed;
  int prec_epochs;     /* passes for the preconditioner head (0 = 4, < 0 = keep Teter) */
  double prec_lr;      /* its Adam learning rate (0 = 1e-2) */
  int prec_max_solves; /* cap on its training solves (0 = 1024) */
} stern_train_opts;

typedef struct {
  int n_samples;       /* training solves used for the net */
  int steps;           /* Adam steps */
  double loss_first;   /* root mean relative squared L2 error of x0 over the first epoch */
  double loss_last;    /* ... over the last epoch */
  int prec_samples;    /* training solves used for the preconditioner head */
  double prec_loss_first; /* mean ||P_c (K o r0) - e0||^2 / ||e0||^2, first epoch (head at zero = Teter) */
  double prec_loss_last;  /* ... last epoch */
  double wall_s;
} stern_train_stats;

/* New model with seeded random weights (the output layer starts near zero, the
 * preconditioner head at zero). */
int stern_model_create(int device, unsigned long long seed, stern_model** out);
/* Trains on n_sys systems (same coarse grid, each with set_occupied): solves
 * their fields dv_r[k] ([n_pert[k]][N][N][N], host or device per mem_kind) with
 * the plain FP64 path, fits the net to the solutions, then solves them again
 * from the trained guess and fits the preconditioner head. Uses the systems'
 * workspaces and streams; synchronous. */
int stern_model_train(stern_model* m, int n_sys, stern_system* const* sys, const int* n_pert,
                      const double* const* dv_r, int mem_kind, const stern_train_opts* opts,
                      stern_train_stats* stats);
/* Number of float parameters: per conv layer l = 0..2, weights [16 out][27
 * neighbours (dx, dy, dz in -1..1, dz fastest)][16 in] then 16 biases; then the
 * head, weights [8 knots][18 features] and 8 biases. Copy them out / in (host
 * memory, n floats); set_weights enables the head when any of it is nonzero. */
int stern_model_num_params(void);
int stern_model_get_weights(const stern_model* m, float* w, int n);
int stern_model_set_weights(stern_model* m, const float* w, int n);
void stern_model_free(stern_model* m);
/* One Adam step of the net on caller-given coarse-grid data, host memory:
 * in [n][Nc][Nc][Nc][5] floats (per point: Re psi_v, Im psi_v, Re b / |b|,
 * Im b / |b|, eps_v), target [n][Nc][Nc][Nc][2] (Re, Im of x / |b|). Runs the
 * forward pass (out, optional [n][Nc^3][2]: the output before the step), the
 * relative L2 loss per solve (loss, optional [n]), the gradient of the summed
 * loss with respect to the three conv layers (grad, optional: the first
 * 3 x (16 x 27 x 16 + 16) parameters in the get_weights layout), then one Adam
 * step of those parameters with learning rate lr and the gradient averaged over
 * the n solves; the head is untouched. Nc >= 4; synchronous. This is how
 * stern_model_train fits the net, exposed for training on data of the
 * caller's own. */
int stern_model_fit_step(stern_model* m, int Nc, int n, const float* in, const float* target, double lr,
                         float* out, float* loss, float* grad);

/* ---- kernel variants and the autotuner ----
 * Tunables of a system (each keeps its value until set again):
 *   STERN_TUNE_PLANE64   yz-plane kernel of the FP64 H apply: 0 the whole plane
 *                        in LDS, 1 only the active z lines in LDS with per-wave
 *                        transforms (the default when its LDS fits), 2 as 1 with
 *                        the next pair's loads issued ahead (more registers)
 *   STERN_TUNE_PLANE32   the same for the FP32 H apply of the mixed inner solve
 *   STERN_TUNE_GEMM64_WG workgroups the split-K FP64 reduces (Psi^H Y, B^H Y) aim
 *                        for; 0 = built-in default (2048)
 *   STERN_TUNE_GEMM16_WG the same for the split-BF16 reduces; 0 = default (512)
 *   STERN_TUNE_GEMM16_EXPAND tile of the split-BF16 expand (Y += Psi C, B D P):
 *                        0 = 256 x 128 per workgroup of 8 waves, 1 = 128 x 128 of
 *                        16 waves, 2 = 128 x 128 of 8 waves */
#define STERN_TUNE_PLANE64 0
#define STERN_TUNE_PLANE32 1
#define STERN_TUNE_GEMM64_WG 2
#define STERN_TUNE_GEMM16_WG 3
#define STERN_TUNE_GEMM16_EXPAND 4
#define STERN_NTUNE 5

/* value >= 0 sets tunable `which` (STERN_ERR_INVALID_ARG for an unknown
 * tunable or a value the system cannot run, e.g. a plane kernel whose LDS does
 * not fit); value < 0 only queries. Returns the tunable's value. */
int stern_tunable(stern_system* sys, int which, int value);

/* Times every candidate of every tunable on this system's shapes with n_vec
 * synthetic rows (HIP events on the system's stream; needs set_occupied) and
 * keeps the fastest. With cache_path != NULL, choices are read from / appended
 * to that text file, keyed by (GPU arch, grid, active z lines, N_pw, padded
 * N_occ, padded atom count, n_vec); a complete hit times nothing. chosen
 * (optional, STERN_NTUNE ints) receives the values. Returns the number of
 * candidates timed. Synchronous; uses the apply workspace. */
int stern_autotune(stern_system* sys, int n_vec, const char* cache_path, int* chosen);
/* Mean time (ms) of every candidate the calling thread's last stern_autotune
 * timed, as JSON text {"plane64": {"0": t, ...}, ...} ("{}" after a cache hit
 * or before any tuning). Valid until the thread's next autotune call. */
const char* stern_autotune_report(void);

/* The Hamiltonian of eq. ks applied as the solver applies it (FFT stage plus
 * projectors): out = (H - shift_k) c_k for n_vec coefficient rows (canonical
 * order), host or device memory per mem_kind; shift [n_vec] may be NULL (zero).
 * Synchronous. */
int stern_apply_h(stern_system* sys, int n_vec, const double* c, const double* shift, double* out, int mem_kind);

/* The projector onto the empty states, P_c = 1 - sum_v |psi_v><psi_v|, that the
 * DFPT route of Sec. II.A uses to avoid empty states: out = P_c c for n_vec rows
 * (canonical order, host or device per mem_kind). STERN_ERR_STATE before
 * set_occupied. Synchronous. */
int stern_apply_pc(stern_system* sys, int n_vec, const double* c, double* out, int mem_kind);

/* ---- TDDFT Liouville superoperator (Sec. II.C.1, eq. bse_tddft) ----
 * Excitations are sets of auxiliary orbitals A = {a_v}, one per occupied band (Delta gamma =
 * sum_v |a_v><psi_v|), stored as n_exc x n_occ rows of n_pw complex coefficients in canonical
 * order ([n_exc][n_occ][n_pw], interleaved re, im). The paper names the terms of the Liouville
 * superoperator but not their formulas; here: Tamm-Dancoff, closed-shell singlet excitations,
 * Hartree kernel (the model Hamiltonian has no exchange-correlation functional, so K1d = 0 unless
 * a fraction of bare exchange is set, stern_liouville_set_kernel):
 *   (L A)_v = P_c (H - eps_v) a_v + 2 P_c [ V[rho_A] psi_v ],  rho_A = sum_v conj(psi_v) a_v,
 *   V[rho](r) = sum_{0 < |q|^2 <= 4 Ecut} (4 pi / |q|^2) rho(q) e^{i q.r},
 * applied to P_c A. L is Hermitian in <A|B> = sum_v <a_v|b_v> and positive definite when the gap
 * is open. FP64 throughout; grids up to 96^3 (STERN_ERR_UNSUPPORTED above: the Hartree stage
 * keeps whole FP64 planes in LDS). STERN_ERR_STATE before set_occupied.
 *
 * out = L A, host or device arrays per mem_kind (they may not overlap). Synchronous. */
int stern_liouville_apply(stern_system* sys, int n_exc, const double* a, double* out, int mem_kind);

/* Hybrid TDDFT: a fraction alpha_x in [0, 1] of bare exchange in the direct term (Sec. II.C.1,
 * the Coulomb integrals of occupied pairs of eq. tau_u), used by every later Liouville call on
 * this system (0, the default, leaves K1d = 0):
 *   (K1d A)_v = alpha_x P_c sum_w tau_{wv} a_w,   tau_{wv}(r) = V[conj(psi_w) psi_v](r),
 * with V as above (q = 0 omitted), and L = D + K1e - K1d. Each apply then forms the n_occ^2
 * pair potentials again (n_occ Poisson solves per band). STERN_ERR_INVALID_ARG outside [0, 1]. */
int stern_liouville_set_kernel(stern_system* sys, double alpha_x);

/* BSE: the screened interaction of eq. tau in the direct term, as a low-rank addition to the bare
 * part set by stern_liouville_set_kernel:
 *   V_W[rho](r) = alpha_x V[rho](r) + sum_a w_a(r) c_a <w_a, rho>,  <f, g> = N^-3 sum_j f(r_j) g(r_j),
 *   tau_{wv} = V_W[conj(psi_w) psi_v],  (K1d A)_v = P_c sum_w tau_{wv} a_w,
 * for n real potentials w [n][N^3] (grid order of the fields of stern_apply_chi0) and weights c [n],
 * host or device per mem_kind (copied). With the PDEP eigenpairs (lambda_a, phi_a) of Sec. II.A
 * (eq. pdep) normalised to a unit cell average of phi_a^2, w_a = v^{1/2} phi_a and
 * c_a = lambda_a / (1 - lambda_a) give W = v + v^{1/2} ((1 - chi-bar0)^{-1} - 1) v^{1/2} on their span,
 * and alpha_x = 1 makes K1d BSE's direct term. n = 0 removes the screening. */
int stern_liouville_set_screening(stern_system* sys, int n, const double* w, const double* c, int mem_kind);

/* Linear systems L z_e = b_e of the Liouville superoperator, as the Z-vector equations of
 * excited-state forces pose them (Sec. II.C.2), for n_exc right-hand sides b [n_exc][n_occ][n_pw]
 * (projected on range(P_c) first): preconditioned CG with one block (all band rows) per
 * excitation, Teter's diagonal per band, from z = 0, at most max_iter (0 = 1000) iterations,
 * accepted on the true residual ||b - L z|| <= tol ||b|| (norms over all bands). iters and resid
 * (host, n_exc each) may be NULL. Returns STERN_OK, STERN_WARN_NOT_CONVERGED (z written) or an
 * error. Synchronous. */
int stern_liouville_solve(stern_system* sys, int n_exc, const double* b, double* z, double tol, int max_iter,
                          int mem_kind, int* iters, double* resid);

/* The n_eig lowest excitation energies w_s of eq. bse_tddft and their auxiliary orbitals by block
 * Davidson (Sec. II.C.1; WEST shares one Davidson between this operator and chi-bar0, Sec. IV):
 * the basis stays on the device, Rayleigh-Ritz through FP64 GEMMs and Jacobi rotations of the
 * projected Hermitian matrix on the host, corrections P_c K (L x - w x) with Teter's K per band,
 * converged pairs kept in the basis without new directions, and when the basis would exceed
 * max_basis a restart from its lowest max(n_eig, max_basis / 2) Ritz vectors. Converged when
 * ||L x - w x|| <= tol |w| (||x|| = 1 over all bands).
 * block (0 = n_eig) new directions per iteration, max_basis (0 = max(8 n_eig, n_eig + 4 block)),
 * max_iter (0 = 200), seed of the random start. eig [n_eig] ascending (host); vec (host, may be
 * NULL) [n_eig][n_occ][n_pw] canonical order; n_iter, max_resid (host) may be NULL. Returns
 * STERN_OK, STERN_WARN_NOT_CONVERGED (max_iter reached or the basis exhausted) or an error. */
int stern_liouville_davidson(stern_system* sys, int n_eig, int block, int max_basis, int max_iter, double tol,
                             unsigned long long seed, double* eig, double* vec, int* n_iter, double* max_resid);

/* Absorption spectra by Lanczos (Sec. II.C.1: over a broad range of energies without the
 * excitation energies or their orbitals): the Hermitian Lanczos chain of L from d_v = P_c dV psi_v,
 * all bands of one real field dV [N^3] (the perturbation that couples to the light, e.g. a long-
 * wavelength potential; host or device per mem_kind). q_0 = d / ||d||; for k = 0 .. n_steps - 1:
 * w = L q_k - beta_{k-1} q_{k-1}, alpha_k = <q_k|w>, w -= alpha_k q_k, beta_k = ||w||,
 * q_{k+1} = w / beta_k (inner products over all bands, no reorthogonalisation). Writes alpha and
 * beta [n_steps] and norm2 = ||d||^2 (host); a chain that closes early is padded with zeros.
 * STERN_ERR_INVALID_ARG if d = 0. Synchronous. */
int stern_liouville_lanczos(stern_system* sys, const double* dv, int n_steps, double* alpha, double* beta,
                            double* norm2, int mem_kind);

/* S(w) = -Im <d|(w + i eta - L)^{-1}|d> / pi from a Lanczos chain, as the continued fraction
 * norm2 / (z - alpha_0 - beta_0^2 / (z - alpha_1 - ...)), z = w + i eta, closed after the last step
 * (host only; eta > 0). */
int stern_lanczos_spectrum(int n_steps, const double* alpha, const double* beta, double norm2, int n_omega,
                           const double* omega, double eta, double* out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): out = P_c c as
 * stern_apply_pc computes it (the same kernels, so bitwise the same result),
 * device pointers only, c and out [n_vec][n_pw] complex in canonical order
 * (they may not overlap). Every temporary lives in a fixed scratch area of
 * STERN_NOALLOC_SCRATCH_BYTES per device, held from the first stern_init_system
 * on that device to the end of the process: 16 n_vec (npw_pad + (s + 1)
 * nocc_pad) bytes, with npw_pad and nocc_pad the plane-wave and band counts
 * rounded up to multiples of 64 and s the split-K factor of the reduce;
 * STERN_ERR_INVALID_ARG when that exceeds the area (about 230 rows of the
 * 72^3, 128-band cell). Enqueued on the system's stream without any
 * synchronisation or allocation; the result is ready when that stream's work
 * is. All calls on one GPU share its area and it keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams, other
 * threads) race, so issue them on one stream. */
#define STERN_NOALLOC_SCRATCH_BYTES (64u << 20)
int stern_apply_pc_noalloc(stern_system* sys, int n_vec, const double* c, double* out);

/* Releases the system and every device buffer it holds (through the caller's
 * dev_free when one was given). NULL-safe. */
void stern_free(stern_system* sys);

/* Message of the last failing call on the calling thread (never NULL). */
const char* stern_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
