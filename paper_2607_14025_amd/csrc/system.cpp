// C ABI of the Sternheimer chi0 library: system setup, occupied states, the
// batched projected-PCG driver and the density response.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stern.h"
#include "basis.hpp"
#include "hostla.hpp"
#include "kernels.hpp"

using namespace stern;

namespace {

thread_local std::string g_err;
thread_local std::string g_tune_report = "{}";  // per-candidate times of this thread's last autotune

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPOK(expr)                                                                                    \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return fail(e_ == hipErrorOutOfMemory ? STERN_ERR_OOM : STERN_ERR_HIP,       \
                                      "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                                      __LINE__);                                                       \
  } while (0)

#define CHECKED(expr)         \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ < 0) return rc_;  \
  } while (0)

// Device allocator of a system: the caller's callbacks (stern_runtime) or, when
// they are NULL, hipMalloc / hipFree. Entry points make their system's allocator
// the current one of the calling thread (Scope); a buffer remembers the allocator
// that gave it its memory and returns the memory there.
struct Alloc {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
thread_local const Alloc* tl_alloc = nullptr;

// A device allocation that only grows.
struct DBuf {
  void* p = nullptr;
  size_t n = 0;
  Alloc al;  // where p came from (al.alloc == nullptr: hipMalloc)
  int ensure(size_t bytes) {
    if (bytes <= n) return 0;
    release();
    if (bytes == 0) return 0;
    if (tl_alloc && tl_alloc->alloc) {
      p = tl_alloc->alloc(bytes, tl_alloc->ctx);
      if (!p) return fail(STERN_ERR_OOM, "the caller's dev_alloc(%zu) returned NULL", bytes);
      al = *tl_alloc;
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        p = nullptr;
        return fail(STERN_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
      }
      al = Alloc();
    }
    n = bytes;
    return 0;
  }
  void release() {
    if (p) {
      if (al.free) {
        // hipFree waits for the work that may still use the memory; a caller's
        // allocator may hand it out again at once, so wait here instead
        (void)hipDeviceSynchronize();
        al.free(p, al.ctx);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    n = 0;
    al = Alloc();
  }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

int upload(DBuf& d, const void* src, size_t bytes, hipStream_t st) {
  CHECKED(d.ensure(bytes));
  if (bytes) HIPOK(hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, st));
  return 0;
}

}  // namespace

// Fixed per-device scratch area of stern_apply_pc_noalloc: every temporary of
// that entry point lives here, so it never allocates. In host code the array's
// name is only a stand-in; its device address comes from hipGetSymbolAddress,
// taken once per device with that device current and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[STERN_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // [device] address of `scratch` on that device

// Device address of the scratch area on `device` (which must be current).
int scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0) return fail(STERN_ERR_INVALID_ARG, "bad device %d", device);
  if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(STERN_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                  hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return 0;
}
}  // namespace

struct stern_system {
  int device = 0;
  Alloc alloc;  // device allocator of every buffer of this system
  int n_cu = 256;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;  // non-blocking stream for graph capture (created on demand)
  CellParams cell;
  HostBasis hb;
  int n_atoms = 0, natoms_pad = 0;
  // static device data
  DBuf col_start, col_len, col_xmin, col_pos, zl, ycol, g2h, tw64, tw32, v_r, v_r32, v_t, v_t32, kb, perm;
  // yz-plane kernel of the H apply per precision: 0 full-plane, 1 compact wave-local
  int plane_var64 = 1, plane_var32 = 1;
  // split-K workgroup targets of the FP64 and split-BF16 reduces (0 = default)
  int gemm64_wg = 0, gemm16_wg = 0;
  int gemm16_expand = 0;  // tile variant of the split-BF16 expand
  size_t lds_max = 160 * 1024;
  // occupied states
  int n_occ = 0, nocc_pad = 0;
  bool have_occ = false;
  std::vector<double> eps, invT;
  double alpha_pv = 0.0;  // shift of the occupied subspace in the mixed inner operator
  DBuf psi, psi_r;
  // split BF16 copies of Psi and of the KB rows (row and transposed layouts)
  DBuf psi_hi, psi_lo, psiT_hi, psiT_lo, kb_hi, kb_lo, kbT_hi, kbT_lo;
  // projected FP32 operator: transposed split of the stacked rows [P_c KB (natoms_pad); Psi (nocc_pad)];
  // proj_m = 0 without atoms
  DBuf projT_hi, projT_lo;
  int proj_m = 0;
  // workspace
  DBuf wx, wr, wp, wq, wz, wb, pen, cpart, cpart2, cmat, sv_eps, sv_invT, sv_band, sv_pert, sv_bb, sv_rz, sv_rr, sv_flag,
      sv_iters, sv_tres, list_act, list_f, pert_out, dv_dev, dn_dev, tmp_in, tmp_out;
  DBuf m_d, m_r, m_p, m_q, m_z, m_rz, m_rr0, m_beta, m_flag;  // mixed inner solve
  DBuf m_cnt;                 // device count of the inner solve's active list (list_f)
  DBuf negk;                  // [npw_pad] index of -G of each coefficient (column order)
  DBuf sv_rzi;                // [nbatch] imaginary parts of the shifted solves' (r, z)_J
  // solutions kept by a call with keep_solutions, [n_pert][bands][npw_pad] complex FP64, valid
  // while keep_np > 0 for that call's field count and band range [keep_v0, keep_v1)
  DBuf xkeep;
  int keep_np = 0, keep_v0 = 0, keep_v1 = 0;
  const int* live = nullptr;  // while set, FP32 launches cover only the first *live list entries
  // coarse (N/2)^3 grid of the learned guess, when it holds the sphere
  bool have_coarse = false;
  HostBasis hbc;
  DBuf c_col_start, c_col_len, c_col_xmin, c_col_pos, c_zl, c_ycol, c_tw64, psi_c, c_pen, c_field, net_a0, net_a1,
      net_a2, net_out, g_rej, net_feat, net_coef, kprec, band_eps, band_invT, band_feat;
  int ws_solves = 0, ws32_solves = 0;
  // 4 Ecut sphere on the same grid (densities and the Hartree potential of the Liouville apply),
  // built at its first use, and the Liouville work buffers
  bool have_dens = false;
  HostBasis hbd;
  DBuf d_col_start, d_col_len, d_col_xmin, d_col_pos, d_zl, d_ycol, d_g2h;
  DBuf lv_ar, lv_rho, lv_rhog, lv_pend, lv_k, lv_eps, lv_dot, lv_coef, lv_tau, lv_acc;
  double lv_alpha = 0.0;  // fraction of bare exchange in the direct term K1d
  // screening of the direct term: n_scr real potentials [n_scr][N^3] and weights, and projections
  int n_scr = 0;
  DBuf scr_w, scr_c, scr_proj;
  DBuf dv_V, dv_W, dv_X, dv_LX, dv_T, dv_LT, dv_part, dv_cm;  // Liouville Davidson

  // per-launch event profile (opts->profile)
  struct Rec {
    int cls;
    int ev;
    double bytes, flops;
  };
  bool prof_on = false;
  std::vector<hipEvent_t> events;
  std::vector<Rec> recs;
  size_t ev_used = 0;

  FftGeom geom() const {
    FftGeom g;
    g.N = hb.N;
    g.npw = hb.npw;
    g.npw_pad = hb.npw_pad;
    g.ncol = hb.ncol;
    g.ncol_pad = hb.ncol_pad;
    g.nza = hb.nza;
    g.col_start = col_start.as<int>();
    g.col_len = col_len.as<int>();
    g.col_xmin = col_xmin.as<int>();
    g.col_pos = col_pos.as<int>();
    g.zl = zl.as<int>();
    g.ycol = ycol.as<int>();
    g.zact_lo = hb.zact_lo;
    g.zact_hi = hb.zact_hi;
    g.n_cu = n_cu;
    g.g2h = g2h.as<double>();
    g.tw64 = tw64.as<Z64>();
    g.tw32 = tw32.as<Z32>();
    g.live = live;
    return g;
  }

  FftGeom geom_d() const {
    FftGeom g;
    g.N = hbd.N;
    g.npw = hbd.npw;
    g.npw_pad = hbd.npw_pad;
    g.ncol = hbd.ncol;
    g.ncol_pad = hbd.ncol_pad;
    g.nza = hbd.nza;
    g.col_start = d_col_start.as<int>();
    g.col_len = d_col_len.as<int>();
    g.col_xmin = d_col_xmin.as<int>();
    g.col_pos = d_col_pos.as<int>();
    g.zl = d_zl.as<int>();
    g.ycol = d_ycol.as<int>();
    g.zact_lo = hbd.zact_lo;
    g.zact_hi = hbd.zact_hi;
    g.n_cu = n_cu;
    g.g2h = d_g2h.as<double>();
    g.tw64 = tw64.as<Z64>();  // same grid
    g.tw32 = nullptr;
    return g;
  }

  FftGeom geom_c() const {
    FftGeom g;
    g.N = hbc.N;
    g.npw = hbc.npw;
    g.npw_pad = hbc.npw_pad;
    g.ncol = hbc.ncol;
    g.ncol_pad = hbc.ncol_pad;
    g.nza = hbc.nza;
    g.col_start = c_col_start.as<int>();
    g.col_len = c_col_len.as<int>();
    g.col_xmin = c_col_xmin.as<int>();
    g.col_pos = c_col_pos.as<int>();
    g.zl = c_zl.as<int>();
    g.ycol = c_ycol.as<int>();
    g.zact_lo = hbc.zact_lo;
    g.zact_hi = hbc.zact_hi;
    g.n_cu = n_cu;
    g.g2h = g2h.as<double>();
    g.tw64 = c_tw64.as<Z64>();
    g.tw32 = nullptr;
    return g;
  }

  void release_all() {
    DBuf* all[] = {&ycol, &tw32, &v_r32, &col_start, &col_len,  &col_xmin, &col_pos, &zl,       &g2h,     &tw64,     &v_r,      &kb,
                   &perm,      &psi,      &psi_r,    &wx,      &wr,       &wp,      &wq,       &wz,       &wb,
                   &pen,       &cpart,    &cmat,     &sv_eps,  &sv_invT,  &sv_band, &sv_pert,  &sv_bb,    &sv_rz,
                   &sv_rr,     &sv_flag,  &sv_iters, &sv_tres, &list_act, &list_f,  &pert_out, &dv_dev,   &dn_dev,
                   &tmp_in,    &tmp_out,  &psi_hi,  &psi_lo,   &psiT_hi, &psiT_lo,  &kb_hi,    &kb_lo,
                   &kbT_hi,    &kbT_lo,   &m_d,     &m_r,      &m_p,     &m_q,      &m_z,      &m_rz,  &m_beta,
                   &m_rr0,     &m_flag,   &c_col_start, &c_col_len, &c_col_xmin, &c_col_pos, &c_zl, &c_ycol,
                   &c_tw64,    &psi_c,    &c_pen,   &c_field,  &net_a0,  &net_a1,   &net_a2,   &net_out,
                   &g_rej,     &net_feat, &net_coef, &kprec,  &v_t,     &v_t32,    &band_eps, &band_invT,
                   &band_feat, &projT_hi, &projT_lo, &cpart2, &m_cnt, &negk, &sv_rzi, &xkeep,
                   &d_col_start, &d_col_len, &d_col_xmin, &d_col_pos, &d_zl, &d_ycol, &d_g2h, &lv_ar, &lv_rho,
                   &lv_rhog, &lv_pend, &lv_k, &lv_eps, &lv_dot, &lv_coef, &lv_tau, &lv_acc, &scr_w, &scr_c, &scr_proj, &dv_V, &dv_W, &dv_X, &dv_LX,
                   &dv_T, &dv_LT, &dv_part, &dv_cm};
    for (DBuf* d : all) d->release();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    events.clear();
    if (own_stream) (void)hipStreamDestroy(own_stream);
    own_stream = nullptr;
  }
};

// Weights of the learned-guess net: per layer [co][27][ci] floats then 16 biases.
struct stern_model {
  int device = 0;
  DBuf w, m, v, grad, part, wbf, wtf;
  int step = 0;
  bool trained = false;
  bool prec_trained = false;  // the preconditioner head has been fitted (else Teter is used)
  int prec_step = 0;
  DBuf a0, a1, a2, out, tgt, g3, g2, gbf, loss, din, dtgt;  // training workspace
  DBuf r0set, e0set, fset, fb, coef, gc, kb, idx;          // preconditioner-head training
  static constexpr int LP = kNetLayerParams;
  static constexpr int WN = kNetChannels * 27 * kNetChannels;
  static constexpr int HEAD = kNetLayers * LP;  // offset of the preconditioner head
  const __bf16* wb(int l) const { return wbf.as<__bf16>() + (size_t)l * WN; }
  const float* bias(int l) const { return w.as<float>() + (size_t)l * LP + WN; }
  const float* head() const { return w.as<float>() + HEAD; }
  void release_all() {
    DBuf* all[] = {&w, &m, &v, &grad, &part, &wbf, &wtf, &a0, &a1, &a2, &out, &tgt, &g3, &g2, &gbf, &loss, &din,
                   &dtgt, &r0set, &e0set, &fset, &fb, &coef, &gc, &kb, &idx};
    for (DBuf* d : all) d->release();
  }
};

namespace {

// Launches `launch` on the system stream; with profiling on, brackets it with
// an event pair and records the algorithmic bytes and flops of the launch.
template <class F>
int timed(stern_system* S, int cls, double bytes, double flops, F&& launch) {
  if (!S->prof_on) {
    launch();
    return 0;
  }
  while (S->events.size() < S->ev_used + 2) {
    hipEvent_t e;
    HIPOK(hipEventCreate(&e));
    S->events.push_back(e);
  }
  const int ev = (int)S->ev_used;
  S->ev_used += 2;
  HIPOK(hipEventRecord(S->events[ev], S->stream));
  launch();
  HIPOK(hipEventRecord(S->events[ev + 1], S->stream));
  S->recs.push_back({cls, ev, bytes, flops});
  return 0;
}

// ---- operator pieces on solve rows `list` (device ints) of batch buffers ----

// Y <- P_c Y on rows list[0..n)
int apply_pc_rows(stern_system* S, Z64* Y, const int* list, int n) {
  if (n <= 0) return 0;
  const int K = S->hb.npw_pad;
  const double npw = S->hb.npw, m = S->n_occ, zb = sizeof(Z64);
  const int ns = choose_nsplit(S->nocc_pad, n, K, S->gemm64_wg);
  CHECKED(timed(S, STERN_K_PC_REDUCE, zb * npw * (n + m), 8.0 * m * npw * n, [&] {
    launch_zgemm_reduce(S->psi.as<Z64>(), S->nocc_pad, Y, K, list, n, K, S->cpart.as<Z64>(), ns, S->stream);
  }));
  CHECKED(timed(S, STERN_K_SUM_PARTS, zb * m * n * (ns + 1), 0.0, [&] {
    launch_sum_parts(S->cpart.as<Z64>(), ns, n, S->nocc_pad, -1.0, S->cmat.as<Z64>(), S->stream);
  }));
  CHECKED(timed(S, STERN_K_PC_EXPAND, zb * npw * (2.0 * n + m), 8.0 * m * npw * n, [&] {
    launch_zgemm_expand(S->psi.as<Z64>(), S->nocc_pad, S->cmat.as<Z64>(), Y, K, list, n, K, S->stream);
  }));
  return 0;
}

// FFT flops of the yz pass of one vector's H apply, 5 L log2 L per length-L
// transform: per plane the inverse and forward y transforms of the nza active z
// lines and the inverse and forward z transforms of all N rows, plus the V
// multiply (2 flops per complex point)
double plane_flops(const stern_system* S) {
  const double N = S->hb.N, nza = S->hb.nza;
  return N * ((2.0 * nza + 2.0 * N) * 5.0 * N * std::log2(N) + 2.0 * N * N);
}

// out = (H - eps_s) in on rows list (without projection); eps per row index
int apply_h_rows(stern_system* S, const Z64* in, Z64* out, const int* list, int n, const double* eps_rows) {
  if (n <= 0) return 0;
  const FftGeom g = S->geom();
  const int K = S->hb.npw_pad;
  const double zb = sizeof(Z64), npw = S->hb.npw, N = S->hb.N, pen = N * S->hb.ncol * zb;
  CHECKED(timed(S, STERN_K_XINV, n * (npw * zb + pen), 0.0,
                [&] { launch_xinv(g, in, list, n, S->pen.as<Z64>(), S->stream); }));
  CHECKED(timed(S, STERN_K_PLANE_H, n * 2.0 * pen + N * N * N * sizeof(double), n * plane_flops(S),
                [&] {
                  if (S->plane_var64 >= 1)
                    launch_plane_hw<double>(g, S->pen.as<Z64>(), list, n, S->v_t.as<double>(), S->plane_var64 == 2,
                                            S->stream);
                  else
                    launch_plane_vloc(g, S->pen.as<Z64>(), list, n, S->v_r.as<double>(), S->stream);
                }));
  CHECKED(timed(S, STERN_K_XFWD, n * (pen + 2.0 * npw * zb), 0.0,
                [&] { launch_xfwd(g, S->pen.as<Z64>(), list, n, out, 1, in, eps_rows, 0.0, S->stream); }));
  if (S->n_atoms > 0) {
    const double na = S->n_atoms;
    const int ns = choose_nsplit(S->natoms_pad, n, K, S->gemm64_wg);
    CHECKED(timed(S, STERN_K_KB_REDUCE, zb * npw * (n + na), 8.0 * na * npw * n, [&] {
      launch_zgemm_reduce(S->kb.as<Z64>(), S->natoms_pad, in, K, list, n, K, S->cpart.as<Z64>(), ns, S->stream);
    }));
    CHECKED(timed(S, STERN_K_SUM_PARTS, zb * na * n * (ns + 1), 0.0, [&] {
      launch_sum_parts(S->cpart.as<Z64>(), ns, n, S->natoms_pad, S->cell.D, S->cmat.as<Z64>(), S->stream);
    }));
    CHECKED(timed(S, STERN_K_KB_EXPAND, zb * npw * (2.0 * n + na), 8.0 * na * npw * n, [&] {
      launch_zgemm_expand(S->kb.as<Z64>(), S->natoms_pad, S->cmat.as<Z64>(), out, K, list, n, K, S->stream);
    }));
  }
  return 0;
}

// ---- mixed-precision operator pieces (FP32 vectors, split-BF16 GEMMs) ----

// Y <- P_c Y (FP32 rows, BF16 MFMA)
int apply_psi32_rows(stern_system* S, const Z32* X, Z32* Y, const int* list, int n, float scale);
int apply_pc32_rows(stern_system* S, Z32* Y, const int* list, int n) { return apply_psi32_rows(S, Y, Y, list, n, -1.f); }

// Y += scale Psi (Psi^H X) on rows `list` (FP32 rows, split-BF16 MFMA); X may be Y
int apply_psi32_rows(stern_system* S, const Z32* X, Z32* Y, const int* list, int n, float scale) {
  if (n <= 0) return 0;
  const int K = S->hb.npw_pad;
  const double npw = S->hb.npw, m = S->n_occ;
  const int ns = choose_nsplit_bf16(S->nocc_pad, n, K, S->gemm16_wg);
  Z32* cp = S->cpart.as<Z32>();
  __bf16* cm = S->cmat.as<__bf16>();
  CHECKED(timed(S, STERN_K_GEMM_BF16, 8.0 * npw * (n + m), 8.0 * m * npw * n, [&] {
    launch_reduce_bf16(S->psi_hi.as<__bf16>(), S->psi_lo.as<__bf16>(), S->nocc_pad, X, K, list, n, K, cp, ns,
                       S->stream, S->live);
  }));
  CHECKED(timed(S, STERN_K_SUM_PARTS, 8.0 * m * n * (ns + 1), 0.0,
                [&] { launch_sum_parts32(cp, ns, n, S->nocc_pad, scale, cm, S->stream, S->live); }));
  CHECKED(timed(S, STERN_K_GEMM_BF16, 8.0 * npw * (2.0 * n + m), 8.0 * m * npw * n, [&] {
    launch_expand_bf16(S->psiT_hi.as<__bf16>(), S->psiT_lo.as<__bf16>(), S->nocc_pad, cm, Y, K, list, n, K,
                       S->gemm16_expand, S->stream, nullptr, nullptr, S->live);
  }));
  return 0;
}

// p = P_c z + beta p on rows `list` (FP32 rows, split-BF16 MFMA): the projection
// of z and the CG direction update in one reduce and one expand; z is left as it is
int apply_pc32_update(stern_system* S, const Z32* Z, Z32* P, const double* beta, const int* list, int n) {
  if (n <= 0) return 0;
  const int K = S->hb.npw_pad;
  const double npw = S->hb.npw, m = S->n_occ;
  const int ns = choose_nsplit_bf16(S->nocc_pad, n, K, S->gemm16_wg);
  Z32* cp = S->cpart.as<Z32>();
  __bf16* cm = S->cmat.as<__bf16>();
  CHECKED(timed(S, STERN_K_GEMM_BF16, 8.0 * npw * (n + m), 8.0 * m * npw * n, [&] {
    launch_reduce_bf16(S->psi_hi.as<__bf16>(), S->psi_lo.as<__bf16>(), S->nocc_pad, Z, K, list, n, K, cp, ns,
                       S->stream, S->live);
  }));
  CHECKED(timed(S, STERN_K_SUM_PARTS, 8.0 * m * n * (ns + 1), 0.0,
                [&] { launch_sum_parts32(cp, ns, n, S->nocc_pad, -1.f, cm, S->stream, S->live); }));
  CHECKED(timed(S, STERN_K_GEMM_BF16, 8.0 * npw * (3.0 * n + m), 8.0 * m * npw * n, [&] {
    launch_expand_bf16(S->psiT_hi.as<__bf16>(), S->psiT_lo.as<__bf16>(), S->nocc_pad, cm, const_cast<Z32*>(Z), K,
                       list, n, K, S->gemm16_expand, S->stream, P, beta, S->live);
  }));
  return 0;
}

// out = P_c (H - eps_s) in for FP32 rows: FP32 FFTs, then one split-BF16 expand
// over the stacked rows [P_c KB; Psi] that adds the projected KB term and removes
// Psi^H of the local part. The KB rows are projected once at set-up, so the two
// reduces (KB rows against `in`, Psi against the local part) are independent of
// each other and the coefficients need no further product.
int apply_h32_rows(stern_system* S, const Z32* in, Z32* out, const int* list, int n, const double* eps_rows);
int apply_hproj32_rows(stern_system* S, const Z32* in, Z32* out, const int* list, int n, const double* eps_rows) {
  if (n <= 0) return 0;
  if (S->proj_m == 0) {  // no atoms: local part, then P_c
    CHECKED(apply_h32_rows(S, in, out, list, n, eps_rows));
    return apply_pc32_rows(S, out, list, n);
  }
  const FftGeom g = S->geom();
  const int K = S->hb.npw_pad;
  const double zb = sizeof(Z32), npw = S->hb.npw, N = S->hb.N, pen = N * S->hb.ncol * zb;
  const double na = S->n_atoms, m = S->n_occ;
  Z32* pen32 = S->pen.as<Z32>();
  CHECKED(timed(S, STERN_K_X32, n * (npw * zb + pen), 0.0,
                [&] { launch_xinv<float>(g, in, list, n, pen32, S->stream); }));
  CHECKED(timed(S, STERN_K_PLANE_H32, n * 2.0 * pen + N * N * N * sizeof(float), n * plane_flops(S),
                [&] {
                  if (S->plane_var32 >= 1)
                    launch_plane_hw<float>(g, pen32, list, n, S->v_t32.as<float>(), S->plane_var32 == 2, S->stream);
                  else
                    launch_plane_vloc<float>(g, pen32, list, n, S->v_r32.as<float>(), S->stream);
                }));
  CHECKED(timed(S, STERN_K_X32, n * (pen + 2.0 * npw * zb), 0.0,
                [&] { launch_xfwd<float>(g, pen32, list, n, out, 1, in, eps_rows, 0.0, S->stream); }));
  const int Ma = S->natoms_pad, Mb = S->nocc_pad;
  const int ns_a = choose_nsplit_bf16(Ma, n, K, S->gemm16_wg), ns_b = choose_nsplit_bf16(Mb, n, K, S->gemm16_wg);
  Z32 *cpa = S->cpart.as<Z32>(), *cpb = S->cpart2.as<Z32>();
  __bf16* cm = S->cmat.as<__bf16>();
  CHECKED(timed(S, STERN_K_GEMM_BF16, zb * npw * (n + na), 8.0 * na * npw * n, [&] {
    launch_reduce_bf16(S->kb_hi.as<__bf16>(), S->kb_lo.as<__bf16>(), Ma, in, K, list, n, K, cpa, ns_a, S->stream,
                       S->live);
  }));
  CHECKED(timed(S, STERN_K_GEMM_BF16, zb * npw * (n + m), 8.0 * m * npw * n, [&] {
    launch_reduce_bf16(S->psi_hi.as<__bf16>(), S->psi_lo.as<__bf16>(), Mb, out, K, list, n, K, cpb, ns_b,
                       S->stream, S->live);
  }));
  CHECKED(timed(S, STERN_K_SUM_PARTS, zb * n * (na * (ns_a + 1) + m * (ns_b + 1)), 0.0, [&] {
    launch_sum_proj32(cpa, ns_a, cpb, ns_b, n, Ma, Mb, (float)S->cell.D, cm, S->stream, S->live);
  }));
  CHECKED(timed(S, STERN_K_GEMM_BF16, zb * npw * (2.0 * n + na + m), 8.0 * (na + m) * npw * n, [&] {
    launch_expand_bf16(S->projT_hi.as<__bf16>(), S->projT_lo.as<__bf16>(), S->proj_m, cm, out, K, list, n, K,
                       S->gemm16_expand, S->stream, nullptr, nullptr, S->live);
  }));
  return 0;
}

// out = (H - eps_s) in for FP32 rows: FP32 FFTs, BF16 KB projectors
int apply_h32_rows(stern_system* S, const Z32* in, Z32* out, const int* list, int n, const double* eps_rows) {
  if (n <= 0) return 0;
  const FftGeom g = S->geom();
  const int K = S->hb.npw_pad;
  const double zb = sizeof(Z32), npw = S->hb.npw, N = S->hb.N, pen = N * S->hb.ncol * zb;
  Z32* pen32 = S->pen.as<Z32>();
  CHECKED(timed(S, STERN_K_X32, n * (npw * zb + pen), 0.0,
                [&] { launch_xinv<float>(g, in, list, n, pen32, S->stream); }));
  CHECKED(timed(S, STERN_K_PLANE_H32, n * 2.0 * pen + N * N * N * sizeof(float), n * plane_flops(S),
                [&] {
                  if (S->plane_var32 >= 1)
                    launch_plane_hw<float>(g, pen32, list, n, S->v_t32.as<float>(), S->plane_var32 == 2, S->stream);
                  else
                    launch_plane_vloc<float>(g, pen32, list, n, S->v_r32.as<float>(), S->stream);
                }));
  CHECKED(timed(S, STERN_K_X32, n * (pen + 2.0 * npw * zb), 0.0,
                [&] { launch_xfwd<float>(g, pen32, list, n, out, 1, in, eps_rows, 0.0, S->stream); }));
  if (S->n_atoms > 0) {
    const double na = S->n_atoms;
    const int ns = choose_nsplit_bf16(S->natoms_pad, n, K, S->gemm16_wg);
    Z32* cp = S->cpart.as<Z32>();
    __bf16* cm = S->cmat.as<__bf16>();
    CHECKED(timed(S, STERN_K_GEMM_BF16, zb * npw * (n + na), 8.0 * na * npw * n, [&] {
      launch_reduce_bf16(S->kb_hi.as<__bf16>(), S->kb_lo.as<__bf16>(), S->natoms_pad, in, K, list, n, K, cp, ns,
                         S->stream, S->live);
    }));
    CHECKED(timed(S, STERN_K_SUM_PARTS, zb * na * n * (ns + 1), 0.0,
                  [&] { launch_sum_parts32(cp, ns, n, S->natoms_pad, (float)S->cell.D, cm, S->stream, S->live); }));
    CHECKED(timed(S, STERN_K_GEMM_BF16, zb * npw * (2.0 * n + na), 8.0 * na * npw * n, [&] {
      launch_expand_bf16(S->kbT_hi.as<__bf16>(), S->kbT_lo.as<__bf16>(), S->natoms_pad, cm, out, K, list, n, K,
                         S->gemm16_expand, S->stream, nullptr, nullptr, S->live);
    }));
  }
  return 0;
}

// bytes of split-K partials for up to nmax columns (FP64 and FP32 partials)
size_t cpart_capacity(const stern_system* S, int M_pad, int nmax, int K) {
  size_t best = 0;
  for (int n = 1; n <= nmax; ++n) {
    const size_t c = std::max((size_t)choose_nsplit(M_pad, n, K, S->gemm64_wg) * sizeof(Z64),
                              (size_t)choose_nsplit_bf16(M_pad, n, K, S->gemm16_wg) * sizeof(Z32)) * n;
    if (c > best) best = c;
  }
  return best * M_pad;
}

// workspace for `ns` rows held at once
int ensure_workspace(stern_system* S, int ns) {
  const size_t K = S->hb.npw_pad;
  const size_t vec = (size_t)ns * K * sizeof(Z64);
  for (DBuf* d : {&S->wx, &S->wr, &S->wp, &S->wq, &S->wz, &S->wb}) CHECKED(d->ensure(vec));
  CHECKED(S->pen.ensure((size_t)ns * S->hb.N * S->hb.ncol_pad * sizeof(Z64)));
  const int mp = std::max(S->nocc_pad, S->natoms_pad);
  CHECKED(S->cpart.ensure(std::max(cpart_capacity(S, std::max(S->nocc_pad, 64), ns, (int)K),
                                   cpart_capacity(S, S->natoms_pad, ns, (int)K))));
  CHECKED(S->cmat.ensure((size_t)ns * mp * sizeof(Z64)));
  CHECKED(S->cpart2.ensure(cpart_capacity(S, std::max(S->nocc_pad, 64), ns, (int)K)));
  for (DBuf* d : {&S->sv_eps, &S->sv_invT, &S->sv_bb, &S->sv_rz, &S->sv_rr, &S->sv_tres, &S->sv_rzi})
    CHECKED(d->ensure((size_t)ns * sizeof(double)));
  for (DBuf* d : {&S->sv_band, &S->sv_pert, &S->sv_flag, &S->sv_iters, &S->list_act, &S->list_f})
    CHECKED(d->ensure((size_t)ns * sizeof(int)));
  // padding entries of every vector stay zero: clear once when (re)allocated
  if (S->ws_solves < ns) {
    for (DBuf* d : {&S->wx, &S->wr, &S->wp, &S->wq, &S->wz, &S->wb})
      launch_fill_zero(d->as<Z64>(), (size_t)ns * K, S->stream);
    S->ws_solves = ns;
  }
  return 0;
}

int ensure_workspace32(stern_system* S, int ns) {
  const size_t K = S->hb.npw_pad;
  for (DBuf* d : {&S->m_d, &S->m_r, &S->m_p, &S->m_q, &S->m_z}) CHECKED(d->ensure((size_t)ns * K * sizeof(Z32)));
  for (DBuf* d : {&S->m_rz, &S->m_rr0, &S->m_beta}) CHECKED(d->ensure((size_t)ns * sizeof(double)));
  CHECKED(S->m_flag.ensure((size_t)ns * sizeof(int)));
  CHECKED(S->m_cnt.ensure(sizeof(int)));
  if (S->ws32_solves < ns) {
    for (DBuf* d : {&S->m_d, &S->m_r, &S->m_p, &S->m_q, &S->m_z})
      launch_fill_zero32(d->as<Z32>(), (size_t)ns * K, S->stream);
    S->ws32_solves = ns;
  }
  return 0;
}

Cg32State cg32_state(stern_system* S, int* iters) {
  Cg32State c;
  c.d = S->m_d.as<Z32>();
  c.r = S->m_r.as<Z32>();
  c.p = S->m_p.as<Z32>();
  c.q = S->m_q.as<Z32>();
  c.z = S->m_z.as<Z32>();
  c.rz = S->m_rz.as<double>();
  c.rr0 = S->m_rr0.as<double>();
  c.beta = S->m_beta.as<double>();
  c.flag = S->m_flag.as<int>();
  c.iters = iters;
  c.invT = S->sv_invT.as<double>();
  c.g2h = S->g2h.as<double>();
  c.kprec = nullptr;
  c.npw_pad = S->hb.npw_pad;
  return c;
}

CgState cg_state(stern_system* S) {
  CgState c;
  c.x = S->wx.as<Z64>();
  c.r = S->wr.as<Z64>();
  c.p = S->wp.as<Z64>();
  c.q = S->wq.as<Z64>();
  c.z = S->wz.as<Z64>();
  c.b = S->wb.as<Z64>();
  c.bb = S->sv_bb.as<double>();
  c.rz = S->sv_rz.as<double>();
  c.rr = S->sv_rr.as<double>();
  c.flag = S->sv_flag.as<int>();
  c.iters = S->sv_iters.as<int>();
  c.tres = S->sv_tres.as<double>();
  c.eps = S->sv_eps.as<double>();
  c.invT = S->sv_invT.as<double>();
  c.g2h = S->g2h.as<double>();
  c.kprec = nullptr;
  c.npw_pad = S->hb.npw_pad;
  return c;
}

// q = A x for rows in list with the FP64 projected operator, then the true-residual test
int true_residual(stern_system* S, const CgState& cs, const int* list, int n, double tol) {
  launch_copy_rows(cs.x, cs.z, S->hb.npw_pad, list, n, S->stream);
  CHECKED(apply_pc_rows(S, cs.z, list, n));
  CHECKED(apply_h_rows(S, cs.z, cs.q, list, n, cs.eps));
  CHECKED(apply_pc_rows(S, cs.q, list, n));
  launch_true_resid(cs, list, n, tol, S->stream);
  return 0;
}

int launch_check() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(STERN_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return 0;
}

// Makes `dev` the current device and `al` the current allocator of the calling
// thread for the lifetime of the object.
struct Scope {
  int dev_prev = -1;
  const Alloc* al_prev = nullptr;
  explicit Scope(int dev, const Alloc* al = nullptr) : al_prev(tl_alloc) {
    (void)hipGetDevice(&dev_prev);
    (void)hipSetDevice(dev);
    tl_alloc = al;
  }
  ~Scope() {
    if (dev_prev >= 0) (void)hipSetDevice(dev_prev);
    tl_alloc = al_prev;
  }
};


// ---- learned initial guess ----

size_t net_bytes_per_solve(const stern_system* S) {
  const int Nc = S->hbc.N;
  const size_t ldp = (size_t)net_ldp(Nc);
  return (size_t)Nc * S->hbc.ncol_pad * sizeof(Z64) + (size_t)Nc * Nc * Nc * sizeof(Z64) +
         3 * ldp * kNetChannels * sizeof(__bf16) + ldp * kNetChannels * sizeof(float);
}

// coarse-grid fields of rows [s0, s0 + c) of `rows` (sphere vectors): c_field = inverse yz of pencils
int coarse_fields(stern_system* S, const Z64* rows, int s0, int c) {
  const FftGeom gc = S->geom_c();
  launch_xinv(gc, rows + (size_t)s0 * S->hb.npw_pad, nullptr, c, S->c_pen.as<Z64>(), S->stream);
  launch_plane_full_inv(gc, S->c_pen.as<Z64>(), c, S->c_field.as<Z64>(), S->stream);
  return 0;
}

// net input of rows [s0, s0 + c) into a0 (needs b and ||b||^2 of the rows)
int net_input(stern_system* S, const CgState& cs, int s0, int c, __bf16* a0) {
  CHECKED(coarse_fields(S, cs.b, s0, c));
  launch_pack_input(S->psi_c.as<Z64>(), S->c_field.as<Z64>(), S->sv_band.as<int>() + s0, cs.eps + s0, cs.bb + s0, a0,
                    S->hbc.N, c, S->stream);
  return 0;
}

// the two hidden layers only (their output feeds the preconditioner features)
void net_trunk(const stern_model* M, const __bf16* a0, __bf16* a1, __bf16* a2, int Nc, int c, hipStream_t st) {
  launch_conv3(a0, M->wb(0), M->bias(0), a1, Nc, c, 1, false, st);
  launch_conv3(a1, M->wb(1), M->bias(1), a2, Nc, c, 1, false, st);
}

void net_forward(const stern_model* M, const __bf16* a0, __bf16* a1, __bf16* a2, float* out, int Nc, int c,
                 hipStream_t st) {
  launch_conv3(a0, M->wb(0), M->bias(0), a1, Nc, c, 1, false, st);
  launch_conv3(a1, M->wb(1), M->bias(1), a2, Nc, c, 1, false, st);
  launch_conv3(a2, M->wb(2), M->bias(2), out, Nc, c, 0, true, st);
}

// x = P_c (net output mapped to the sphere) for all ns rows; then r = b - A x in FP64,
// dropping guesses whose residual is non-finite or not below ||b||.
// Learned start of the ns solves of the batch. The preconditioner features
// come from the net's hidden layers evaluated per band on (psi_v, 0, eps_v)
// (n_occ evaluations, shared by all fields); with_x0 also predicts x0 per solve
// (x = P_c (net output mapped to the sphere)) and forms r = b - A x in FP64 or,
// for a defect-correction start, FP32, dropping guesses whose residual is
// non-finite or not below ||b||. Without x0 the batch keeps x = 0, r = b.
int learned_guess(stern_system* S, const stern_model* M, CgState& cs, int ns, int& n_rej, bool fp32_resid,
                  bool with_x0, bool want_feat = false) {
  hipStream_t st = S->stream;
  const FftGeom gc = S->geom_c();
  const int Nc = gc.N, K = S->hb.npw_pad;
  const size_t ldp = (size_t)net_ldp(Nc), nc3 = (size_t)Nc * Nc * Nc;
  const int chunk = std::min(std::max(with_x0 ? ns : 0, S->n_occ), 1024);
  CHECKED(S->c_pen.ensure((size_t)chunk * Nc * gc.ncol_pad * sizeof(Z64)));
  CHECKED(S->c_field.ensure((size_t)chunk * nc3 * sizeof(Z64)));
  for (DBuf* d : {&S->net_a0, &S->net_a1, &S->net_a2})
    CHECKED(d->ensure((size_t)chunk * ldp * kNetChannels * sizeof(__bf16)));
  CHECKED(S->net_out.ensure((size_t)chunk * ldp * kNetChannels * sizeof(float)));
  CHECKED(S->g_rej.ensure((size_t)S->ws_solves * sizeof(int)));
  CHECKED(S->net_feat.ensure((size_t)S->ws_solves * kPrecIn * sizeof(float)));
  CHECKED(S->band_feat.ensure((size_t)S->n_occ * kPrecIn * sizeof(float)));
  const double flops2 = 2.0 * 2.0 * kNetChannels * 27 * kNetChannels * (double)nc3;
  if (M->prec_trained || want_feat) {  // per-band features, then per solve by its band
    for (int b0 = 0; b0 < S->n_occ; b0 += chunk) {
      const int c = std::min(chunk, S->n_occ - b0);
      CHECKED(timed(S, STERN_K_NET, c * (double)(nc3 * 16 + ldp * 16 * 10), c * flops2, [&] {
        launch_pack_band(S->psi_c.as<Z64>() + (size_t)b0 * nc3, S->band_eps.as<double>() + b0,
                         S->net_a0.as<__bf16>(), Nc, c, st);
        net_trunk(M, S->net_a0.as<__bf16>(), S->net_a1.as<__bf16>(), S->net_a2.as<__bf16>(), Nc, c, st);
        launch_pool(S->net_a2.as<__bf16>(), S->band_eps.as<double>() + b0, S->band_invT.as<double>() + b0,
                    S->band_feat.as<float>() + (size_t)b0 * kPrecIn, Nc, c, st);
      }));
    }
    launch_gather_f32(S->net_feat.as<float>(), S->band_feat.as<float>(), S->sv_band.as<int>(), kPrecIn, ns, st);
  }
  const double flops = 3.0 * 2.0 * kNetChannels * 27 * kNetChannels * (double)nc3;
  for (int s0 = 0; with_x0 && s0 < ns; s0 += chunk) {
    const int c = std::min(chunk, ns - s0);
    CHECKED(timed(S, STERN_K_NET, c * (double)(nc3 * 16 * 4 + ldp * 16 * 14), c * flops, [&] {
      (void)net_input(S, cs, s0, c, S->net_a0.as<__bf16>());
      net_forward(M, S->net_a0.as<__bf16>(), S->net_a1.as<__bf16>(), S->net_a2.as<__bf16>(),
                  S->net_out.as<float>(), Nc, c, st);
      launch_unpack_output(S->net_out.as<float>(), cs.bb + s0, S->c_field.as<Z64>(), Nc, c, st);
      launch_plane_full_fwd(gc, S->c_field.as<Z64>(), c, S->c_pen.as<Z64>(), st);
      launch_xfwd<double>(gc, S->c_pen.as<Z64>(), nullptr, c, cs.x + (size_t)s0 * K, 2, nullptr, nullptr,
                          1.0 / (double)nc3, st);
    }));
  }
  // learned diagonal preconditioner of every solve
  cs.kprec = nullptr;
  if (M->prec_trained) {
    CHECKED(S->net_coef.ensure((size_t)S->ws_solves * kPrecKnots * sizeof(float)));
    CHECKED(S->kprec.ensure((size_t)S->ws_solves * K * sizeof(float)));
    CHECKED(timed(S, STERN_K_NET, ns * (double)K * 12.0, 0.0, [&] {
      launch_prec_coef(M->head(), S->net_feat.as<float>(), S->net_coef.as<float>(), ns, st);
      launch_prec_build(S->net_coef.as<float>(), S->net_feat.as<float>(), cs.g2h, S->kprec.as<float>(), K, ns, st);
    }));
    cs.kprec = S->kprec.as<float>();
  }
  if (!with_x0) return launch_check();
  CHECKED(apply_pc_rows(S, cs.x, nullptr, ns));
  if (fp32_resid) {  // residual of the guess with the FP32 operator (it seeds a defect-correction step)
    Z32* x32 = S->m_p.as<Z32>();
    Z32* q32 = S->m_q.as<Z32>();
    launch_to32(cs.x, x32, (size_t)ns * K, st);
    CHECKED(apply_h32_rows(S, x32, q32, nullptr, ns, cs.eps));
    CHECKED(apply_pc32_rows(S, q32, nullptr, ns));
    launch_guess_resid(cs, nullptr, ns, q32, S->g_rej.as<int>(), st);
  } else {
    CHECKED(apply_h_rows(S, cs.x, cs.q, nullptr, ns, cs.eps));
    CHECKED(apply_pc_rows(S, cs.q, nullptr, ns));
    launch_guess_resid(cs, nullptr, ns, nullptr, S->g_rej.as<int>(), st);
  }
  CHECKED(launch_check());
  std::vector<int> rej(ns);
  HIPOK(hipMemcpyAsync(rej.data(), S->g_rej.p, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  for (int v : rej) n_rej += v;
  return 0;
}

// Warm start of the solves [0, ns) of a batch from the kept solutions at row `row0`:
// x = P_c x_kept, r = b - (P_c (H - eps) P_c - i u) x in FP64 (u = 0: the static system);
// starts already within tol are marked converged, those with ||r|| >= ||b|| replaced by zero.
int warm_start(stern_system* S, const CgState& cs, size_t row0, int ns, double u, double tol, int& n_rej) {
  hipStream_t st = S->stream;
  const int K = S->hb.npw_pad;
  CHECKED(S->g_rej.ensure((size_t)S->ws_solves * sizeof(int)));
  HIPOK(hipMemcpyAsync(cs.x, S->xkeep.as<Z64>() + row0 * K, (size_t)ns * K * sizeof(Z64), hipMemcpyDeviceToDevice,
                       st));
  CHECKED(apply_pc_rows(S, cs.x, nullptr, ns));
  CHECKED(apply_h_rows(S, cs.x, cs.q, nullptr, ns, cs.eps));
  CHECKED(apply_pc_rows(S, cs.q, nullptr, ns));
  launch_guess_resid(cs, nullptr, ns, nullptr, S->g_rej.as<int>(), st, u, tol * tol);
  CHECKED(launch_check());
  std::vector<int> rej(ns);
  HIPOK(hipMemcpyAsync(rej.data(), S->g_rej.p, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  for (int v : rej) n_rej += v;
  return 0;
}

// Per-solve arrays, right-hand sides b = -P_c [dV psi_v] and x = 0, r = b for the
// solves of perturbations [i0, i1) x bands [v0, v0 + nb) (row s = (i - i0) nb + v - v0).
// A right-hand side P_c dV psi_v whose norm is at most this fraction of ||dV psi_v|| is
// zero: dV psi_v lies in the occupied span (dV constant, for one), and what the FP64
// projection leaves is rounding, about n_occ * 1e-16 of the product at most. Left in,
// part of it lies along the occupied states, which the projected operator cannot reduce.
constexpr double kRhsCut = 1e-12;

int setup_batch(stern_system* S, int i0, int i1, int v0, int nb, const double* dv_dev, double vecb) {
  hipStream_t st = S->stream;
  const HostBasis& hb = S->hb;
  const int N = hb.N;
  const size_t n3 = (size_t)N * N * N;
  const int ns = (i1 - i0) * nb;
  std::vector<int> h_band(ns), h_pert(ns);
  std::vector<double> h_eps(ns), h_invT(ns);
  for (int s = 0; s < ns; ++s) {
    h_band[s] = v0 + s % nb;
    h_pert[s] = i0 + s / nb;
    h_eps[s] = S->eps[h_band[s]];
    h_invT[s] = S->invT[h_band[s]];
  }
  HIPOK(hipMemcpyAsync(S->sv_band.p, h_band.data(), ns * sizeof(int), hipMemcpyHostToDevice, st));
  HIPOK(hipMemcpyAsync(S->sv_pert.p, h_pert.data(), ns * sizeof(int), hipMemcpyHostToDevice, st));
  HIPOK(hipMemcpyAsync(S->sv_eps.p, h_eps.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
  HIPOK(hipMemcpyAsync(S->sv_invT.p, h_invT.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
  const CgState cs = cg_state(S);
  const FftGeom g = S->geom();
  // psi_v(r) once per band, dV_i(r) and the pencils once per solve
  CHECKED(timed(S, STERN_K_RHS, nb * (double)n3 * 16.0 + ns * ((double)n3 * 8.0 + (double)N * hb.ncol * 16.0), 0.0, [&] {
    launch_plane_rhs(g, S->psi_r.as<Z64>(), dv_dev, v0, nb, i0, i1 - i0, S->sv_band.as<int>(),
                     S->sv_pert.as<int>(), S->pen.as<Z64>(), st);
  }));
  CHECKED(timed(S, STERN_K_XFWD, ns * ((double)N * hb.ncol * 16.0 + vecb), 0.0, [&] {
    launch_xfwd<double>(g, S->pen.as<Z64>(), nullptr, ns, cs.b, 2, nullptr, nullptr, -1.0 / (double)n3, st);
  }));
  launch_row_norm2(cs.b, cs.npw_pad, ns, cs.bb, st);  // ||dV psi_v|| before the projection
  CHECKED(apply_pc_rows(S, cs.b, nullptr, ns));
  launch_outer_init(cs, nullptr, ns, kRhsCut, st);  // x = 0, r = b, ||b||, counters
  HIPOK(hipStreamSynchronize(st));         // the host arrays above are released on return
  return 0;
}

// Runs `body` (one CG iteration's launches on the system stream) `steps` times:
// eagerly, or captured once into a hipGraph and replayed.
template <class F>
int run_steps(stern_system* S, int steps, bool graph, F&& body) {
  if (steps <= 0) return 0;
  if (!graph || S->prof_on) {
    for (int k = 0; k < steps; ++k) CHECKED(body());
    return 0;
  }
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  HIPOK(hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal));
  const int rc = body();
  hipError_t e = hipStreamEndCapture(S->stream, &g);
  if (rc < 0) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(STERN_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(STERN_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  for (int k = 0; k < steps && e == hipSuccess; ++k) e = hipGraphLaunch(ex, S->stream);
  (void)hipGraphExecDestroy(ex);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(STERN_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
  return 0;
}

// Plain FP64 projected PCG from zero on the solves in `list` (batch row indices).
int run_pcg64(stern_system* S, const CgState& cs, const std::vector<int>& list, double tol, int max_iter,
              int check_every, int& n_restart, double vecb, bool use_graph, bool keep_x = false) {
  hipStream_t st = S->stream;
  const int ns_all = S->ws_solves;
  std::vector<int> h_flag(ns_all), act, flist;
  if (list.empty()) return 0;
  const int n0 = (int)list.size();
  HIPOK(hipMemcpyAsync(S->list_act.p, list.data(), n0 * sizeof(int), hipMemcpyHostToDevice, st));
  {
    const int* L = S->list_act.as<int>();
    CHECKED(timed(S, STERN_K_CG, vecb * n0 * 4.0, 0.0, [&] { launch_cg_init(cs, L, n0, keep_x, st); }));
    CHECKED(apply_pc_rows(S, cs.z, L, n0));
    CHECKED(timed(S, STERN_K_CG, vecb * n0 * 3.0, 0.0, [&] { launch_cg_init2(cs, L, n0, st); }));
  }
  CHECKED(launch_check());
  HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  for (int s : list)
    if (h_flag[s] == 0) act.push_back(s);
  int it = 0;
  while (!act.empty()) {
    const int na = (int)act.size();
    HIPOK(hipMemcpyAsync(S->list_act.p, act.data(), na * sizeof(int), hipMemcpyHostToDevice, st));
    const int* L = S->list_act.as<int>();
    const int nsteps = std::min(check_every, max_iter - it);
    CHECKED(run_steps(S, nsteps, use_graph && it > 0, [&]() -> int {
      CHECKED(apply_h_rows(S, cs.p, cs.q, L, na, cs.eps));
      CHECKED(apply_pc_rows(S, cs.q, L, na));
      CHECKED(timed(S, STERN_K_CG, vecb * na * 7.0, 0.0, [&] { launch_cg_alpha(cs, L, na, tol * tol, st); }));
      CHECKED(apply_pc_rows(S, cs.z, L, na));
      CHECKED(timed(S, STERN_K_CG, vecb * na * 4.0, 0.0, [&] { launch_cg_beta(cs, L, na, st); }));
      return 0;
    }));
    it += nsteps;
    CHECKED(launch_check());
    HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    const bool last = it >= max_iter;
    flist.clear();
    for (int s : act)
      if (h_flag[s] == 1 || last) flist.push_back(s);
    if (!flist.empty()) {
      const int nf = (int)flist.size();
      HIPOK(hipMemcpyAsync(S->list_f.p, flist.data(), nf * sizeof(int), hipMemcpyHostToDevice, st));
      const int* F = S->list_f.as<int>();
      if (last) launch_set_flag(cs.flag, F, nf, 1, st);  // final check on everything still running
      CHECKED(true_residual(S, cs, F, nf, tol));
      if (!last) {
        CHECKED(apply_pc_rows(S, cs.z, F, nf));
        launch_cg_restart(cs, F, nf, st);
      }
      CHECKED(launch_check());
      HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPOK(hipStreamSynchronize(st));
      if (!last)
        for (int s : flist)
          if (h_flag[s] == 0) ++n_restart;
    }
    if (last) break;
    std::vector<int> nxt;
    for (int s : act)
      if (h_flag[s] != 2) nxt.push_back(s);
    act.swap(nxt);
  }
  return 0;
}

// Response at imaginary frequency i u: (P_c (H - eps_v) P_c - i u) x = b by preconditioned
// conjugate orthogonal CG in FP64 (the shifted operator is symmetric in (a, b)_J =
// sum_G a(-G) b(G); see the kernels). Same structure as run_pcg64: per-solve flags, the active
// list compacted every check_every iterations, the FP64 true residual of the shifted system at
// recurrence convergence, restart from it when it fails.
int run_cocg64(stern_system* S, const CgState& cs, const std::vector<int>& list, double u, double tol, int max_iter,
               int check_every, int& n_restart, double vecb, bool keep_x = false) {
  hipStream_t st = S->stream;
  const int ns_all = S->ws_solves;
  const int* negk = S->negk.as<int>();
  double* rzi = S->sv_rzi.as<double>();
  std::vector<int> h_flag(ns_all), act, flist;
  if (list.empty()) return 0;
  const int n0 = (int)list.size();
  HIPOK(hipMemcpyAsync(S->list_act.p, list.data(), n0 * sizeof(int), hipMemcpyHostToDevice, st));
  {
    const int* L = S->list_act.as<int>();
    CHECKED(timed(S, STERN_K_CG, vecb * n0 * 4.0, 0.0, [&] { launch_cg_init(cs, L, n0, keep_x, st); }));
    CHECKED(apply_pc_rows(S, cs.z, L, n0));
    CHECKED(timed(S, STERN_K_CG, vecb * n0 * 3.0, 0.0, [&] { launch_cocg_start(cs, negk, rzi, L, n0, 0, st); }));
  }
  CHECKED(launch_check());
  HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  for (int s : list)
    if (h_flag[s] == 0) act.push_back(s);
  int it = 0;
  while (!act.empty()) {
    const int na = (int)act.size();
    HIPOK(hipMemcpyAsync(S->list_act.p, act.data(), na * sizeof(int), hipMemcpyHostToDevice, st));
    const int* L = S->list_act.as<int>();
    const int nsteps = std::min(check_every, max_iter - it);
    for (int k = 0; k < nsteps; ++k) {
      CHECKED(apply_h_rows(S, cs.p, cs.q, L, na, cs.eps));
      CHECKED(apply_pc_rows(S, cs.q, L, na));
      CHECKED(timed(S, STERN_K_CG, vecb * na * 8.0, 0.0,
                    [&] { launch_cocg_alpha(cs, negk, rzi, u, L, na, tol * tol, st); }));
      CHECKED(apply_pc_rows(S, cs.z, L, na));
      CHECKED(timed(S, STERN_K_CG, vecb * na * 4.0, 0.0, [&] { launch_cocg_beta(cs, negk, rzi, L, na, st); }));
    }
    it += nsteps;
    CHECKED(launch_check());
    HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    const bool last = it >= max_iter;
    flist.clear();
    for (int s : act)
      if (h_flag[s] == 1 || last) flist.push_back(s);
    if (!flist.empty()) {
      const int nf = (int)flist.size();
      HIPOK(hipMemcpyAsync(S->list_f.p, flist.data(), nf * sizeof(int), hipMemcpyHostToDevice, st));
      const int* F = S->list_f.as<int>();
      if (last) launch_set_flag(cs.flag, F, nf, 1, st);  // final check on everything still running
      launch_copy_rows(cs.x, cs.z, S->hb.npw_pad, F, nf, st);
      CHECKED(apply_pc_rows(S, cs.z, F, nf));
      CHECKED(apply_h_rows(S, cs.z, cs.q, F, nf, cs.eps));
      CHECKED(apply_pc_rows(S, cs.q, F, nf));
      launch_cocg_true(cs, u, F, nf, tol, st);
      if (!last) {
        CHECKED(apply_pc_rows(S, cs.z, F, nf));
        launch_cocg_start(cs, negk, rzi, F, nf, 3, st);
      }
      CHECKED(launch_check());
      HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPOK(hipStreamSynchronize(st));
      if (!last)
        for (int s : flist)
          if (h_flag[s] == 0) ++n_restart;
    }
    if (last) break;
    std::vector<int> nxt;
    for (int s : act)
      if (h_flag[s] != 2) nxt.push_back(s);
    act.swap(nxt);
  }
  return 0;
}

// Mixed precision: FP64 defect correction around FP32/BF16 inner PCG solves.
//   repeat: solve A d = r to inner_tol with FP32 FFTs and split-BF16 MFMA GEMMs
//           (FP64 dots and scalars); x += d; r = b - A x (FP64)
//   until ||r|| <= tol ||b||; then x = P_c x (FP64); solves still above tol after
//   max_outer steps are re-solved by FP64 PCG from zero.
// Inner operators (inner_op):
//  projected: q = P_c (H - eps) p and z = P_c K r. The alpha step takes the new
//    (r, z) before z is projected, which equals (r, P_c z) as r stays in
//    range(P_c); so beta is known before the projection, and the projection
//    of z and p = P_c z + beta p run as one GEMM pair.
//  shifted: H - eps + alpha P_v (Baroni et al., Rev. Mod. Phys. 73, 515 (2001)),
//    positive definite for alpha above the occupied band width, and z = K r.
//    On range(P_c) it agrees with the projected operator up to the commutator
//    of H with P_v; with Teter's K, which does not commute with P_v, it takes
//    more than twice the inner iterations.
// The FP64 outer residual uses the projected operator, so the accepted
// solution is the projected system's whichever operator runs inside.
int run_mixed(stern_system* S, const CgState& cs, const std::vector<int>& list, double tol, double inner_tol,
              int max_outer, int max_iter, int check_every, int& n_restart, int& n_fallback, double vecb,
              bool use_graph, int inner_op) {
  const bool projected = inner_op == STERN_INNER_PROJECTED;
  hipStream_t st = S->stream;
  const int ns_all = S->ws_solves;
  const int K = S->hb.npw_pad;
  const double vec32 = vecb / 2;
  Cg32State c32 = cg32_state(S, cs.iters);
  c32.kprec = cs.kprec;
  const int ns32 = S->ws32_solves;  // rows of the FP32 workspace (the FP64 one may hold more)
  std::vector<int> h_flag(ns_all), h_iflag(ns32), act, iact;
  HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  for (int s : list)
    if (h_flag[s] == 0) act.push_back(s);
  const int max_inner = std::max(1, max_iter);
  for (int outer = 0; outer < max_outer && !act.empty(); ++outer) {
    const int na = (int)act.size();
    HIPOK(hipMemcpyAsync(S->list_act.p, act.data(), na * sizeof(int), hipMemcpyHostToDevice, st));
    const int* L = S->list_act.as<int>();
    CHECKED(timed(S, STERN_K_CG32, na * (vecb + 3.0 * vec32), 0.0, [&] { launch_cg32_init(c32, cs.r, L, na, st); }));
    if (projected) CHECKED(apply_pc32_rows(S, c32.z, L, na));
    CHECKED(timed(S, STERN_K_CG32, na * 3.0 * vec32, 0.0, [&] { launch_cg32_init2(c32, L, na, st); }));
    CHECKED(launch_check());
    HIPOK(hipMemcpyAsync(h_iflag.data(), c32.flag, ns32 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    iact.clear();
    for (int s : act)
      if (h_iflag[s] == 0) iact.push_back(s);
    // The active list (list_f) and its count (m_cnt) live on the device: every inner
    // iteration ends with an in-place stable compaction, and its launches, sized for
    // the count at the last poll, cover only the first *m_cnt entries. A window of
    // check_every iterations (eager, or captured once into a hipGraph and replayed)
    // needs one read of the count at its end and no other host round trip.
    int ni = (int)iact.size();
    int* F = S->list_f.as<int>();
    int* cnt = S->m_cnt.as<int>();
    if (ni > 0) {
      HIPOK(hipMemcpyAsync(F, iact.data(), ni * sizeof(int), hipMemcpyHostToDevice, st));
      launch_set_int(cnt, ni, st);
    }
    int cap = ni;  // the grids' bound: the count at the last poll
    int it = 0;
    while (ni > 0 && it < max_inner) {
      const int nsteps = S->prof_on ? 1 : std::min(check_every, max_inner - it);
      S->live = cnt;
      const int rc = run_steps(S, nsteps, use_graph && (it > 0 || outer > 0), [&]() -> int {
        if (projected) {
          CHECKED(apply_hproj32_rows(S, c32.p, c32.q, F, cap, cs.eps));
        } else {
          CHECKED(apply_h32_rows(S, c32.p, c32.q, F, cap, cs.eps));
          CHECKED(apply_psi32_rows(S, c32.p, c32.q, F, cap, (float)S->alpha_pv));
        }
        CHECKED(timed(S, STERN_K_CG32, vec32 * cap * 7.0, 0.0,
                      [&] { launch_cg32_alpha(c32, F, cap, inner_tol * inner_tol, st, cnt); }));
        if (projected)  // p = P_c z + beta p
          CHECKED(apply_pc32_update(S, c32.z, c32.p, c32.beta, F, cap));
        else
          CHECKED(timed(S, STERN_K_CG32, vec32 * cap * 3.0, 0.0, [&] { launch_cg32_beta(c32, F, cap, st, cnt); }));
        CHECKED(timed(S, STERN_K_OTHER, 8.0 * cap, 0.0, [&] { launch_compact(F, cnt, c32.flag, st); }));
        return 0;
      });
      S->live = nullptr;
      CHECKED(rc);
      it += nsteps;
      CHECKED(launch_check());
      HIPOK(hipMemcpyAsync(&ni, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPOK(hipStreamSynchronize(st));
      cap = std::min(cap, ni);
    }
    // FP64 update and true residual. x keeps the occupied components the inner solves leave (at
    // the level of their split-BF16 projections); on them P_c (H - eps) acts as P_c Psi (E - eps)
    // = 0 up to the ground state's eigen-residual, so the residual needs no projection of x, which
    // is projected once after the last step.
    CHECKED(timed(S, STERN_K_CG, na * (2.0 * vecb + vec32), 0.0, [&] { launch_add_d(cs.x, c32.d, K, L, na, st); }));
    CHECKED(apply_h_rows(S, cs.x, cs.q, L, na, cs.eps));
    CHECKED(apply_pc_rows(S, cs.q, L, na));
    CHECKED(timed(S, STERN_K_CG, na * 3.0 * vecb, 0.0, [&] { launch_outer_resid(cs, L, na, tol, st); }));
    CHECKED(launch_check());
    HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    std::vector<int> nxt;
    for (int s : act)
      if (h_flag[s] != 2) nxt.push_back(s);
    act.swap(nxt);
  }
  {  // the solutions in range(P_c) (those falling back below restart from zero)
    const int n = (int)list.size();
    HIPOK(hipMemcpyAsync(S->list_act.p, list.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    CHECKED(apply_pc_rows(S, cs.x, S->list_act.as<int>(), n));
    HIPOK(hipStreamSynchronize(st));  // list_act is rewritten by the fallback
  }
  if (!act.empty()) {  // Teter-preconditioned FP64 PCG from zero
    n_fallback += (int)act.size();
    CgState teter = cs;
    teter.kprec = nullptr;
    CHECKED(run_pcg64(S, teter, act, tol, max_iter, check_every, n_restart, vecb, use_graph));
  }
  return 0;
}

}  // namespace

// ============================================================== C ABI ======

namespace {

// mean time (ms) of `reps` calls of fn on the system stream, after one warm-up call
template <class F>
int time_ms(stern_system* S, int reps, double& ms, F&& fn) {
  hipEvent_t e0, e1;
  HIPOK(hipEventCreate(&e0));
  HIPOK(hipEventCreate(&e1));
  int rc = fn();
  if (rc >= 0) rc = launch_check();
  (void)hipEventRecord(e0, S->stream);
  for (int r = 0; r < reps && rc >= 0; ++r) rc = fn();
  (void)hipEventRecord(e1, S->stream);
  const hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  if (rc >= 0 && e == hipSuccess) (void)hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc < 0) return rc;
  if (e != hipSuccess) return fail(STERN_ERR_HIP, "autotune timing: %s", hipGetErrorString(e));
  ms = t / reps;
  return 0;
}

}  // namespace

extern "C" {

const char* stern_last_error(void) { return g_err.c_str(); }

static int cell_from_abi(const stern_cell* c, CellParams& p) {
  if (!c) return fail(STERN_ERR_INVALID_ARG, "cell is NULL");
  if (c->n_atoms < 0 || (c->n_atoms > 0 && !c->pos)) return fail(STERN_ERR_INVALID_ARG, "bad atoms");
  if (!(c->L > 0) || !(c->ecut_ry > 0)) return fail(STERN_ERR_INVALID_ARG, "L and ecut_ry must be > 0");
  if (c->fft_n < 0) return fail(STERN_ERR_INVALID_ARG, "fft_n must be >= 0");
  p.L = c->L;
  p.ecut = c->ecut_ry;
  p.pos.assign(c->pos, c->pos + 3 * (size_t)c->n_atoms);
  p.amp = c->vloc_amp;
  p.sigma = c->vloc_sigma;
  p.D = c->kb_D;
  p.width = c->kb_width;
  p.fft_n = c->fft_n;
  if (!(p.sigma > 0) || !(p.width > 0)) return fail(STERN_ERR_INVALID_ARG, "vloc_sigma and kb_width must be > 0");
  return 0;
}

int stern_basis_info(const stern_cell* cell, int* n_pw, int* fft_n, int32_t* miller) {
  CellParams p;
  CHECKED(cell_from_abi(cell, p));
  HostBasis hb;
  std::string e = build_basis(p, hb);
  if (!e.empty()) return fail(STERN_ERR_INVALID_ARG, "%s", e.c_str());
  if (n_pw) *n_pw = hb.npw;
  if (fft_n) *fft_n = hb.N;
  if (miller) std::memcpy(miller, hb.miller.data(), hb.miller.size() * sizeof(int32_t));
  return STERN_OK;
}

int stern_init_system(const stern_cell* cell, const stern_runtime* rt, stern_system** out) {
  if (!out) return fail(STERN_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  CellParams p;
  CHECKED(cell_from_abi(cell, p));
  if (rt && (rt->dev_alloc == nullptr) != (rt->dev_free == nullptr))
    return fail(STERN_ERR_INVALID_ARG, "dev_alloc and dev_free must be given together");
  stern_system* S = new stern_system();
  S->device = rt ? rt->device : 0;
  S->stream = rt ? (hipStream_t)rt->stream : nullptr;
  if (rt && rt->dev_alloc) {
    S->alloc.alloc = rt->dev_alloc;
    S->alloc.free = rt->dev_free;
    S->alloc.ctx = rt->alloc_ctx;
  }
  S->cell = p;
  std::string e = build_basis(p, S->hb);
  if (!e.empty()) {
    delete S;
    return fail(STERN_ERR_INVALID_ARG, "%s", e.c_str());
  }
  const HostBasis& hb = S->hb;
  if (!fft_size_supported(hb.N)) {
    delete S;
    return fail(STERN_ERR_UNSUPPORTED, "FFT grid %d is not a supported 2^a 3^b size", hb.N);
  }
  Scope sc(S->device, &S->alloc);
  {
    void* scr = nullptr;
    const int rc = scratch_address(S->device, &scr);
    if (rc < 0) {
      delete S;
      return rc;
    }
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, S->device) != hipSuccess) {
    delete S;
    return fail(STERN_ERR_HIP, "hipGetDeviceProperties failed");
  }
  {  // yz-plane kernels: the compact H apply when its LDS fits, else the full plane
    const size_t lds_max = std::max((size_t)prop.sharedMemPerBlock, (size_t)prop.maxSharedMemoryPerMultiProcessor);
    const bool c64 = plane_hw_lds(hb.N, hb.nza, true) <= lds_max, c32 = plane_hw_lds(hb.N, hb.nza, false) <= lds_max;
    const bool f64 = plane_lds_bytes(hb.N, sizeof(Z64)) <= lds_max, f32 = plane_lds_bytes(hb.N, sizeof(Z32)) <= lds_max;
    const size_t rhs = plane_fp64_lds(hb.N, hb.nza);
    if (!(c64 || f64) || !(c32 || f32) || rhs > lds_max) {
      delete S;
      return fail(STERN_ERR_UNSUPPORTED, "the yz-plane kernels of grid %d do not fit in %zu bytes of LDS", hb.N,
                  lds_max);
    }
    S->plane_var64 = c64 ? 1 : 0;
    S->plane_var32 = c32 ? 1 : 0;
    S->lds_max = lds_max;
  }
  S->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  S->n_atoms = (int)(p.pos.size() / 3);
  S->natoms_pad = std::max(64, (S->n_atoms + 63) / 64 * 64);
  auto run = [&]() -> int {
    hipStream_t st = S->stream;
    CHECKED(upload(S->col_start, hb.col_start.data(), hb.col_start.size() * sizeof(int), st));
    CHECKED(upload(S->col_len, hb.col_len.data(), hb.col_len.size() * sizeof(int), st));
    CHECKED(upload(S->col_xmin, hb.col_xmin.data(), hb.col_xmin.size() * sizeof(int), st));
    CHECKED(upload(S->col_pos, hb.col_pos.data(), hb.col_pos.size() * sizeof(int), st));
    CHECKED(upload(S->zl, hb.zl.data(), hb.zl.size() * sizeof(int), st));
    CHECKED(upload(S->ycol, hb.ycol.data(), hb.ycol.size() * sizeof(int), st));
    CHECKED(upload(S->g2h, hb.g2h.data(), hb.g2h.size() * sizeof(double), st));
    {  // -G of every coefficient in column order (the sphere is symmetric under G -> -G)
      std::map<std::array<int32_t, 3>, int> canon;
      for (int c = 0; c < hb.npw; ++c)
        canon[{hb.miller[3 * c], hb.miller[3 * c + 1], hb.miller[3 * c + 2]}] = c;
      std::vector<int> nk(hb.npw_pad);
      for (int k = hb.npw; k < hb.npw_pad; ++k) nk[k] = k;
      for (int c = 0; c < hb.npw; ++c) {
        const auto it = canon.find({-hb.miller[3 * c], -hb.miller[3 * c + 1], -hb.miller[3 * c + 2]});
        if (it == canon.end()) return fail(STERN_ERR_UNSUPPORTED, "the sphere is not symmetric under G -> -G");
        nk[hb.perm[c]] = hb.perm[it->second];
      }
      CHECKED(upload(S->negk, nk.data(), nk.size() * sizeof(int), st));
      HIPOK(hipStreamSynchronize(st));  // nk is released at the end of this block
    }
    CHECKED(upload(S->perm, hb.perm.data(), hb.perm.size() * sizeof(int), st));
    std::vector<Z64> tw(hb.N);
    for (int m = 0; m < hb.N; ++m) {
      const double a = 6.283185307179586476925286766559 * m / hb.N;
      tw[m] = zmk(std::cos(a), -std::sin(a));
    }
    CHECKED(upload(S->tw64, tw.data(), tw.size() * sizeof(Z64), st));
    std::vector<Z32> tw32(hb.N);
    for (int m = 0; m < hb.N; ++m) tw32[m] = zmk((float)tw[m].re, (float)tw[m].im);
    CHECKED(upload(S->tw32, tw32.data(), tw32.size() * sizeof(Z32), st));
    const double n3 = (double)hb.N * hb.N * hb.N;
    std::vector<double> v = vloc_grid(p, hb, 1.0 / n3);
    CHECKED(upload(S->v_r, v.data(), v.size() * sizeof(double), st));
    std::vector<float> v32(v.begin(), v.end());
    CHECKED(upload(S->v_r32, v32.data(), v32.size() * sizeof(float), st));
    {  // [x][z][y] copies for the compact plane kernel
      const size_t Nn = hb.N;
      std::vector<double> vt(v.size());
      std::vector<float> vt32(v.size());
      for (size_t x = 0; x < Nn; ++x)
        for (size_t y = 0; y < Nn; ++y)
          for (size_t z = 0; z < Nn; ++z) {
            vt[(x * Nn + z) * Nn + y] = v[(x * Nn + y) * Nn + z];
            vt32[(x * Nn + z) * Nn + y] = (float)v[(x * Nn + y) * Nn + z];
          }
      CHECKED(upload(S->v_t, vt.data(), vt.size() * sizeof(double), st));
      CHECKED(upload(S->v_t32, vt32.data(), vt32.size() * sizeof(float), st));
      HIPOK(hipStreamSynchronize(st));  // vt, vt32 are released at the end of this block
    }
    std::vector<std::complex<double>> B = kb_projectors(p, hb, S->natoms_pad);
    CHECKED(upload(S->kb, B.data(), B.size() * sizeof(Z64), st));
    const size_t kbn = (size_t)S->natoms_pad * hb.npw_pad * 2 * sizeof(__bf16);
    for (DBuf* d : {&S->kb_hi, &S->kb_lo, &S->kbT_hi, &S->kbT_lo}) CHECKED(d->ensure(kbn));
    launch_split_bf16(S->kb.as<Z64>(), S->natoms_pad, hb.npw_pad, S->kb_hi.as<__bf16>(), S->kb_lo.as<__bf16>(),
                      S->kbT_hi.as<__bf16>(), S->kbT_lo.as<__bf16>(), st);
    // coarse grid of the learned guess
    if (hb.N % 2 == 0 && fft_size_supported(hb.N / 2)) {
      CellParams pc = p;
      pc.fft_n = hb.N / 2;
      if (build_basis(pc, S->hbc, true).empty() && S->hbc.npw == hb.npw) {
        const HostBasis& c = S->hbc;
        CHECKED(upload(S->c_col_start, c.col_start.data(), c.col_start.size() * sizeof(int), st));
        CHECKED(upload(S->c_col_len, c.col_len.data(), c.col_len.size() * sizeof(int), st));
        CHECKED(upload(S->c_col_xmin, c.col_xmin.data(), c.col_xmin.size() * sizeof(int), st));
        CHECKED(upload(S->c_col_pos, c.col_pos.data(), c.col_pos.size() * sizeof(int), st));
        CHECKED(upload(S->c_zl, c.zl.data(), c.zl.size() * sizeof(int), st));
        CHECKED(upload(S->c_ycol, c.ycol.data(), c.ycol.size() * sizeof(int), st));
        std::vector<Z64> twc(c.N);
        for (int m = 0; m < c.N; ++m) {
          const double a = 6.283185307179586476925286766559 * m / c.N;
          twc[m] = zmk(std::cos(a), -std::sin(a));
        }
        CHECKED(upload(S->c_tw64, twc.data(), twc.size() * sizeof(Z64), st));
        S->have_coarse = true;
      }
    }
    HIPOK(hipStreamSynchronize(st));
    return 0;
  };
  int rc = run();
  if (rc < 0) {
    S->release_all();
    delete S;
    return rc;
  }
  *out = S;
  return STERN_OK;
}

int stern_query(const stern_system* S, int* n_pw, int* fft_n, double* omega) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (n_pw) *n_pw = S->hb.npw;
  if (fft_n) *fft_n = S->hb.N;
  if (omega) *omega = S->hb.omega;
  return STERN_OK;
}

int stern_get_miller(const stern_system* S, int32_t* miller) {
  if (!S || !miller) return fail(STERN_ERR_INVALID_ARG, "system and miller must not be NULL");
  std::memcpy(miller, S->hb.miller.data(), S->hb.miller.size() * sizeof(int32_t));
  return STERN_OK;
}

int stern_set_occupied(stern_system* S, int n_occ, const double* psi, const double* eps, int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (n_occ <= 0 || !psi || !eps) return fail(STERN_ERR_INVALID_ARG, "need n_occ > 0, psi and eps");
  if (mem_kind != STERN_MEM_HOST && mem_kind != STERN_MEM_DEVICE) return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  Scope sc(S->device, &S->alloc);
  S->keep_np = 0;  // kept solutions belong to the previous occupied states
  const HostBasis& hb = S->hb;
  hipStream_t st = S->stream;
  const int npw = hb.npw, K = hb.npw_pad, N = hb.N;
  std::vector<double> h_psi, h_eps(n_occ);
  const double* hp = psi;
  if (mem_kind == STERN_MEM_DEVICE) {
    h_psi.resize((size_t)n_occ * npw * 2);
    HIPOK(hipMemcpy(h_psi.data(), psi, h_psi.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPOK(hipMemcpy(h_eps.data(), eps, n_occ * sizeof(double), hipMemcpyDeviceToHost));
    hp = h_psi.data();
  } else {
    std::memcpy(h_eps.data(), eps, n_occ * sizeof(double));
  }
  // kinetic energy per band, T_v = sum_G |G|^2/2 |c|^2, floored at (2 pi / L)^2 / 2
  S->eps = h_eps;
  {  // alpha of the shifted inner operator: twice the occupied band width, at least 0.01 Ha
    const auto mm = std::minmax_element(h_eps.begin(), h_eps.end());
    S->alpha_pv = std::max(0.01, 2.0 * (*mm.second - *mm.first));
  }
  S->invT.assign(n_occ, 0.0);
  const double floor_t = 0.5 * hb.b * hb.b;
  for (int v = 0; v < n_occ; ++v) {
    double t = 0.0;
    for (int k = 0; k < npw; ++k) {
      const double re = hp[2 * ((size_t)v * npw + k)], im = hp[2 * ((size_t)v * npw + k) + 1];
      t += hb.g2h[hb.perm[k]] * (re * re + im * im);
    }
    S->invT[v] = 1.0 / std::max(t, floor_t);
  }
  S->n_occ = n_occ;
  S->nocc_pad = std::max(64, (n_occ + 63) / 64 * 64);
  CHECKED(upload(S->band_eps, S->eps.data(), n_occ * sizeof(double), st));
  CHECKED(upload(S->band_invT, S->invT.data(), n_occ * sizeof(double), st));
  CHECKED(S->psi.ensure((size_t)S->nocc_pad * K * sizeof(Z64)));
  launch_fill_zero(S->psi.as<Z64>(), (size_t)S->nocc_pad * K, st);
  // tmp_in also holds P_c KB below
  CHECKED(S->tmp_in.ensure(std::max((size_t)n_occ * npw, (size_t)S->natoms_pad * K) * sizeof(Z64)));
  HIPOK(hipMemcpyAsync(S->tmp_in.p, hp, (size_t)n_occ * npw * sizeof(Z64), hipMemcpyHostToDevice, st));
  launch_permute(S->tmp_in.as<Z64>(), npw, S->psi.as<Z64>(), K, S->perm.as<int>(), npw, n_occ, true, st);
  const size_t psn = (size_t)S->nocc_pad * K * 2 * sizeof(__bf16);
  for (DBuf* d : {&S->psi_hi, &S->psi_lo, &S->psiT_hi, &S->psiT_lo}) CHECKED(d->ensure(psn));
  launch_split_bf16(S->psi.as<Z64>(), S->nocc_pad, K, S->psi_hi.as<__bf16>(), S->psi_lo.as<__bf16>(),
                    S->psiT_hi.as<__bf16>(), S->psiT_lo.as<__bf16>(), st);
  S->proj_m = 0;
  if (S->n_atoms > 0) {  // stacked rows [P_c KB; Psi], P_c beta_a = beta_a - sum_b psi_b <psi_b|beta_a> in FP64
    const int Ma = S->natoms_pad, Mb = S->nocc_pad, Mt = Ma + Mb;
    const size_t tn = (size_t)Mt * K * 2 * sizeof(__bf16);
    for (DBuf* d : {&S->projT_hi, &S->projT_lo}) CHECKED(d->ensure(tn));
    __bf16 *th = S->projT_hi.as<__bf16>(), *tl = S->projT_lo.as<__bf16>();
    Z64* pkb = S->tmp_in.as<Z64>();
    HIPOK(hipMemcpyAsync(pkb, S->kb.p, (size_t)Ma * K * sizeof(Z64), hipMemcpyDeviceToDevice, st));
    const int ns = choose_nsplit(Mb, Ma, K, S->gemm64_wg);
    CHECKED(S->cpart.ensure((size_t)ns * Ma * Mb * sizeof(Z64)));
    CHECKED(S->cmat.ensure((size_t)Ma * Mb * sizeof(Z64)));
    launch_zgemm_reduce(S->psi.as<Z64>(), Mb, S->kb.as<Z64>(), K, nullptr, Ma, K, S->cpart.as<Z64>(), ns, st);
    launch_sum_parts(S->cpart.as<Z64>(), ns, Ma, Mb, -1.0, S->cmat.as<Z64>(), st);
    launch_zgemm_expand(S->psi.as<Z64>(), Mb, S->cmat.as<Z64>(), pkb, K, nullptr, Ma, K, st);
    launch_split_bf16_rows(pkb, Ma, K, 0, Mt, nullptr, nullptr, th, tl, st);
    launch_split_bf16_rows(S->psi.as<Z64>(), Mb, K, Ma, Mt, nullptr, nullptr, th, tl, st);
    CHECKED(launch_check());
    S->proj_m = Mt;
  }
  // psi_v(r) on the grid (unnormalised sum_G c_G e^{iG.r}) for the RHS and dn
  CHECKED(S->psi_r.ensure((size_t)n_occ * N * N * N * sizeof(Z64)));
  CHECKED(S->pen.ensure((size_t)n_occ * N * hb.ncol_pad * sizeof(Z64)));
  const FftGeom g = S->geom();
  launch_xinv(g, S->psi.as<Z64>(), nullptr, n_occ, S->pen.as<Z64>(), st);
  launch_plane_full_inv(g, S->pen.as<Z64>(), n_occ, S->psi_r.as<Z64>(), st);
  if (S->have_coarse) {  // psi_v(r) on the coarse grid, input of the learned guess
    const FftGeom gc = S->geom_c();
    const size_t nc3 = (size_t)gc.N * gc.N * gc.N;
    CHECKED(S->psi_c.ensure((size_t)n_occ * nc3 * sizeof(Z64)));
    launch_xinv(gc, S->psi.as<Z64>(), nullptr, n_occ, S->pen.as<Z64>(), st);
    launch_plane_full_inv(gc, S->pen.as<Z64>(), n_occ, S->psi_c.as<Z64>(), st);
  }
  CHECKED(launch_check());
  HIPOK(hipStreamSynchronize(st));
  S->have_occ = true;
  return STERN_OK;
}

static int rows_in(stern_system* S, int n_vec, const double* c, int mem_kind, DBuf& dst) {
  const int npw = S->hb.npw, K = S->hb.npw_pad;
  CHECKED(dst.ensure((size_t)n_vec * K * sizeof(Z64)));
  launch_fill_zero(dst.as<Z64>(), (size_t)n_vec * K, S->stream);
  CHECKED(S->tmp_out.ensure((size_t)n_vec * npw * sizeof(Z64)));
  HIPOK(hipMemcpyAsync(S->tmp_out.p, c, (size_t)n_vec * npw * sizeof(Z64),
                       mem_kind == STERN_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, S->stream));
  launch_permute(S->tmp_out.as<Z64>(), npw, dst.as<Z64>(), K, S->perm.as<int>(), npw, n_vec, true, S->stream);
  return 0;
}

static int rows_out(stern_system* S, int n_vec, const Z64* src, const int* rows_host, double* out, int mem_kind) {
  const int npw = S->hb.npw, K = S->hb.npw_pad;
  CHECKED(S->tmp_out.ensure((size_t)n_vec * npw * sizeof(Z64)));
  for (int v = 0; v < n_vec; ++v) {
    const int row = rows_host ? rows_host[v] : v;
    launch_permute(src + (size_t)row * K, K, S->tmp_out.as<Z64>() + (size_t)v * npw, npw, S->perm.as<int>(), npw, 1,
                   false, S->stream);
  }
  HIPOK(hipMemcpyAsync(out, S->tmp_out.p, (size_t)n_vec * npw * sizeof(Z64),
                       mem_kind == STERN_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, S->stream));
  HIPOK(hipStreamSynchronize(S->stream));
  return 0;
}

int stern_apply_h(stern_system* S, int n_vec, const double* c, const double* shift, double* out, int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (n_vec <= 0) return STERN_OK;
  if (!c || !out) return fail(STERN_ERR_INVALID_ARG, "NULL array");
  Scope sc(S->device, &S->alloc);
  CHECKED(ensure_workspace(S, std::max(n_vec, S->ws_solves)));
  CHECKED(rows_in(S, n_vec, c, mem_kind, S->wp));
  std::vector<double> sh(n_vec, 0.0);
  if (shift) {
    if (mem_kind == STERN_MEM_DEVICE)
      HIPOK(hipMemcpy(sh.data(), shift, n_vec * sizeof(double), hipMemcpyDeviceToHost));
    else
      std::memcpy(sh.data(), shift, n_vec * sizeof(double));
  }
  HIPOK(hipMemcpyAsync(S->sv_eps.p, sh.data(), n_vec * sizeof(double), hipMemcpyHostToDevice, S->stream));
  CHECKED(apply_h_rows(S, S->wp.as<Z64>(), S->wq.as<Z64>(), nullptr, n_vec, S->sv_eps.as<double>()));
  CHECKED(launch_check());
  return rows_out(S, n_vec, S->wq.as<Z64>(), nullptr, out, mem_kind);
}

// ---- TDDFT Liouville superoperator (Tamm-Dancoff, Hartree kernel) ----------

// the 4 Ecut sphere on the system's grid: transition densities and the Hartree potential
static int ensure_density_geom(stern_system* S) {
  if (S->have_dens) return 0;
  const HostBasis& hb = S->hb;
  if (plane_lds_bytes(hb.N, sizeof(Z64)) > S->lds_max)
    return fail(STERN_ERR_UNSUPPORTED, "grid %d: the Liouville apply needs full FP64 planes in LDS (N <= 96)", hb.N);
  CellParams pd;
  pd.L = hb.L;
  pd.ecut = 4.0 * hb.ecut;
  pd.fft_n = hb.N;
  const std::string e = build_basis(pd, S->hbd, true);
  if (!e.empty()) return fail(STERN_ERR_UNSUPPORTED, "density sphere: %s", e.c_str());
  const HostBasis& d = S->hbd;
  hipStream_t st = S->stream;
  CHECKED(upload(S->d_col_start, d.col_start.data(), d.col_start.size() * sizeof(int), st));
  CHECKED(upload(S->d_col_len, d.col_len.data(), d.col_len.size() * sizeof(int), st));
  CHECKED(upload(S->d_col_xmin, d.col_xmin.data(), d.col_xmin.size() * sizeof(int), st));
  CHECKED(upload(S->d_col_pos, d.col_pos.data(), d.col_pos.size() * sizeof(int), st));
  CHECKED(upload(S->d_zl, d.zl.data(), d.zl.size() * sizeof(int), st));
  CHECKED(upload(S->d_ycol, d.ycol.data(), d.ycol.size() * sizeof(int), st));
  CHECKED(upload(S->d_g2h, d.g2h.data(), d.g2h.size() * sizeof(double), st));
  HIPOK(hipStreamSynchronize(st));
  S->have_dens = true;
  return 0;
}

// excitations per chunk of the grid stage: ce nb full grids of a_r and their pencils in flight
static int liouville_chunk(const stern_system* S, int n_exc) {
  const size_t n3 = (size_t)S->hb.N * S->hb.N * S->hb.N, nb = S->n_occ;
  const size_t per = nb * (n3 + (size_t)S->hb.N * S->hb.ncol_pad + S->hb.npw_pad) * sizeof(Z64);
  const size_t budget = (size_t)2 << 30;
  int ce = (int)std::max<size_t>(1, budget / per);
  ce = std::min(ce, std::max(1, 65535 / (int)nb));  // rows of one grid launch
  return std::min(ce, n_exc);
}

// n full grids (in place) -> fac / (|q|^2 / 2) times their components on the 4 Ecut sphere,
// zero at q = 0, back on the grid: the Hartree potential for fac = 2 pi
static void potential_grids(stern_system* S, Z64* buf, int n, double fac) {
  const FftGeom gd = S->geom_d();
  const size_t n3 = (size_t)gd.N * gd.N * gd.N;
  hipStream_t st = S->stream;
  launch_plane_full_fwd(gd, buf, n, S->lv_pend.as<Z64>(), st);
  launch_xfwd<double>(gd, S->lv_pend.as<Z64>(), nullptr, n, S->lv_rhog.as<Z64>(), 2, nullptr, nullptr, 1.0 / (double)n3,
                      st);
  launch_coulomb(S->lv_rhog.as<Z64>(), gd.g2h, gd.npw_pad, n, fac, st);
  launch_xinv(gd, S->lv_rhog.as<Z64>(), nullptr, n, S->lv_pend.as<Z64>(), st);
  launch_plane_full_inv(gd, S->lv_pend.as<Z64>(), n, buf, st);
}

// out = L A for n_exc excitations of n_occ band rows each (column order, stride npw_pad; A in
// range(P_c)): out_v = P_c [ (H - eps_v) a_v + 2 V[rho_A] psi_v - alpha sum_w tau_{wv} a_w ],
// rho_A = sum_v conj(psi_v) a_v, tau_{wv} = V[conj(psi_w) psi_v] (eq. tau_u),
// V[rho] = sum_{0 < |q|^2 <= 4 Ecut} 4 pi / |q|^2 rho(q) e^{i q.r}.
static int liouville_rows(stern_system* S, const Z64* A, Z64* out, int n_exc) {
  const HostBasis& hb = S->hb;
  const int nb = S->n_occ, K = hb.npw_pad, N = hb.N, n = n_exc * nb;
  const size_t n3 = (size_t)N * N * N;
  hipStream_t st = S->stream;
  const FftGeom g = S->geom();
  const int Kd = S->hbd.npw_pad;
  const int ce = liouville_chunk(S, n_exc);
  const bool exch = S->lv_alpha != 0.0 || S->n_scr > 0;
  const int np = std::max(ce, exch ? nb : 0);  // grids through the potential stage at once
  CHECKED(S->lv_ar.ensure((size_t)ce * nb * n3 * sizeof(Z64)));
  CHECKED(S->lv_rho.ensure((size_t)ce * n3 * sizeof(Z64)));
  CHECKED(S->lv_rhog.ensure((size_t)np * Kd * sizeof(Z64)));
  CHECKED(S->lv_pend.ensure((size_t)np * N * S->hbd.ncol_pad * sizeof(Z64)));
  if (exch) {
    CHECKED(S->lv_tau.ensure((size_t)nb * n3 * sizeof(Z64)));
    CHECKED(S->lv_acc.ensure((size_t)ce * nb * n3 * sizeof(Z64)));
    if (S->n_scr > 0) CHECKED(S->scr_proj.ensure((size_t)nb * S->n_scr * sizeof(Z64)));
  }
  CHECKED(S->lv_k.ensure((size_t)n * K * sizeof(Z64)));
  CHECKED(S->lv_eps.ensure((size_t)n * sizeof(double)));
  {
    std::vector<double> e(n);
    for (int r = 0; r < n; ++r) e[r] = S->eps[r % nb];
    HIPOK(hipMemcpyAsync(S->lv_eps.p, e.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    HIPOK(hipStreamSynchronize(st));
  }
  // D A
  CHECKED(apply_h_rows(S, A, out, nullptr, n, S->lv_eps.as<double>()));
  // K1e A, ce excitations at a time
  Z64* ar = S->lv_ar.as<Z64>();
  Z64* rho = S->lv_rho.as<Z64>();
  Z64* kt = S->lv_k.as<Z64>();
  launch_fill_zero(kt, (size_t)n * K, st);  // the padding entries are added to out below
  for (int e0 = 0; e0 < n_exc; e0 += ce) {
    const int c = std::min(ce, n_exc - e0), m = c * nb;
    const Z64* Ae = A + (size_t)e0 * nb * K;
    for (int r0 = 0; r0 < m; r0 += S->ws_solves) {  // pencils hold ws_solves rows
      const int rm = std::min(S->ws_solves, m - r0);
      launch_xinv(g, Ae + (size_t)r0 * K, nullptr, rm, S->pen.as<Z64>(), st);
      launch_plane_full_inv(g, S->pen.as<Z64>(), rm, ar + (size_t)r0 * n3, st);
    }
    constexpr double kPi = 3.14159265358979323846;
    if (exch)  // sum_w tau_{wv} a_w of every band v, the pair potentials one band v at a time
      for (int v = 0; v < nb; ++v) {
        Z64* tau = S->lv_tau.as<Z64>();
        launch_pair_density(S->psi_r.as<Z64>(), v, nb, n3, 1.0 / hb.omega, tau, st);
        if (S->n_scr > 0)
          launch_scr_proj(tau, S->scr_w.as<double>(), S->n_scr, nb, n3, S->scr_proj.as<Z64>(), st);
        potential_grids(S, tau, nb, 2.0 * kPi * S->lv_alpha);  // alpha V[rho]
        if (S->n_scr > 0)
          launch_scr_add(tau, S->scr_w.as<double>(), S->scr_proj.as<Z64>(), S->scr_c.as<double>(), S->n_scr, nb, n3,
                         st);
        launch_exch_acc(tau, ar, c, nb, v, n3, S->lv_acc.as<Z64>(), st);
      }
    launch_band_density(S->psi_r.as<Z64>(), ar, c, nb, n3, 1.0 / hb.omega, rho, st);
    // 2 x 4 pi / |q|^2 = 4 pi / (|q|^2 / 2): the factor 2 of the singlet exchange term folded in
    potential_grids(S, rho, c, 4.0 * kPi);
    launch_grid_mul(rho, S->psi_r.as<Z64>(), c, nb, n3, exch ? S->lv_acc.as<Z64>() : nullptr, 1.0, ar, st);
    for (int r0 = 0; r0 < m; r0 += S->ws_solves) {
      const int rm = std::min(S->ws_solves, m - r0);
      launch_plane_full_fwd(g, ar + (size_t)r0 * n3, rm, S->pen.as<Z64>(), st);
      launch_xfwd<double>(g, S->pen.as<Z64>(), nullptr, rm, kt + ((size_t)e0 * nb + r0) * K, 2, nullptr, nullptr,
                          1.0 / (double)n3, st);
    }
  }
  launch_add(out, kt, (size_t)n * K, st);
  CHECKED(apply_pc_rows(S, out, nullptr, n));
  return launch_check();
}

static int liouville_setup(stern_system* S, int n_exc) {
  if (!S->have_occ) return fail(STERN_ERR_STATE, "set_occupied has not been called");
  if (n_exc <= 0) return fail(STERN_ERR_INVALID_ARG, "n_exc must be > 0");
  CHECKED(ensure_density_geom(S));
  const int nb = S->n_occ;
  // pencils for whole excitations' rows at a time (the chunk), and the six block vectors of the solve
  CHECKED(ensure_workspace(S, std::max(S->ws_solves, std::max(n_exc * nb, liouville_chunk(S, n_exc) * nb))));
  return 0;
}

int stern_liouville_set_kernel(stern_system* S, double alpha_x) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!(alpha_x >= 0.0 && alpha_x <= 1.0)) return fail(STERN_ERR_INVALID_ARG, "alpha_x must lie in [0, 1]");
  S->lv_alpha = alpha_x;
  return STERN_OK;
}

int stern_liouville_set_screening(stern_system* S, int n, const double* w, const double* c, int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (n < 0 || (n > 0 && (!w || !c))) return fail(STERN_ERR_INVALID_ARG, "need n >= 0, w and c");
  if (mem_kind != STERN_MEM_HOST && mem_kind != STERN_MEM_DEVICE) return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  Scope sc(S->device, &S->alloc);
  S->n_scr = 0;
  if (n == 0) return STERN_OK;
  const size_t n3 = (size_t)S->hb.N * S->hb.N * S->hb.N;
  std::vector<double> hc(n);
  if (mem_kind == STERN_MEM_DEVICE)
    HIPOK(hipMemcpy(hc.data(), c, n * sizeof(double), hipMemcpyDeviceToHost));
  else
    std::memcpy(hc.data(), c, n * sizeof(double));
  for (double x : hc)
    if (!std::isfinite(x)) return fail(STERN_ERR_INVALID_ARG, "screening weights must be finite");
  CHECKED(S->scr_w.ensure((size_t)n * n3 * sizeof(double)));
  CHECKED(S->scr_c.ensure((size_t)n * sizeof(double)));
  HIPOK(hipMemcpyAsync(S->scr_w.p, w, (size_t)n * n3 * sizeof(double),
                       mem_kind == STERN_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, S->stream));
  HIPOK(hipMemcpyAsync(S->scr_c.p, hc.data(), n * sizeof(double), hipMemcpyHostToDevice, S->stream));
  HIPOK(hipStreamSynchronize(S->stream));
  S->n_scr = n;
  return STERN_OK;
}

int stern_liouville_apply(stern_system* S, int n_exc, const double* a, double* out, int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!a || !out) return fail(STERN_ERR_INVALID_ARG, "NULL array");
  if (mem_kind != STERN_MEM_HOST && mem_kind != STERN_MEM_DEVICE) return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  Scope sc(S->device, &S->alloc);
  CHECKED(liouville_setup(S, n_exc));
  const int n = n_exc * S->n_occ;
  CHECKED(rows_in(S, n, a, mem_kind, S->wp));
  CHECKED(apply_pc_rows(S, S->wp.as<Z64>(), nullptr, n));
  CHECKED(liouville_rows(S, S->wp.as<Z64>(), S->wq.as<Z64>(), n_exc));
  return rows_out(S, n, S->wq.as<Z64>(), nullptr, out, mem_kind);
}

// per-excitation sums of the per-row dots conj(a) . b (bands in order)
static int block_dots(stern_system* S, const Z64* a, const Z64* b, int n_exc, std::vector<Z64>& out) {
  const int nb = S->n_occ, n = n_exc * nb;
  launch_row_dot(a, b, S->hb.npw_pad, n, S->lv_dot.as<Z64>(), S->stream);
  std::vector<Z64> h(n);
  HIPOK(hipMemcpyAsync(h.data(), S->lv_dot.p, n * sizeof(Z64), hipMemcpyDeviceToHost, S->stream));
  HIPOK(hipStreamSynchronize(S->stream));
  out.assign(n_exc, zmk(0.0, 0.0));
  for (int e = 0; e < n_exc; ++e)
    for (int v = 0; v < nb; ++v) out[e] = out[e] + h[(size_t)e * nb + v];
  return 0;
}

static int upload_coef(stern_system* S, const std::vector<Z64>& c) {
  HIPOK(hipMemcpyAsync(S->lv_coef.p, c.data(), c.size() * sizeof(Z64), hipMemcpyHostToDevice, S->stream));
  HIPOK(hipStreamSynchronize(S->stream));  // c may be released or changed on return
  return 0;
}

// z = P_c K r per band row (Teter's K with the band's T_v)
static int precond_rows(stern_system* S, const Z64* r, Z64* z, int n) {
  launch_teter_rows(r, z, S->g2h.as<double>(), S->band_invT.as<double>(), S->n_occ, S->hb.npw_pad, n, S->stream);
  return apply_pc_rows(S, z, nullptr, n);
}

// L z = b by preconditioned CG, one block (all band rows) per excitation: L is Hermitian and,
// with the gap open, positive definite on range(P_c)^n_occ; the block inner product sums the
// band rows. Converged when the recurrence residual meets tol, then judged by the true one.
int stern_liouville_solve(stern_system* S, int n_exc, const double* b, double* z, double tol, int max_iter,
                          int mem_kind, int* iters, double* resid) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!b || !z) return fail(STERN_ERR_INVALID_ARG, "NULL array");
  if (!(tol > 0)) return fail(STERN_ERR_INVALID_ARG, "tol must be > 0");
  if (mem_kind != STERN_MEM_HOST && mem_kind != STERN_MEM_DEVICE) return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  Scope sc(S->device, &S->alloc);
  CHECKED(liouville_setup(S, n_exc));
  const int nb = S->n_occ, n = n_exc * nb, K = S->hb.npw_pad;
  const int mi = max_iter > 0 ? max_iter : 1000;
  hipStream_t st = S->stream;
  CHECKED(S->lv_dot.ensure((size_t)n * sizeof(Z64)));
  CHECKED(S->lv_coef.ensure((size_t)n_exc * sizeof(Z64)));
  Z64 *X = S->wx.as<Z64>(), *R = S->wr.as<Z64>(), *P = S->wp.as<Z64>(), *Q = S->wq.as<Z64>(), *Zv = S->wz.as<Z64>(),
      *B = S->wb.as<Z64>();
  CHECKED(rows_in(S, n, b, mem_kind, S->wb));
  CHECKED(apply_pc_rows(S, B, nullptr, n));
  launch_fill_zero(X, (size_t)n * K, st);
  HIPOK(hipMemcpyAsync(R, B, (size_t)n * K * sizeof(Z64), hipMemcpyDeviceToDevice, st));
  CHECKED(precond_rows(S, R, Zv, n));
  HIPOK(hipMemcpyAsync(P, Zv, (size_t)n * K * sizeof(Z64), hipMemcpyDeviceToDevice, st));
  std::vector<Z64> d;
  CHECKED(block_dots(S, B, B, n_exc, d));
  std::vector<double> bb(n_exc), rz(n_exc);
  for (int e = 0; e < n_exc; ++e) bb[e] = d[e].re;
  CHECKED(block_dots(S, R, Zv, n_exc, d));
  for (int e = 0; e < n_exc; ++e) rz[e] = d[e].re;
  std::vector<int> it(n_exc, 0);
  std::vector<char> done(n_exc, 0);
  for (int e = 0; e < n_exc; ++e) done[e] = !(bb[e] > 0.0);  // b = 0: z = 0
  std::vector<Z64> c(n_exc);
  for (int k = 0; k < mi; ++k) {
    bool any = false;
    for (int e = 0; e < n_exc; ++e) any |= !done[e];
    if (!any) break;
    CHECKED(liouville_rows(S, P, Q, n_exc));
    CHECKED(block_dots(S, P, Q, n_exc, d));
    for (int e = 0; e < n_exc; ++e) c[e] = zmk(done[e] || !(d[e].re > 0.0) ? 0.0 : rz[e] / d[e].re, 0.0);
    CHECKED(upload_coef(S, c));
    launch_blk_axpy(X, P, S->lv_coef.as<Z64>(), nb, K, n, st);
    for (int e = 0; e < n_exc; ++e) c[e].re = -c[e].re;
    CHECKED(upload_coef(S, c));
    launch_blk_axpy(R, Q, S->lv_coef.as<Z64>(), nb, K, n, st);
    CHECKED(block_dots(S, R, R, n_exc, d));
    for (int e = 0; e < n_exc; ++e)
      if (!done[e]) {
        ++it[e];
        if (d[e].re <= tol * tol * bb[e]) done[e] = 1;
      }
    CHECKED(precond_rows(S, R, Zv, n));
    CHECKED(block_dots(S, R, Zv, n_exc, d));
    for (int e = 0; e < n_exc; ++e) {
      c[e] = zmk(done[e] || !(rz[e] > 0.0) ? 0.0 : d[e].re / rz[e], 0.0);
      rz[e] = d[e].re;
    }
    CHECKED(upload_coef(S, c));
    launch_blk_xpby(P, Zv, S->lv_coef.as<Z64>(), nb, K, n, st);
  }
  // true residual b - L x
  CHECKED(liouville_rows(S, X, Q, n_exc));
  HIPOK(hipMemcpyAsync(R, B, (size_t)n * K * sizeof(Z64), hipMemcpyDeviceToDevice, st));
  for (int e = 0; e < n_exc; ++e) c[e] = zmk(-1.0, 0.0);
  CHECKED(upload_coef(S, c));
  launch_blk_axpy(R, Q, S->lv_coef.as<Z64>(), nb, K, n, st);
  CHECKED(block_dots(S, R, R, n_exc, d));
  bool all_ok = true;
  for (int e = 0; e < n_exc; ++e) {
    const double res = bb[e] > 0.0 ? std::sqrt(std::max(0.0, d[e].re) / bb[e]) : 0.0;
    all_ok &= res <= tol;
    if (resid) resid[e] = res;
    if (iters) iters[e] = it[e];
  }
  CHECKED(rows_out(S, n, X, nullptr, z, mem_kind));
  return all_ok ? STERN_OK : STERN_WARN_NOT_CONVERGED;
}


// C[n][i] = <V_i | X_n> for the cap basis rows of V and nx rows of X, rows of length Lt (FP64 MFMA
// reduce), on the host
static int dav_vh_x(stern_system* S, const Z64* V, int cap, const Z64* X, int nx, int Lt, std::vector<Z64>& C) {
  hipStream_t st = S->stream;
  const int ns = choose_nsplit(cap, nx, Lt, S->gemm64_wg);
  CHECKED(S->dv_part.ensure((size_t)ns * nx * cap * sizeof(Z64)));
  CHECKED(S->dv_cm.ensure((size_t)nx * cap * sizeof(Z64)));
  launch_zgemm_reduce(V, cap, X, Lt, nullptr, nx, Lt, S->dv_part.as<Z64>(), ns, st);
  launch_sum_parts(S->dv_part.as<Z64>(), ns, nx, cap, 1.0, S->dv_cm.as<Z64>(), st);
  C.resize((size_t)nx * cap);
  HIPOK(hipMemcpyAsync(C.data(), S->dv_cm.p, C.size() * sizeof(Z64), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  return launch_check();
}

// Y[n] += sum_i V_i C[n][i] (FP64 MFMA expand) for ny rows of length Lt
static int dav_v_c(stern_system* S, const Z64* V, int cap, const std::vector<Z64>& C, Z64* Y, int ny, int Lt) {
  hipStream_t st = S->stream;
  CHECKED(S->dv_cm.ensure((size_t)ny * cap * sizeof(Z64)));
  HIPOK(hipMemcpyAsync(S->dv_cm.p, C.data(), (size_t)ny * cap * sizeof(Z64), hipMemcpyHostToDevice, st));
  launch_zgemm_expand(V, cap, S->dv_cm.as<Z64>(), Y, Lt, nullptr, ny, Lt, st);
  HIPOK(hipStreamSynchronize(st));  // C may change on return
  return launch_check();
}

// T (nt vectors) orthogonalised against the m basis vectors of V (two classical Gram-Schmidt
// passes through the GEMMs) and among themselves (modified Gram-Schmidt), normalised; vectors
// that lose all but 1e-8 of their norm are dropped. Returns the number kept (packed first).
static int dav_orth(stern_system* S, const Z64* V, int cap, int m, Z64* T, int nt, int Lt, int& kept) {
  hipStream_t st = S->stream;
  const int nb = S->n_occ;
  std::vector<Z64> d, C;
  CHECKED(block_dots(S, T, T, nt, d));
  std::vector<double> n0(nt);
  for (int j = 0; j < nt; ++j) n0[j] = std::sqrt(std::max(0.0, d[j].re));
  for (int pass = 0; pass < 2 && m > 0; ++pass) {
    CHECKED(dav_vh_x(S, V, cap, T, nt, Lt, C));
    for (auto& c : C) c = zmk(-c.re, -c.im);
    CHECKED(dav_v_c(S, V, cap, C, T, nt, Lt));
  }
  kept = 0;
  std::vector<Z64> c1(1);
  for (int j = 0; j < nt; ++j) {
    Z64* tj = T + (size_t)j * Lt;
    for (int i = 0; i < kept; ++i) {
      const Z64* ti = T + (size_t)i * Lt;
      CHECKED(block_dots(S, ti, tj, 1, d));
      c1[0] = zmk(-d[0].re, -d[0].im);
      CHECKED(upload_coef(S, c1));
      launch_blk_axpy(tj, ti, S->lv_coef.as<Z64>(), nb, S->hb.npw_pad, nb, st);
    }
    CHECKED(block_dots(S, tj, tj, 1, d));
    const double nn = std::sqrt(std::max(0.0, d[0].re));
    if (!(nn > 1e-8 * n0[j])) continue;
    // unit norm, into slot `kept`
    Z64* tk = T + (size_t)kept * Lt;
    if (tk != tj) HIPOK(hipMemcpyAsync(tk, tj, (size_t)Lt * sizeof(Z64), hipMemcpyDeviceToDevice, st));
    c1[0] = zmk(1.0 / nn, 0.0);
    CHECKED(upload_coef(S, c1));
    launch_blk_scale(tk, S->lv_coef.as<Z64>(), nb, S->hb.npw_pad, nb, st);
    ++kept;
  }
  return launch_check();
}

// Lowest n_eig eigenpairs of the Liouville superoperator (eq. bse_tddft) by block Davidson with
// the basis on the device: Rayleigh-Ritz through the FP64 GEMMs, Jacobi on the host, corrections
// P_c K r with Teter's K per band, converged pairs kept in the basis without new directions,
// restart from the Ritz vectors when the basis is full.
int stern_liouville_davidson(stern_system* S, int n_eig, int block, int max_basis, int max_iter, double tol,
                             unsigned long long seed, double* eig, double* vec, int* n_iter, double* max_resid) {
  using cd = std::complex<double>;
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (n_eig <= 0 || !eig) return fail(STERN_ERR_INVALID_ARG, "need n_eig > 0 and eig");
  if (!(tol > 0)) return fail(STERN_ERR_INVALID_ARG, "tol must be > 0");
  const int bl = block > 0 ? block : n_eig;
  const int mb = max_basis > 0 ? max_basis : std::max(8 * n_eig, n_eig + 4 * bl);
  if (mb < n_eig + bl) return fail(STERN_ERR_INVALID_ARG, "max_basis %d < n_eig + block = %d", mb, n_eig + bl);
  const int mi = max_iter > 0 ? max_iter : 200;
  Scope sc(S->device, &S->alloc);
  const int n_start = std::max(n_eig, bl);
  CHECKED(liouville_setup(S, std::max(n_start, bl)));
  const int nb = S->n_occ, K = S->hb.npw_pad, npw = S->hb.npw;
  const int Lt = nb * K;
  const int cap = (mb + 63) / 64 * 64;
  hipStream_t st = S->stream;
  CHECKED(S->lv_dot.ensure((size_t)std::max(mb, n_start) * nb * sizeof(Z64)));
  CHECKED(S->lv_coef.ensure((size_t)std::max(mb, n_start) * sizeof(Z64)));
  for (DBuf* d : {&S->dv_V, &S->dv_W}) {
    CHECKED(d->ensure((size_t)cap * Lt * sizeof(Z64)));
    launch_fill_zero(d->as<Z64>(), (size_t)cap * Lt, st);
  }
  for (DBuf* d : {&S->dv_X, &S->dv_LX, &S->dv_T}) {
    CHECKED(d->ensure((size_t)std::max(n_start, n_eig) * Lt * sizeof(Z64)));
    launch_fill_zero(d->as<Z64>(), (size_t)std::max(n_start, n_eig) * Lt, st);
  }
  // corrections (block) and, at a restart, the new basis and its L image (up to mb each)
  CHECKED(S->dv_LT.ensure((size_t)(std::max(n_start, bl) + 2 * mb) * Lt * sizeof(Z64)));
  Z64 *V = S->dv_V.as<Z64>(), *W = S->dv_W.as<Z64>(), *X = S->dv_X.as<Z64>(), *LX = S->dv_LX.as<Z64>(),
      *T = S->dv_T.as<Z64>();
  // seeded random start, shaped by P_c K
  {
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd;
    std::vector<double> h((size_t)n_start * nb * npw * 2);
    for (auto& x : h) x = nd(rng);
    CHECKED(rows_in(S, n_start * nb, h.data(), STERN_MEM_HOST, S->wr));
    CHECKED(precond_rows(S, S->wr.as<Z64>(), T, n_start * nb));
  }
  int m = 0, kept = 0;
  CHECKED(dav_orth(S, V, cap, m, T, n_start, Lt, kept));
  if (kept < n_eig)  // the start spans fewer directions than pairs asked for (a smaller space)
    return fail(STERN_ERR_INVALID_ARG, "only %d independent start vectors for %d eigenpairs", kept, n_eig);
  HIPOK(hipMemcpyAsync(V, T, (size_t)kept * Lt * sizeof(Z64), hipMemcpyDeviceToDevice, st));
  CHECKED(liouville_rows(S, V, W, kept));
  m = kept;
  std::vector<double> theta, rn(n_eig, 0.0);
  std::vector<cd> Y;
  std::vector<Z64> C, d;
  bool all_conv = false;
  int it = 0;
  for (; it < mi; ++it) {
    // Rayleigh-Ritz on the m basis vectors
    CHECKED(dav_vh_x(S, V, cap, W, m, Lt, C));  // C[n][i] = <v_i|w_n> = H[i][n]
    std::vector<cd> H((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int n = 0; n < m; ++n) {
        const Z64 a = C[(size_t)n * cap + i], b = C[(size_t)i * cap + n];
        H[(size_t)i * m + n] = 0.5 * (cd(a.re, a.im) + std::conj(cd(b.re, b.im)));
      }
    jacobi_zheev(H, m, theta, Y);
    // Ritz vectors X = V Y and L X = W Y for the n_eig lowest
    std::vector<Z64> Cy((size_t)n_eig * cap, zmk(0.0, 0.0));
    for (int n = 0; n < n_eig; ++n)
      for (int i = 0; i < m; ++i) Cy[(size_t)n * cap + i] = zmk(Y[(size_t)i * m + n].real(), Y[(size_t)i * m + n].imag());
    launch_fill_zero(X, (size_t)n_eig * Lt, st);
    launch_fill_zero(LX, (size_t)n_eig * Lt, st);
    CHECKED(dav_v_c(S, V, cap, Cy, X, n_eig, Lt));
    CHECKED(dav_v_c(S, W, cap, Cy, LX, n_eig, Lt));
    // residuals r = L x - theta x into T
    HIPOK(hipMemcpyAsync(T, LX, (size_t)n_eig * Lt * sizeof(Z64), hipMemcpyDeviceToDevice, st));
    std::vector<Z64> c(n_eig);
    for (int n = 0; n < n_eig; ++n) c[n] = zmk(-theta[n], 0.0);
    CHECKED(upload_coef(S, c));
    launch_blk_axpy(T, X, S->lv_coef.as<Z64>(), nb, K, n_eig * nb, st);
    CHECKED(block_dots(S, T, T, n_eig, d));
    std::vector<int> todo;
    for (int n = 0; n < n_eig; ++n) {
      rn[n] = std::sqrt(std::max(0.0, d[n].re));
      if (!(rn[n] <= tol * std::fabs(theta[n]))) todo.push_back(n);
    }
    if (todo.empty()) {
      all_conv = true;
      break;
    }
    // corrections P_c K r of the unconverged pairs, packed at the front of T
    const int nt = std::min((int)todo.size(), bl);
    for (int j = 0; j < nt; ++j)
      if (todo[j] != j)
        HIPOK(hipMemcpyAsync(T + (size_t)j * Lt, T + (size_t)todo[j] * Lt, (size_t)Lt * sizeof(Z64),
                             hipMemcpyDeviceToDevice, st));
    CHECKED(precond_rows(S, T, S->dv_LT.as<Z64>(), nt * nb));
    HIPOK(hipMemcpyAsync(T, S->dv_LT.p, (size_t)nt * Lt * sizeof(Z64), hipMemcpyDeviceToDevice, st));
    if (m + nt > mb) {  // thick restart: the lowest nk Ritz vectors (at least n_eig, half the basis)
      const int nk = std::min(m, std::max(n_eig, mb / 2));
      std::vector<Z64> Ck((size_t)nk * cap, zmk(0.0, 0.0));
      for (int n = 0; n < nk; ++n)
        for (int i = 0; i < m; ++i)
          Ck[(size_t)n * cap + i] = zmk(Y[(size_t)i * m + n].real(), Y[(size_t)i * m + n].imag());
      Z64 *Vn = S->dv_LT.as<Z64>() + (size_t)nt * Lt, *Wn = Vn + (size_t)nk * Lt;
      launch_fill_zero(Vn, (size_t)2 * nk * Lt, st);
      CHECKED(dav_v_c(S, V, cap, Ck, Vn, nk, Lt));
      CHECKED(dav_v_c(S, W, cap, Ck, Wn, nk, Lt));
      HIPOK(hipMemcpyAsync(V, Vn, (size_t)nk * Lt * sizeof(Z64), hipMemcpyDeviceToDevice, st));
      HIPOK(hipMemcpyAsync(W, Wn, (size_t)nk * Lt * sizeof(Z64), hipMemcpyDeviceToDevice, st));
      launch_fill_zero(V + (size_t)nk * Lt, (size_t)(cap - nk) * Lt, st);
      launch_fill_zero(W + (size_t)nk * Lt, (size_t)(cap - nk) * Lt, st);
      m = nk;
    }
    CHECKED(dav_orth(S, V, cap, m, T, nt, Lt, kept));
    if (kept == 0) break;  // no new direction: the basis is exhausted
    HIPOK(hipMemcpyAsync(V + (size_t)m * Lt, T, (size_t)kept * Lt * sizeof(Z64), hipMemcpyDeviceToDevice, st));
    CHECKED(liouville_rows(S, V + (size_t)m * Lt, W + (size_t)m * Lt, kept));
    m += kept;
  }
  for (int n = 0; n < n_eig; ++n) eig[n] = theta[n];
  double mr = 0.0;
  for (int n = 0; n < n_eig; ++n) mr = std::max(mr, rn[n] / std::max(std::fabs(theta[n]), 1e-300));
  if (n_iter) *n_iter = it;
  if (max_resid) *max_resid = mr;
  if (vec) CHECKED(rows_out(S, n_eig * nb, X, nullptr, vec, STERN_MEM_HOST));
  return all_conv ? STERN_OK : STERN_WARN_NOT_CONVERGED;
}

// Lanczos chain of the Liouville superoperator from d_v = P_c dV psi_v of one field (Sec. II.C.1:
// absorption spectra without the excitation energies): q_0 = d / ||d||, w = L q_k - beta_{k-1} q_{k-1},
// alpha_k = <q_k|w>, w -= alpha_k q_k, beta_k = ||w||, q_{k+1} = w / beta_k; inner products over all
// bands. Plain three-term recurrence, no reorthogonalisation.
int stern_liouville_lanczos(stern_system* S, const double* dv, int n_steps, double* alpha, double* beta, double* norm2,
                            int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!dv || !alpha || !beta || !norm2 || n_steps <= 0) return fail(STERN_ERR_INVALID_ARG, "bad arguments");
  if (mem_kind != STERN_MEM_HOST && mem_kind != STERN_MEM_DEVICE) return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  Scope sc(S->device, &S->alloc);
  CHECKED(liouville_setup(S, 1));
  const int nb = S->n_occ, K = S->hb.npw_pad, N = S->hb.N;
  const size_t n3 = (size_t)N * N * N;
  hipStream_t st = S->stream;
  CHECKED(S->lv_dot.ensure((size_t)nb * sizeof(Z64)));
  CHECKED(S->lv_coef.ensure(sizeof(Z64)));
  const double* dvd = dv;
  if (mem_kind == STERN_MEM_HOST) {
    CHECKED(S->dv_dev.ensure(n3 * sizeof(double)));
    HIPOK(hipMemcpyAsync(S->dv_dev.p, dv, n3 * sizeof(double), hipMemcpyHostToDevice, st));
    dvd = S->dv_dev.as<double>();
  }
  // d_v = -b_v of the Sternheimer right-hand sides of this field (the sign leaves the chain unchanged)
  CHECKED(setup_batch(S, 0, 1, 0, nb, dvd, (double)S->hb.npw * sizeof(Z64)));
  const CgState cs = cg_state(S);
  Z64 *Qp = S->wx.as<Z64>(), *Q = S->wp.as<Z64>(), *Wv = S->wq.as<Z64>();
  std::vector<Z64> d;
  CHECKED(block_dots(S, cs.b, cs.b, 1, d));
  *norm2 = d[0].re;
  if (!(d[0].re > 0.0)) return fail(STERN_ERR_INVALID_ARG, "the field gives P_c dV psi_v = 0 for every band");
  launch_fill_zero(Qp, (size_t)nb * K, st);
  HIPOK(hipMemcpyAsync(Q, cs.b, (size_t)nb * K * sizeof(Z64), hipMemcpyDeviceToDevice, st));
  std::vector<Z64> c(1, zmk(1.0 / std::sqrt(d[0].re), 0.0));
  CHECKED(upload_coef(S, c));
  launch_blk_scale(Q, S->lv_coef.as<Z64>(), nb, K, nb, st);
  double bprev = 0.0;
  for (int k = 0; k < n_steps; ++k) {
    CHECKED(liouville_rows(S, Q, Wv, 1));
    c[0] = zmk(-bprev, 0.0);
    CHECKED(upload_coef(S, c));
    launch_blk_axpy(Wv, Qp, S->lv_coef.as<Z64>(), nb, K, nb, st);
    CHECKED(block_dots(S, Q, Wv, 1, d));
    alpha[k] = d[0].re;
    c[0] = zmk(-alpha[k], 0.0);
    CHECKED(upload_coef(S, c));
    launch_blk_axpy(Wv, Q, S->lv_coef.as<Z64>(), nb, K, nb, st);
    CHECKED(block_dots(S, Wv, Wv, 1, d));
    beta[k] = std::sqrt(std::max(0.0, d[0].re));
    if (k + 1 == n_steps) break;
    if (!(beta[k] > 0.0)) {  // an invariant subspace: the chain ends exactly here
      for (int j = k + 1; j < n_steps; ++j) alpha[j] = beta[j] = 0.0;
      break;
    }
    std::swap(Qp, Q);  // q_{k-1} <- q_k
    HIPOK(hipMemcpyAsync(Q, Wv, (size_t)nb * K * sizeof(Z64), hipMemcpyDeviceToDevice, st));
    c[0] = zmk(1.0 / beta[k], 0.0);
    CHECKED(upload_coef(S, c));
    launch_blk_scale(Q, S->lv_coef.as<Z64>(), nb, K, nb, st);
    bprev = beta[k];
  }
  return launch_check();
}

int stern_lanczos_spectrum(int n_steps, const double* alpha, const double* beta, double norm2, int n_omega,
                           const double* omega, double eta, double* out) {
  if (n_steps <= 0 || n_omega < 0 || !alpha || !beta || (n_omega > 0 && (!omega || !out)) || !(eta > 0.0))
    return fail(STERN_ERR_INVALID_ARG, "bad arguments");
  for (int i = 0; i < n_omega; ++i) {
    const std::complex<double> z(omega[i], eta);
    std::complex<double> g = 0.0;
    for (int k = n_steps - 1; k >= 0; --k) {
      const std::complex<double> tail = k < n_steps - 1 ? beta[k] * beta[k] * g : 0.0;
      g = 1.0 / (z - alpha[k] - tail);
    }
    out[i] = -norm2 * g.imag() / 3.14159265358979323846;
  }
  return STERN_OK;
}

int stern_apply_pc(stern_system* S, int n_vec, const double* c, double* out, int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!S->have_occ) return fail(STERN_ERR_STATE, "set_occupied has not been called");
  if (n_vec <= 0) return STERN_OK;
  if (!c || !out) return fail(STERN_ERR_INVALID_ARG, "NULL array");
  Scope sc(S->device, &S->alloc);
  CHECKED(ensure_workspace(S, std::max(n_vec, S->ws_solves)));
  CHECKED(rows_in(S, n_vec, c, mem_kind, S->wp));
  CHECKED(apply_pc_rows(S, S->wp.as<Z64>(), nullptr, n_vec));
  CHECKED(launch_check());
  return rows_out(S, n_vec, S->wp.as<Z64>(), nullptr, out, mem_kind);
}

int stern_apply_pc_noalloc(stern_system* S, int n_vec, const double* c, double* out) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!S->have_occ) return fail(STERN_ERR_STATE, "set_occupied has not been called");
  if (n_vec < 0) return fail(STERN_ERR_INVALID_ARG, "n_vec must be >= 0");
  if (n_vec == 0) return STERN_OK;
  if (!c || !out) return fail(STERN_ERR_INVALID_ARG, "NULL array");
  const int npw = S->hb.npw, K = S->hb.npw_pad, M = S->nocc_pad;
  const int ns = choose_nsplit(M, n_vec, K, S->gemm64_wg);
  // scratch: rows in column order [n][K], split-K partials [ns][n][M], C [n][M]
  const size_t rows_b = (size_t)n_vec * K * sizeof(Z64);
  const size_t part_b = (size_t)ns * n_vec * M * sizeof(Z64);
  const size_t need = rows_b + part_b + (size_t)n_vec * M * sizeof(Z64);
  if (need > (size_t)STERN_NOALLOC_SCRATCH_BYTES)
    return fail(STERN_ERR_INVALID_ARG, "%d rows need %zu bytes of scratch; the limit is %zu", n_vec, need,
                (size_t)STERN_NOALLOC_SCRATCH_BYTES);
  Scope sc(S->device, &S->alloc);
  void* scr = nullptr;
  CHECKED(scratch_address(S->device, &scr));
  unsigned char* base = static_cast<unsigned char*>(scr);
  Z64* rows = reinterpret_cast<Z64*>(base);
  Z64* part = reinterpret_cast<Z64*>(base + rows_b);
  Z64* cmat = reinterpret_cast<Z64*>(base + rows_b + part_b);
  hipStream_t st = S->stream;
  // the padding entries of the rows take part in the reduce and must be zero
  launch_fill_zero(rows, (size_t)n_vec * K, st);
  launch_permute(reinterpret_cast<const Z64*>(c), npw, rows, K, S->perm.as<int>(), npw, n_vec, true, st);
  launch_zgemm_reduce(S->psi.as<Z64>(), M, rows, K, nullptr, n_vec, K, part, ns, st);
  launch_sum_parts(part, ns, n_vec, M, -1.0, cmat, st);
  launch_zgemm_expand(S->psi.as<Z64>(), M, cmat, rows, K, nullptr, n_vec, K, st);
  launch_permute(rows, K, reinterpret_cast<Z64*>(out), npw, S->perm.as<int>(), npw, n_vec, false, st);
  return launch_check();
}

static int apply_chi0_impl(stern_system* S, int n_pert, const double* dv_r, double* dn_r, const stern_opts* opts,
                           stern_stats* stats);

int stern_apply_chi0(stern_system* S, int n_pert, const double* dv_r, double* dn_r, const stern_opts* opts,
                     stern_stats* stats) {
  if (!S || !opts || !opts->use_graph || opts->profile) return apply_chi0_impl(S, n_pert, dv_r, dn_r, opts, stats);
  // stream capture is not allowed on the legacy default stream: run on the system's own stream
  Scope sc(S->device, &S->alloc);
  if (!S->own_stream) HIPOK(hipStreamCreateWithFlags(&S->own_stream, hipStreamNonBlocking));
  HIPOK(hipStreamSynchronize(S->stream));
  hipStream_t caller = S->stream;
  S->stream = S->own_stream;
  const int rc = apply_chi0_impl(S, n_pert, dv_r, dn_r, opts, stats);
  (void)hipStreamSynchronize(S->stream);
  S->stream = caller;
  return rc;
}

static int apply_chi0_impl(stern_system* S, int n_pert, const double* dv_r, double* dn_r, const stern_opts* opts,
                           stern_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!S->have_occ) return fail(STERN_ERR_STATE, "set_occupied has not been called");
  if (!opts) return fail(STERN_ERR_INVALID_ARG, "opts is NULL");
  if (n_pert <= 0 || !dv_r || !dn_r) return fail(STERN_ERR_INVALID_ARG, "need n_pert > 0, dv_r and dn_r");
  if (opts->precision != STERN_FP64 && opts->precision != STERN_MIXED)
    return fail(STERN_ERR_INVALID_ARG, "precision must be STERN_FP64 or STERN_MIXED");
  if (opts->inner_tol < 0 || opts->max_outer < 0) return fail(STERN_ERR_INVALID_ARG, "bad inner_tol / max_outer");
  if (opts->inner_op != STERN_INNER_PROJECTED && opts->inner_op != STERN_INNER_SHIFTED)
    return fail(STERN_ERR_INVALID_ARG, "inner_op %d is not one of STERN_INNER_*", opts->inner_op);
  if (opts->guess != STERN_GUESS_ZERO && opts->guess != STERN_GUESS_LEARNED && opts->guess != STERN_GUESS_LEARNED_K &&
      opts->guess != STERN_GUESS_PREVIOUS)
    return fail(STERN_ERR_INVALID_ARG, "guess must be one of STERN_GUESS_*");
  const bool learned = opts->guess == STERN_GUESS_LEARNED || opts->guess == STERN_GUESS_LEARNED_K;
  const bool warm = opts->guess == STERN_GUESS_PREVIOUS;
  if (learned) {
    if (!opts->model) return fail(STERN_ERR_INVALID_ARG, "a learned start needs a model");
    if (!S->have_coarse) return fail(STERN_ERR_UNSUPPORTED, "grid %d has no coarse grid for the learned guess", S->hb.N);
    if (opts->model->device != S->device) return fail(STERN_ERR_INVALID_ARG, "model and system on different devices");
  }
  if (opts->mem_kind != STERN_MEM_HOST && opts->mem_kind != STERN_MEM_DEVICE)
    return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  if (!(opts->tol > 0)) return fail(STERN_ERR_INVALID_ARG, "tol must be > 0");
  const double omega = opts->omega_imag;
  if (!(omega >= 0.0) || !std::isfinite(omega)) return fail(STERN_ERR_INVALID_ARG, "omega_imag must be finite and >= 0");
  if (omega > 0.0 && (opts->precision != STERN_FP64 || learned))
    return fail(STERN_ERR_UNSUPPORTED, "the response at imaginary frequency runs in FP64 with Teter's preconditioner");
  const int v0 = opts->band_begin;
  const int v1 = opts->band_end > 0 ? opts->band_end : S->n_occ;
  if (v0 < 0 || v1 > S->n_occ || v0 >= v1) return fail(STERN_ERR_INVALID_ARG, "bad band range [%d, %d)", v0, v1);
  if (warm && (S->keep_np != n_pert || S->keep_v0 != v0 || S->keep_v1 != v1))
    return fail(STERN_ERR_STATE, "no kept solutions for %d fields x bands [%d, %d) (kept: %d x [%d, %d))", n_pert, v0,
                v1, S->keep_np, S->keep_v0, S->keep_v1);
  if (opts->n_sample < 0 || (opts->n_sample > 0 && (!opts->sample_pairs || !opts->sample_x)))
    return fail(STERN_ERR_INVALID_ARG, "bad sample request");
  for (int k = 0; k < opts->n_sample; ++k) {
    const int v = opts->sample_pairs[2 * k], i = opts->sample_pairs[2 * k + 1];
    if (v < v0 || v >= v1 || i < 0 || i >= n_pert) return fail(STERN_ERR_INVALID_ARG, "sample pair %d out of range", k);
  }
  Scope sc(S->device, &S->alloc);
  hipStream_t st = S->stream;
  const HostBasis& hb = S->hb;
  const int N = hb.N, K = hb.npw_pad;
  const size_t n3 = (size_t)N * N * N;
  const int nb = v1 - v0;
  const int max_iter = opts->max_iter > 0 ? opts->max_iter : 1000;
  const int check_every = opts->check_every > 0 ? opts->check_every : 1;
  const double tol = opts->tol;
  const double inner_tol = opts->inner_tol > 0 ? opts->inner_tol : 1e-4;
  const int max_outer = opts->max_outer > 0 ? opts->max_outer : 8;
  const bool use_graph = opts->use_graph != 0;
  const double vecb = (double)hb.npw * sizeof(Z64);  // bytes of one coefficient vector
  S->prof_on = opts->profile != 0;
  S->recs.clear();
  S->ev_used = 0;

  // perturbations per batch
  int per = opts->max_batch > 0 ? std::max(1, opts->max_batch / nb) : 0;
  if (per == 0) {
    size_t free_b = 0, total_b = 0;
    HIPOK(hipMemGetInfo(&free_b, &total_b));
    const size_t have = (size_t)S->ws_solves >= (size_t)nb ? S->wx.n * 6 + S->pen.n : 0;
    const size_t per_solve = (size_t)K * sizeof(Z64) * 6 + (size_t)N * hb.ncol_pad * sizeof(Z64) +
                             (size_t)(2 * std::max(S->nocc_pad, 64)) * sizeof(Z64) * 2 + 64;
    const size_t budget = (size_t)(0.6 * (double)(free_b + have));
    per = (int)std::max<size_t>(1, budget / (per_solve * nb));
  }
  per = std::min(per, n_pert);
  const int max_ns = per * nb;
  CHECKED(ensure_workspace(S, max_ns));
  if (opts->precision == STERN_MIXED) CHECKED(ensure_workspace32(S, max_ns));
  CHECKED(S->pert_out.ensure((size_t)n_pert * sizeof(int)));
  {
    std::vector<int> po(n_pert);
    for (int i = 0; i < n_pert; ++i) po[i] = i;
    HIPOK(hipMemcpyAsync(S->pert_out.p, po.data(), n_pert * sizeof(int), hipMemcpyHostToDevice, st));
    HIPOK(hipStreamSynchronize(st));  // po is released at the end of this block
  }
  const double* dv_dev = dv_r;
  double* dn_dev = dn_r;
  if (opts->mem_kind == STERN_MEM_HOST) {
    CHECKED(S->dv_dev.ensure((size_t)n_pert * n3 * sizeof(double)));
    CHECKED(S->dn_dev.ensure((size_t)n_pert * n3 * sizeof(double)));
    HIPOK(hipMemcpyAsync(S->dv_dev.p, dv_r, (size_t)n_pert * n3 * sizeof(double), hipMemcpyHostToDevice, st));
    dv_dev = S->dv_dev.as<double>();
    dn_dev = S->dn_dev.as<double>();
  }
  const bool keep = opts->keep_solutions != 0;
  if (keep) {  // invalid until every batch has stored its solutions
    if (!warm) S->keep_np = 0;
    CHECKED(S->xkeep.ensure((size_t)n_pert * nb * K * sizeof(Z64)));
  }
  CgState cs = cg_state(S);
  const FftGeom g = S->geom();
  std::vector<int> all_iters, all_flag;
  std::vector<double> all_tres;
  all_iters.reserve((size_t)n_pert * nb);
  long long tot_iters = 0;
  int n_restart = 0, n_fallback = 0, n_rejected = 0;

  std::vector<int> h_flag(max_ns);
  for (int i0 = 0; i0 < n_pert; i0 += per) {
    const int i1 = std::min(n_pert, i0 + per);
    const int ns = (i1 - i0) * nb;
    CHECKED(setup_batch(S, i0, i1, v0, nb, dv_dev, vecb));
    const bool with_x0 = opts->guess == STERN_GUESS_LEARNED || warm;
    if (learned)
      CHECKED(learned_guess(S, opts->model, cs, ns, n_rejected, opts->precision == STERN_MIXED, with_x0));
    if (warm) CHECKED(warm_start(S, cs, (size_t)i0 * nb, ns, omega, tol, n_rejected));
    std::vector<int> all;
    if (warm) {  // starts already within tol are done
      HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPOK(hipStreamSynchronize(st));
      for (int s = 0; s < ns; ++s)
        if (h_flag[s] != 2) all.push_back(s);
    } else {
      all.resize(ns);
      for (int s = 0; s < ns; ++s) all[s] = s;
    }
    if (omega > 0.0) {
      CHECKED(run_cocg64(S, cs, all, omega, tol, max_iter, check_every, n_restart, vecb, warm));
    } else if (opts->precision == STERN_MIXED) {
      CHECKED(run_mixed(S, cs, all, tol, inner_tol, max_outer, max_iter, check_every, n_restart, n_fallback, vecb,
                        use_graph, opts->inner_op));
    } else {
      CHECKED(run_pcg64(S, cs, all, tol, max_iter, check_every, n_restart, vecb, use_graph, with_x0));
      if (learned || warm) {  // solves the start did not bring below tol: Teter-PCG from zero
        HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPOK(hipStreamSynchronize(st));
        std::vector<int> rest;
        for (int s = 0; s < ns; ++s)
          if (h_flag[s] != 2) rest.push_back(s);
        if (!rest.empty()) {
          n_fallback += (int)rest.size();
          CgState teter = cs;
          teter.kprec = nullptr;
          CHECKED(run_pcg64(S, teter, rest, tol, max_iter, check_every, n_restart, vecb, use_graph));
        }
      }
    }
    if (keep)
      HIPOK(hipMemcpyAsync(S->xkeep.as<Z64>() + (size_t)i0 * nb * K, cs.x, (size_t)ns * K * sizeof(Z64),
                           hipMemcpyDeviceToDevice, st));
    // dn_i = 4/Omega Re sum_v conj(psi_v(r)) x_{v,i}(r)
    CHECKED(timed(S, STERN_K_XINV, ns * (vecb + (double)N * hb.ncol * 16.0), 0.0,
                  [&] { launch_xinv(g, cs.x, nullptr, ns, S->pen.as<Z64>(), st); }));
    CHECKED(timed(S, STERN_K_DN,
                  ns * (double)N * hb.ncol * 16.0 + (double)(i1 - i0) * nb * n3 * 16.0 + (double)(i1 - i0) * n3 * 8.0,
                  0.0, [&] {
                    launch_plane_dn(g, S->pen.as<Z64>(), S->psi_r.as<Z64>(), v0, nb, i1 - i0,
                                    S->pert_out.as<int>() + i0, 4.0 / hb.omega, dn_dev, st);
                  }));
    CHECKED(launch_check());
    // per-solve statistics
    std::vector<int> hi(ns);
    std::vector<double> ht(ns);
    HIPOK(hipMemcpyAsync(hi.data(), cs.iters, ns * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPOK(hipMemcpyAsync(ht.data(), cs.tres, ns * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPOK(hipMemcpyAsync(h_flag.data(), cs.flag, ns * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    for (int s = 0; s < ns; ++s) {
      all_iters.push_back(hi[s]);
      all_tres.push_back(ht[s]);
      all_flag.push_back(h_flag[s]);
      tot_iters += hi[s];
    }
    // sampled solution vectors
    for (int k = 0; k < opts->n_sample; ++k) {
      const int v = opts->sample_pairs[2 * k], i = opts->sample_pairs[2 * k + 1];
      if (i < i0 || i >= i1) continue;
      const int row = (i - i0) * nb + (v - v0);
      CHECKED(rows_out(S, 1, cs.x, &row, opts->sample_x + 2 * (size_t)k * hb.npw, STERN_MEM_HOST));
    }
  }
  if (opts->mem_kind == STERN_MEM_HOST)
    HIPOK(hipMemcpyAsync(dn_r, dn_dev, (size_t)n_pert * n3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  if (keep) {
    S->keep_np = n_pert;
    S->keep_v0 = v0;
    S->keep_v1 = v1;
  }
  if (stats) {
    for (int k = 0; k < STERN_NKERNEL; ++k) {
      stats->kernel_launches[k] = 0;
      stats->kernel_ms[k] = stats->kernel_bytes[k] = stats->kernel_flops[k] = 0.0;
    }
    for (const auto& r : S->recs) {
      float ms = 0.f;
      HIPOK(hipEventElapsedTime(&ms, S->events[r.ev], S->events[r.ev + 1]));
      stats->kernel_launches[r.cls] += 1;
      stats->kernel_ms[r.cls] += ms;
      stats->kernel_bytes[r.cls] += r.bytes;
      stats->kernel_flops[r.cls] += r.flops;
    }
  }
  S->prof_on = false;
  S->recs.clear();
  const int nsol = (int)all_iters.size();
  int nconv = 0, mx = 0;
  double mres = 0.0;
  for (int s = 0; s < nsol; ++s) {
    if (all_flag[s] == 2) ++nconv;
    mx = std::max(mx, all_iters[s]);
    mres = std::max(mres, all_tres[s]);
  }
  if (stats) {
    stats->n_solves = nsol;
    stats->n_converged = nconv;
    stats->n_fallback = n_fallback;
    stats->n_restarts = n_restart;
    stats->n_guess_rejected = n_rejected;
    stats->total_iters = tot_iters;
    stats->max_iters = mx;
    stats->max_true_resid = mres;
    if (stats->iters) std::memcpy(stats->iters, all_iters.data(), nsol * sizeof(int));
    if (stats->resid) std::memcpy(stats->resid, all_tres.data(), nsol * sizeof(double));
    stats->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return nconv == nsol ? STERN_OK : STERN_WARN_NOT_CONVERGED;
}

int stern_apply_chi0_many(int n_sys, stern_system* const* sys, const int* n_pert, const double* const* dv_r,
                          double* const* dn_r, const stern_opts* opts, stern_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (n_sys <= 0 || !sys || !n_pert || !dv_r || !dn_r || !opts)
    return fail(STERN_ERR_INVALID_ARG, "need n_sys > 0 and non-NULL arrays");
  for (int k = 0; k < n_sys; ++k) {
    if (!sys[k]) return fail(STERN_ERR_INVALID_ARG, "system %d is NULL", k);
    if (!sys[k]->have_occ) return fail(STERN_ERR_STATE, "system %d has no occupied states", k);
    for (int j = 0; j < k; ++j)
      if (sys[j] == sys[k]) return fail(STERN_ERR_INVALID_ARG, "system %d appears twice", k);
  }
  const int workers = std::min(n_sys, 8);
  std::vector<hipStream_t> streams(workers, nullptr);
  std::vector<hipStream_t> saved(n_sys);
  for (int k = 0; k < n_sys; ++k) {  // inputs were produced on the systems' own streams
    Scope sc(sys[k]->device, &sys[k]->alloc);
    HIPOK(hipStreamSynchronize(sys[k]->stream));
    saved[k] = sys[k]->stream;
  }
  for (int w = 0; w < workers; ++w) {
    Scope sc(sys[w]->device);
    HIPOK(hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking));
  }
  std::vector<int> rc(n_sys, 0);
  std::vector<stern_stats> st(n_sys);
  std::vector<std::string> err(n_sys);
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w) {
    pool.emplace_back([&, w]() {
      for (int k = w; k < n_sys; k += workers) {
        stern_system* S = sys[k];
        S->stream = streams[w];
        std::memset(&st[k], 0, sizeof(stern_stats));
        rc[k] = stern_apply_chi0(S, n_pert[k], dv_r[k], dn_r[k], opts, stats ? &st[k] : nullptr);
        if (rc[k] < 0) err[k] = g_err;
        S->stream = saved[k];
      }
    });
  }
  for (auto& t : pool) t.join();
  for (int w = 0; w < workers; ++w) {
    Scope sc(sys[w]->device);
    (void)hipStreamDestroy(streams[w]);
  }
  int out = STERN_OK;
  for (int k = 0; k < n_sys; ++k) {
    if (rc[k] < 0) {
      g_err = "system " + std::to_string(k) + ": " + err[k];
      return rc[k];
    }
    if (rc[k] == STERN_WARN_NOT_CONVERGED) out = STERN_WARN_NOT_CONVERGED;
  }
  if (stats) {
    stern_stats a;
    std::memset(&a, 0, sizeof a);
    for (int k = 0; k < n_sys; ++k) {
      a.n_solves += st[k].n_solves;
      a.n_converged += st[k].n_converged;
      a.n_fallback += st[k].n_fallback;
      a.n_restarts += st[k].n_restarts;
      a.n_guess_rejected += st[k].n_guess_rejected;
      a.total_iters += st[k].total_iters;
      a.max_iters = std::max(a.max_iters, st[k].max_iters);
      a.max_true_resid = std::max(a.max_true_resid, st[k].max_true_resid);
      for (int c = 0; c < STERN_NKERNEL; ++c) {
        a.kernel_launches[c] += st[k].kernel_launches[c];
        a.kernel_ms[c] += st[k].kernel_ms[c];
        a.kernel_bytes[c] += st[k].kernel_bytes[c];
        a.kernel_flops[c] += st[k].kernel_flops[c];
      }
    }
    a.iters = stats->iters;
    a.resid = stats->resid;
    a.wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *stats = a;
  }
  return out;
}

// ---------------------------------------------------------- PDEP Davidson ----
// Sec. II.A, eq. pdep: the lowest eigenpairs of chi-bar0 = v^{1/2} chi0 v^{1/2},
// v^{1/2}(G) = sqrt(4 pi) / |G|, found iteratively, every chi-bar0 product being
// one stern_apply_chi0 over a block of trial potentials.
//
// Potentials are real and band-limited to |G|^2 < ecut_pot, G != 0. They are
// carried as real coordinates u in R^{2m}, m = number of half-space
// representatives G_j: u[2j] = sqrt(2) Re c(G_j), u[2j + 1] = sqrt(2) Im c(G_j),
// c(-G) = conj c(G), which makes sum_G |c(G)|^2 = |u|^2, so chi-bar0 is a real
// symmetric matrix in these coordinates.

namespace {


// Band-limited potentials of a system: canonical indices of each half-space
// representative G_j and of -G_j in the wave-function sphere, and v^{1/2}(G_j);
// `all` lists every G of the potential sphere (both signs), canonical order.
struct PotBasis {
  std::vector<int> rep, neg, all;
  std::vector<double> vh;
};

static int pot_basis(const stern_system* S, double ecut_pot, PotBasis& pb) {
  const HostBasis& hb = S->hb;
  if (!(ecut_pot > 0) || ecut_pot > hb.ecut)
    return fail(STERN_ERR_INVALID_ARG, "ecut_pot must be in (0, ecut] (got %g)", ecut_pot);
  const double b2 = hb.b * hb.b;
  for (int k = 0; k < hb.npw; ++k) {
    const int x = hb.miller[3 * k], y = hb.miller[3 * k + 1], z = hb.miller[3 * k + 2];
    const double g2 = b2 * (double)(x * x + y * y + z * z);
    if (g2 == 0.0 || !(g2 < ecut_pot)) continue;
    pb.all.push_back(k);
    if (!(x > 0 || (x == 0 && y > 0) || (x == 0 && y == 0 && z > 0))) continue;
    int kn = -1;  // -G sits in the same |n|^2 shell of the canonical order
    for (int q = 0; q < hb.npw && kn < 0; ++q)
      if (hb.miller[3 * q] == -x && hb.miller[3 * q + 1] == -y && hb.miller[3 * q + 2] == -z) kn = q;
    if (kn < 0) return fail(STERN_ERR_INVALID_ARG, "-G of a potential G is missing from the sphere");
    pb.rep.push_back(k);
    pb.neg.push_back(kn);
    pb.vh.push_back(std::sqrt(4.0 * M_PI / g2));
  }
  if (pb.rep.empty()) return fail(STERN_ERR_INVALID_ARG, "no nonzero G with |G|^2 < %g", ecut_pot);
  return 0;
}

struct PdepWork {
  DBuf rows, pen, zf, dv, dn;
  void release() {
    for (DBuf* d : {&rows, &pen, &zf, &dv, &dn}) d->release();
  }
};

// W = chi-bar0 U for nb coordinate vectors U [nb][2m] (host), through one chi0 apply.
static int pdep_apply(stern_system* S, const PotBasis& pb, const stern_opts& o, const double* U, int nb, double* W,
               PdepWork& wk, long long& solves, long long& iters) {
  const HostBasis& hb = S->hb;
  const int K = hb.npw_pad, N = hb.N, m = (int)pb.rep.size();
  const size_t n3 = (size_t)N * N * N;
  hipStream_t st = S->stream;
  CHECKED(wk.rows.ensure((size_t)nb * K * sizeof(Z64)));
  CHECKED(wk.pen.ensure((size_t)nb * N * hb.ncol_pad * sizeof(Z64)));
  CHECKED(wk.zf.ensure((size_t)nb * n3 * sizeof(Z64)));
  CHECKED(wk.dv.ensure((size_t)nb * n3 * sizeof(double)));
  CHECKED(wk.dn.ensure((size_t)nb * n3 * sizeof(double)));
  // coefficients of v^{1/2} phi on the wave-function sphere (column order), zero elsewhere
  std::vector<Z64> h((size_t)nb * K, zmk(0.0, 0.0));
  const double r2 = 1.0 / std::sqrt(2.0);
  for (int f = 0; f < nb; ++f)
    for (int j = 0; j < m; ++j) {
      const double re = pb.vh[j] * r2 * U[(size_t)f * 2 * m + 2 * j];
      const double im = pb.vh[j] * r2 * U[(size_t)f * 2 * m + 2 * j + 1];
      h[(size_t)f * K + hb.perm[pb.rep[j]]] = zmk(re, im);
      h[(size_t)f * K + hb.perm[pb.neg[j]]] = zmk(re, -im);
    }
  HIPOK(hipMemcpyAsync(wk.rows.p, h.data(), h.size() * sizeof(Z64), hipMemcpyHostToDevice, st));
  const FftGeom g = S->geom();
  launch_xinv(g, wk.rows.as<Z64>(), nullptr, nb, wk.pen.as<Z64>(), st);
  launch_plane_full_inv(g, wk.pen.as<Z64>(), nb, wk.zf.as<Z64>(), st);
  launch_z_real(wk.zf.as<Z64>(), 1.0, wk.dv.as<double>(), (size_t)nb * n3, st);
  CHECKED(launch_check());
  HIPOK(hipStreamSynchronize(st));  // h is released on return
  stern_opts oo = o;
  oo.mem_kind = STERN_MEM_DEVICE;
  oo.n_sample = 0;
  oo.sample_pairs = nullptr;
  oo.sample_x = nullptr;
  oo.profile = 0;
  oo.band_begin = 0;
  oo.band_end = 0;
  stern_stats cst;
  std::memset(&cst, 0, sizeof cst);
  const int rc = stern_apply_chi0(S, nb, wk.dv.as<double>(), wk.dn.as<double>(), &oo, &cst);
  if (rc < 0) return rc;
  if (rc == STERN_WARN_NOT_CONVERGED)
    return fail(STERN_ERR_STATE, "a chi0 apply of the Davidson iteration left %d of %d solves above tol",
                cst.n_solves - cst.n_converged, cst.n_solves);
  solves += cst.n_solves;
  iters += cst.total_iters;
  // dn(G) on the sphere: forward planes of the real field, then the x pass scaled by 1/N^3
  launch_real_to_z(wk.dn.as<double>(), wk.zf.as<Z64>(), (size_t)nb * n3, st);
  launch_plane_full_fwd(g, wk.zf.as<Z64>(), nb, wk.pen.as<Z64>(), st);
  launch_xfwd<double>(g, wk.pen.as<Z64>(), nullptr, nb, wk.rows.as<Z64>(), 2, nullptr, nullptr, 1.0 / (double)n3, st);
  CHECKED(launch_check());
  HIPOK(hipMemcpyAsync(h.data(), wk.rows.p, h.size() * sizeof(Z64), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  const double s2 = std::sqrt(2.0);
  for (int f = 0; f < nb; ++f)
    for (int j = 0; j < m; ++j) {
      const Z64 v = h[(size_t)f * K + hb.perm[pb.rep[j]]];
      W[(size_t)f * 2 * m + 2 * j] = s2 * pb.vh[j] * v.re;
      W[(size_t)f * 2 * m + 2 * j + 1] = s2 * pb.vh[j] * v.im;
    }
  return 0;
}

static double dotv(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

}  // namespace

int stern_pdep_basis(const stern_system* S, double ecut_pot_ry, int* n_g, int32_t* miller) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  PotBasis pb;
  CHECKED(pot_basis(S, ecut_pot_ry > 0 ? ecut_pot_ry : S->hb.ecut / 4.0, pb));
  if (n_g) *n_g = (int)pb.all.size();
  if (miller)
    for (size_t k = 0; k < pb.all.size(); ++k)
      for (int c = 0; c < 3; ++c) miller[3 * k + c] = S->hb.miller[3 * (size_t)pb.all[k] + c];
  return STERN_OK;
}

int stern_pdep_potentials(stern_system* S, int n, const double* vec, double ecut_pot_ry, double* w, int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (n <= 0 || !vec || !w) return fail(STERN_ERR_INVALID_ARG, "need n > 0, vec and w");
  if (mem_kind != STERN_MEM_HOST && mem_kind != STERN_MEM_DEVICE) return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  const HostBasis& hb = S->hb;
  if (!plane_full_fwd_fits(hb.N, S->lds_max))
    return fail(STERN_ERR_UNSUPPORTED, "the potential transforms of grid %d do not fit in LDS", hb.N);
  Scope sc(S->device, &S->alloc);
  PotBasis pb;
  CHECKED(pot_basis(S, ecut_pot_ry > 0 ? ecut_pot_ry : hb.ecut / 4.0, pb));
  const int ng = (int)pb.all.size(), K = hb.npw_pad, N = hb.N;
  const size_t n3 = (size_t)N * N * N;
  std::vector<double> hv((size_t)n * ng * 2);
  if (mem_kind == STERN_MEM_DEVICE)
    HIPOK(hipMemcpy(hv.data(), vec, hv.size() * sizeof(double), hipMemcpyDeviceToHost));
  else
    std::memcpy(hv.data(), vec, hv.size() * sizeof(double));
  // v^{1/2}(G) phi_a(G) on the wave-function sphere (column order), zero elsewhere
  std::vector<Z64> h((size_t)n * K, zmk(0.0, 0.0));
  for (int a = 0; a < n; ++a)
    for (int k = 0; k < ng; ++k) {
      const int c = pb.all[k];
      const double x = hb.miller[3 * (size_t)c], y = hb.miller[3 * (size_t)c + 1], z = hb.miller[3 * (size_t)c + 2];
      const double vh = std::sqrt(4.0 * 3.14159265358979323846) / (hb.b * std::sqrt(x * x + y * y + z * z));
      h[(size_t)a * K + hb.perm[c]] = zmk(vh * hv[2 * ((size_t)a * ng + k)], vh * hv[2 * ((size_t)a * ng + k) + 1]);
    }
  hipStream_t st = S->stream;
  CHECKED(ensure_workspace(S, std::max(S->ws_solves, n)));
  CHECKED(S->tmp_in.ensure((size_t)n * n3 * sizeof(Z64)));
  CHECKED(S->dv_dev.ensure((size_t)n * n3 * sizeof(double)));
  HIPOK(hipMemcpyAsync(S->wp.p, h.data(), h.size() * sizeof(Z64), hipMemcpyHostToDevice, st));
  const FftGeom g = S->geom();
  launch_xinv(g, S->wp.as<Z64>(), nullptr, n, S->pen.as<Z64>(), st);
  launch_plane_full_inv(g, S->pen.as<Z64>(), n, S->tmp_in.as<Z64>(), st);
  launch_z_real(S->tmp_in.as<Z64>(), 1.0, S->dv_dev.as<double>(), (size_t)n * n3, st);
  CHECKED(launch_check());
  HIPOK(hipMemcpyAsync(w, S->dv_dev.p, (size_t)n * n3 * sizeof(double),
                       mem_kind == STERN_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));  // h is released on return
  return STERN_OK;
}

int stern_pdep_davidson(stern_system* S, const stern_pdep_opts* o, double* eig, double* vec, stern_pdep_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!S || !o || !eig || !o->chi0) return fail(STERN_ERR_INVALID_ARG, "need a system, options, chi0 options and eig");
  if (!S->have_occ) return fail(STERN_ERR_STATE, "set_occupied has not been called");
  const int ne = o->n_eig;
  if (ne <= 0) return fail(STERN_ERR_INVALID_ARG, "n_eig must be > 0");
  Scope sc(S->device, &S->alloc);
  size_t lds_max = S->lds_max;
  if (!plane_full_fwd_fits(S->hb.N, lds_max))
    return fail(STERN_ERR_UNSUPPORTED, "the potential transforms of grid %d do not fit in LDS", S->hb.N);
  PotBasis pb;
  CHECKED(pot_basis(S, o->ecut_pot_ry > 0 ? o->ecut_pot_ry : S->hb.ecut / 4.0, pb));
  const int m = (int)pb.rep.size(), dim = 2 * m;
  if (ne > dim) return fail(STERN_ERR_INVALID_ARG, "n_eig %d exceeds the %d potentials of the basis", ne, dim);
  const int nb = std::min(o->block > 0 ? o->block : ne, dim);
  const int max_basis = std::min(dim, std::max(o->max_basis > 0 ? o->max_basis : 4 * ne, ne + nb));
  const int max_iter = o->max_iter > 0 ? o->max_iter : 50;
  const double tol = o->tol > 0 ? o->tol : 1e-6;
  PdepWork wk;
  long long solves = 0, cg_iters = 0;
  int calls = 0;
  std::vector<std::vector<double>> V, W;  // orthonormal basis and chi-bar0 of it
  // orthonormalise x against V (twice) and normalise; false when nothing is left
  auto orth = [&](std::vector<double>& x) -> bool {
    const double n0 = std::sqrt(dotv(x.data(), x.data(), dim));
    if (!(n0 > 0)) return false;
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& v : V) {
        const double c = dotv(v.data(), x.data(), dim);
        for (int i = 0; i < dim; ++i) x[i] -= c * v[i];
      }
    const double n1 = std::sqrt(dotv(x.data(), x.data(), dim));
    if (!(n1 > 1e-10 * n0)) return false;
    for (double& e : x) e /= n1;
    return true;
  };
  auto expand = [&](std::vector<std::vector<double>>& block) -> int {
    std::vector<std::vector<double>> keep;
    for (auto& x : block)
      if (orth(x)) {
        V.push_back(x);
        keep.push_back(x);
      }
    const int n = (int)keep.size();
    if (n == 0) return 0;
    std::vector<double> U((size_t)n * dim), R((size_t)n * dim);
    for (int f = 0; f < n; ++f) std::copy(keep[f].begin(), keep[f].end(), U.begin() + (size_t)f * dim);
    const int rc = pdep_apply(S, pb, *o->chi0, U.data(), n, R.data(), wk, solves, cg_iters);
    if (rc < 0) return rc;
    ++calls;
    for (int f = 0; f < n; ++f) W.emplace_back(R.begin() + (size_t)f * dim, R.begin() + (size_t)(f + 1) * dim);
    return n;
  };
  int rc = 0;
  {  // seeded random start
    std::mt19937_64 rng(o->seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<std::vector<double>> block(nb, std::vector<double>(dim));
    for (auto& x : block)
      for (double& e : x) e = nd(rng);
    rc = expand(block);
  }
  std::vector<double> theta, Y, res(ne, 0.0);
  std::vector<std::vector<double>> X(ne), AX(ne);
  int it = 0, nconv = 0;
  for (; rc >= 0 && it < max_iter; ++it) {
    const int k = (int)V.size();
    std::vector<double> Hs((size_t)k * k);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j <= i; ++j) {
        const double h = 0.5 * (dotv(V[i].data(), W[j].data(), dim) + dotv(V[j].data(), W[i].data(), dim));
        Hs[(size_t)i * k + j] = Hs[(size_t)j * k + i] = h;
      }
    jacobi_eigh(Hs, k, theta, Y);
    const int nr = std::min(k, max_basis);  // Ritz pairs kept on a restart
    std::vector<std::vector<double>> XR(std::min(k, std::max(ne, nr))), AXR(XR.size());
    for (size_t a = 0; a < XR.size(); ++a) {
      XR[a].assign(dim, 0.0);
      AXR[a].assign(dim, 0.0);
      for (int i = 0; i < k; ++i) {
        const double y = Y[(size_t)i * k + a];
        for (int d = 0; d < dim; ++d) {
          XR[a][d] += y * V[i][d];
          AXR[a][d] += y * W[i][d];
        }
      }
    }
    // residuals of the wanted pairs; unconverged ones give the next block
    std::vector<std::vector<double>> block;
    nconv = 0;
    for (int a = 0; a < std::min(ne, k); ++a) {
      std::vector<double> r(dim);
      for (int d = 0; d < dim; ++d) r[d] = AXR[a][d] - theta[a] * XR[a][d];
      res[a] = std::sqrt(dotv(r.data(), r.data(), dim));
      if (res[a] <= tol * std::fabs(theta[a])) {
        ++nconv;  // converged pairs add no directions (they stay in the basis, deflated)
      } else if ((int)block.size() < nb) {
        block.push_back(r);
      }
    }
    if (nconv == ne && k >= ne) {
      for (int a = 0; a < ne; ++a) {
        X[a] = XR[a];
        AX[a] = AXR[a];
      }
      break;
    }
    if (k + (int)block.size() > max_basis) {  // restart from the Ritz vectors
      const int keep = std::max(ne, max_basis - nb);
      V.assign(XR.begin(), XR.begin() + std::min<size_t>(keep, XR.size()));
      W.assign(AXR.begin(), AXR.begin() + std::min<size_t>(keep, AXR.size()));
    }
    for (int a = 0; a < ne; ++a) {
      X[a] = a < (int)XR.size() ? XR[a] : std::vector<double>(dim, 0.0);
    }
    rc = expand(block);
    if (rc == 0 && nconv < ne) {  // no new direction survived: the basis is exhausted
      rc = 0;
      break;
    }
  }
  wk.release();
  if (rc < 0) return rc;
  for (int a = 0; a < ne; ++a) eig[a] = a < (int)theta.size() ? theta[a] : 0.0;
  if (vec) {  // complex coefficients over the whole potential sphere, canonical order
    const size_t ng = pb.all.size();
    std::vector<int> pos_of(S->hb.npw, -1);
    for (size_t q = 0; q < ng; ++q) pos_of[pb.all[q]] = (int)q;
    const double r2 = 1.0 / std::sqrt(2.0);
    for (int a = 0; a < ne; ++a) {
      double* out = vec + 2 * (size_t)a * ng;
      std::fill(out, out + 2 * ng, 0.0);
      for (int j = 0; j < m; ++j) {
        const double re = r2 * X[a][2 * j], im = r2 * X[a][2 * j + 1];
        const int p = pos_of[pb.rep[j]], q = pos_of[pb.neg[j]];
        out[2 * p] = re;
        out[2 * p + 1] = im;
        out[2 * q] = re;
        out[2 * q + 1] = -im;
      }
    }
  }
  if (stats) {
    stats->iterations = it + 1;
    stats->n_converged = nconv;
    stats->chi0_calls = calls;
    stats->total_solves = solves;
    stats->total_cg_iters = cg_iters;
    stats->basis_dim = dim;
    double mr = 0.0;
    for (int a = 0; a < ne; ++a) mr = std::max(mr, res[a] / std::max(std::fabs(eig[a]), 1e-300));
    stats->max_rel_resid = mr;
    stats->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return nconv == ne ? STERN_OK : STERN_WARN_NOT_CONVERGED;
}

// ------------------------------------------------------------- autotuner ----

const char* stern_autotune_report(void) { return g_tune_report.c_str(); }

int stern_tunable(stern_system* S, int which, int value) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  int* slot = nullptr;
  switch (which) {
    case STERN_TUNE_PLANE64: slot = &S->plane_var64; break;
    case STERN_TUNE_PLANE32: slot = &S->plane_var32; break;
    case STERN_TUNE_GEMM64_WG: slot = &S->gemm64_wg; break;
    case STERN_TUNE_GEMM16_WG: slot = &S->gemm16_wg; break;
    case STERN_TUNE_GEMM16_EXPAND: slot = &S->gemm16_expand; break;
    default: return fail(STERN_ERR_INVALID_ARG, "unknown tunable %d", which);
  }
  if (value >= 0) {
    if (which == STERN_TUNE_GEMM16_EXPAND) {
      if (value > 2) return fail(STERN_ERR_INVALID_ARG, "expand variant must be 0, 1 or 2");
    } else if (which == STERN_TUNE_PLANE64 || which == STERN_TUNE_PLANE32) {
      if (value > 2) return fail(STERN_ERR_INVALID_ARG, "plane kernel variant must be 0, 1 or 2");
      const bool fp64 = which == STERN_TUNE_PLANE64;
      if (value >= 1 && plane_hw_lds(S->hb.N, S->hb.nza, fp64) > S->lds_max)
        return fail(STERN_ERR_INVALID_ARG, "the compact plane kernel does not fit in LDS for grid %d", S->hb.N);
      if (value == 0 && plane_lds_bytes(S->hb.N, fp64 ? sizeof(Z64) : sizeof(Z32)) > S->lds_max)
        return fail(STERN_ERR_INVALID_ARG, "the full-plane kernel does not fit in LDS for grid %d", S->hb.N);
    } else if (value > 65536) {
      return fail(STERN_ERR_INVALID_ARG, "workgroup target %d out of range", value);
    }
    *slot = value;
  }
  return *slot;
}

int stern_autotune(stern_system* S, int n_vec, const char* cache_path, int* chosen) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!S->have_occ) return fail(STERN_ERR_STATE, "set_occupied has not been called");
  if (n_vec <= 0 || n_vec > 65536) return fail(STERN_ERR_INVALID_ARG, "n_vec must be in [1, 65536]");
  Scope sc(S->device, &S->alloc);
  hipStream_t st = S->stream;
  S->prof_on = false;
  S->recs.clear();
  S->ev_used = 0;
  hipDeviceProp_t prop;
  HIPOK(hipGetDeviceProperties(&prop, S->device));
  char key[512];
  std::snprintf(key, sizeof key, "%s N=%d nza=%d npw=%d nocc_pad=%d natoms_pad=%d nvec=%d", prop.gcnArchName,
                S->hb.N, S->hb.nza, S->hb.npw, S->nocc_pad, S->natoms_pad, n_vec);
  int* slots[STERN_NTUNE] = {&S->plane_var64, &S->plane_var32, &S->gemm64_wg, &S->gemm16_wg, &S->gemm16_expand};
  // cached choices
  if (cache_path) {
    std::FILE* f = std::fopen(cache_path, "r");
    int found[STERN_NTUNE];
    for (int w = 0; w < STERN_NTUNE; ++w) found[w] = -1;
    if (f) {
      char line[768];
      const size_t kl = std::strlen(key);
      while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, key, kl) != 0 || line[kl] != ' ') continue;
        int w = -1, v = -1;
        if (std::sscanf(line + kl, " tune=%d value=%d", &w, &v) == 2 && w >= 0 && w < STERN_NTUNE) found[w] = v;
      }
      std::fclose(f);
    }
    bool all = true;
    for (int w = 0; w < STERN_NTUNE; ++w) all = all && found[w] >= 0;
    if (all) {
      for (int w = 0; w < STERN_NTUNE; ++w) CHECKED(stern_tunable(S, w, found[w]));
      if (chosen)
        for (int w = 0; w < STERN_NTUNE; ++w) chosen[w] = *slots[w];
      return 0;
    }
  }
  // synthetic rows: seeded complex values on the sphere, zero padding; eps of bands 0, 1, ...
  const int K = S->hb.npw_pad, npw = S->hb.npw;
  CHECKED(ensure_workspace(S, n_vec));
  CHECKED(ensure_workspace32(S, n_vec));
  {
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<Z64> h((size_t)n_vec * K, zmk(0.0, 0.0));
    std::vector<double> e(n_vec);
    for (int v = 0; v < n_vec; ++v) {
      for (int k = 0; k < npw; ++k) h[(size_t)v * K + k] = zmk(nd(rng), nd(rng));
      e[v] = S->eps[v % S->n_occ];
    }
    HIPOK(hipMemcpyAsync(S->wp.p, h.data(), h.size() * sizeof(Z64), hipMemcpyHostToDevice, st));
    HIPOK(hipMemcpyAsync(S->sv_eps.p, e.data(), n_vec * sizeof(double), hipMemcpyHostToDevice, st));
    launch_to32(S->wp.as<Z64>(), S->m_p.as<Z32>(), h.size(), st);
    HIPOK(hipStreamSynchronize(st));  // h and e are released at the end of this block
  }
  const double* eps = S->sv_eps.as<double>();
  const int reps = 3;
  int n_timed = 0;
  static const char* names[STERN_NTUNE] = {"plane64", "plane32", "gemm64_wg", "gemm16_wg", "gemm16_expand"};
  std::string report = "{";
  auto tune = [&](int which, const std::vector<int>& cand, auto&& fn) -> int {
    double best = 1e300;
    int bestv = *slots[which];
    report += std::string(which ? ", \"" : "\"") + names[which] + "\": {";
    bool first = true;
    for (int v : cand) {
      if (stern_tunable(S, which, v) < 0) continue;  // not runnable here
      CHECKED(ensure_workspace(S, n_vec));             // split-K partials for this target
      double ms = 0.0;
      CHECKED(time_ms(S, reps, ms, fn));
      ++n_timed;
      char item[64];
      std::snprintf(item, sizeof item, "%s\"%d\": %.4f", first ? "" : ", ", v, ms);
      report += item;
      first = false;
      if (ms < best) {
        best = ms;
        bestv = v;
      }
    }
    report += "}";
    CHECKED(stern_tunable(S, which, bestv));
    return 0;
  };
  CHECKED(tune(STERN_TUNE_PLANE64, {0, 1, 2},
               [&] { return apply_h_rows(S, S->wp.as<Z64>(), S->wq.as<Z64>(), nullptr, n_vec, eps); }));
  CHECKED(tune(STERN_TUNE_PLANE32, {0, 1, 2},
               [&] { return apply_h32_rows(S, S->m_p.as<Z32>(), S->m_q.as<Z32>(), nullptr, n_vec, eps); }));
  CHECKED(tune(STERN_TUNE_GEMM64_WG, {256, 384, 512, 768, 1024, 2048, 4096},
               [&] { return apply_pc_rows(S, S->wq.as<Z64>(), nullptr, n_vec); }));
  CHECKED(tune(STERN_TUNE_GEMM16_WG, {128, 192, 256, 384, 512, 1024, 2048},
               [&] { return apply_pc32_rows(S, S->m_q.as<Z32>(), nullptr, n_vec); }));
  CHECKED(tune(STERN_TUNE_GEMM16_EXPAND, {0, 1, 2},
               [&] { return apply_pc32_rows(S, S->m_q.as<Z32>(), nullptr, n_vec); }));
  CHECKED(ensure_workspace(S, n_vec));
  g_tune_report = report + "}";
  if (chosen)
    for (int w = 0; w < STERN_NTUNE; ++w) chosen[w] = *slots[w];
  if (cache_path) {
    std::FILE* f = std::fopen(cache_path, "a");
    if (f) {
      for (int w = 0; w < STERN_NTUNE; ++w) std::fprintf(f, "%s tune=%d value=%d\n", key, w, *slots[w]);
      std::fclose(f);
    }
  }
  return n_timed;
}

// ---------------------------------------------------------- learned model ----

int stern_model_num_params(void) { return kNetLayers * kNetLayerParams + kPrecParams; }

static int model_refresh_bf16(stern_model* M, hipStream_t st) {
  for (int l = 0; l < kNetLayers; ++l)
    launch_f32_to_bf16(M->w.as<float>() + (size_t)l * stern_model::LP, M->wbf.as<__bf16>() + (size_t)l * stern_model::WN,
                       stern_model::WN, st);
  return launch_check();
}

int stern_model_create(int device, unsigned long long seed, stern_model** out) {
  if (!out) return fail(STERN_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  Scope sc(device);
  stern_model* M = new stern_model();
  M->device = device;
  const int np = stern_model_num_params();
  auto run = [&]() -> int {
    CHECKED(M->w.ensure(np * sizeof(float)));
    CHECKED(M->m.ensure(np * sizeof(float)));
    CHECKED(M->v.ensure(np * sizeof(float)));
    CHECKED(M->grad.ensure(np * sizeof(float)));
    CHECKED(M->wbf.ensure((size_t)kNetLayers * stern_model::WN * sizeof(__bf16)));
    CHECKED(M->wtf.ensure((size_t)stern_model::WN * sizeof(__bf16)));
    // He-normal weights for the ReLU layers (fan-in 27 x 5 input channels for the
    // first layer, 27 x 16 after), a small output layer, zero biases
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    std::vector<float> w(np, 0.f), z(np, 0.f);
    for (int l = 0; l < kNetLayers; ++l) {
      const float sd = l == 0 ? std::sqrt(2.f / (27.f * 5.f)) : (l == 1 ? std::sqrt(2.f / (27.f * 16.f)) : 1e-3f);
      for (int co = 0; co < kNetChannels; ++co)
        for (int n = 0; n < 27; ++n)
          for (int ci = 0; ci < kNetChannels; ++ci) {
            const bool live = (l == 0 ? ci < 5 : true) && (l == 2 ? co < 2 : true);
            w[(size_t)l * stern_model::LP + ((size_t)co * 27 + n) * kNetChannels + ci] = live ? sd * nd(rng) : 0.f;
          }
    }
    HIPOK(hipMemcpy(M->w.p, w.data(), np * sizeof(float), hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(M->m.p, z.data(), np * sizeof(float), hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(M->v.p, z.data(), np * sizeof(float), hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(M->grad.p, z.data(), np * sizeof(float), hipMemcpyHostToDevice));
    CHECKED(model_refresh_bf16(M, nullptr));
    HIPOK(hipDeviceSynchronize());
    return 0;
  };
  const int rc = run();
  if (rc < 0) {
    M->release_all();
    delete M;
    return rc;
  }
  *out = M;
  return STERN_OK;
}

int stern_model_get_weights(const stern_model* M, float* w, int n) {
  if (!M || !w || n != stern_model_num_params()) return fail(STERN_ERR_INVALID_ARG, "bad model or size");
  Scope sc(M->device);
  HIPOK(hipMemcpy(w, M->w.p, n * sizeof(float), hipMemcpyDeviceToHost));
  return n;
}

int stern_model_set_weights(stern_model* M, const float* w, int n) {
  if (!M || !w || n != stern_model_num_params()) return fail(STERN_ERR_INVALID_ARG, "bad model or size");
  Scope sc(M->device);
  HIPOK(hipMemcpy(M->w.p, w, n * sizeof(float), hipMemcpyHostToDevice));
  CHECKED(model_refresh_bf16(M, nullptr));
  HIPOK(hipDeviceSynchronize());
  M->trained = true;
  M->prec_trained = false;
  for (int k = stern_model::HEAD; k < n; ++k) M->prec_trained = M->prec_trained || w[k] != 0.f;
  return n;
}

void stern_model_free(stern_model* M) {
  if (!M) return;
  {
    Scope sc(M->device);
    (void)hipDeviceSynchronize();
    M->release_all();
  }
  delete M;
}

// One Adam step of the net on the nb solves staged in M->a0 (inputs) and M->tgt
// (targets): forward, relative-L2 loss (per-solve values in M->loss, dL/dout in
// M->g3), backward through the three layers (weight gradients summed over the
// solves into M->grad, data gradients by the flipped-weight convolution, ReLU
// masks from the stored BF16 activations), then Adam on the conv weights with
// the gradient averaged over the solves. The preconditioner head is untouched.
static int net_fit_step(stern_model* M, int Nc, int nb_, float lr, hipStream_t st) {
  const size_t ldp = (size_t)net_ldp(Nc), C = kNetChannels;
  const int np_layer = stern_model::LP;
  net_forward(M, M->a0.as<__bf16>(), M->a1.as<__bf16>(), M->a2.as<__bf16>(), M->out.as<float>(), Nc, nb_, st);
  launch_loss(M->out.as<float>(), M->tgt.as<float>(), M->g3.as<float>(), M->loss.as<float>(), Nc, nb_, st);
  const size_t nact = (size_t)nb_ * ldp * C;
  float* gw = M->grad.as<float>();
  // layer 3 (index 2)
  launch_conv3_wgrad(M->a2.as<__bf16>(), M->g3.as<float>(), M->part.as<float>(), gw + 2 * np_layer, Nc, nb_, st);
  launch_flip_weights(M->w.as<float>() + 2 * np_layer, M->wtf.as<__bf16>(), st);
  launch_f32_to_bf16(M->g3.as<float>(), M->gbf.as<__bf16>(), nact, st);
  launch_conv3(M->gbf.as<__bf16>(), M->wtf.as<__bf16>(), nullptr, M->g2.as<float>(), Nc, nb_, 0, true, st);
  launch_relu_bwd(M->g2.as<float>(), M->a2.as<__bf16>(), nact, st);
  // layer 2 (index 1)
  launch_conv3_wgrad(M->a1.as<__bf16>(), M->g2.as<float>(), M->part.as<float>(), gw + 1 * np_layer, Nc, nb_, st);
  launch_flip_weights(M->w.as<float>() + 1 * np_layer, M->wtf.as<__bf16>(), st);
  launch_f32_to_bf16(M->g2.as<float>(), M->gbf.as<__bf16>(), nact, st);
  launch_conv3(M->gbf.as<__bf16>(), M->wtf.as<__bf16>(), nullptr, M->g3.as<float>(), Nc, nb_, 0, true, st);
  launch_relu_bwd(M->g3.as<float>(), M->a1.as<__bf16>(), nact, st);
  // layer 1 (index 0)
  launch_conv3_wgrad(M->a0.as<__bf16>(), M->g3.as<float>(), M->part.as<float>(), gw, Nc, nb_, st);
  ++M->step;  // the trunk only: the head's gradient is not formed here
  launch_adam(M->w.as<float>(), M->m.as<float>(), M->v.as<float>(), gw, stern_model::HEAD, lr, M->step,
              1.f / (float)nb_, st);
  return model_refresh_bf16(M, st);
}

// training workspace of mini-batches of B solves on an Nc^3 coarse grid
static int net_train_workspace(stern_model* M, int Nc, int B) {
  const size_t ldp = (size_t)net_ldp(Nc), C = kNetChannels;
  CHECKED(M->a0.ensure((size_t)B * ldp * C * sizeof(__bf16)));
  CHECKED(M->a1.ensure((size_t)B * ldp * C * sizeof(__bf16)));
  CHECKED(M->a2.ensure((size_t)B * ldp * C * sizeof(__bf16)));
  CHECKED(M->gbf.ensure((size_t)B * ldp * C * sizeof(__bf16)));
  for (DBuf* d : {&M->out, &M->g3, &M->g2}) CHECKED(d->ensure((size_t)B * ldp * C * sizeof(float)));
  CHECKED(M->tgt.ensure((size_t)B * ldp * 2 * sizeof(float)));
  CHECKED(M->loss.ensure((size_t)B * sizeof(float)));
  CHECKED(M->part.ensure((size_t)conv3_wgrad_parts(Nc) * stern_model::LP * sizeof(float)));
  return 0;
}

int stern_model_fit_step(stern_model* M, int Nc, int n, const float* in, const float* target, double lr,
                         float* out, float* loss, float* grad) {
  if (!M || !in || !target || n <= 0 || Nc < 4 || !(lr >= 0))
    return fail(STERN_ERR_INVALID_ARG, "need a model, n > 0, Nc >= 4, lr >= 0, inputs and targets");
  Scope sc(M->device);
  const size_t P = (size_t)Nc * Nc * Nc, ldp = (size_t)net_ldp(Nc), C = kNetChannels;
  CHECKED(net_train_workspace(M, Nc, n));
  // channels-last staging: inputs [n][ldp][16] (5 live channels), targets [n][ldp][2]
  std::vector<float> a((size_t)n * ldp * C, 0.f), t((size_t)n * ldp * 2, 0.f);
  for (size_t s = 0; s < (size_t)n; ++s)
    for (size_t p = 0; p < P; ++p) {
      for (int c = 0; c < kNetInputs; ++c) a[(s * ldp + p) * C + c] = in[(s * P + p) * kNetInputs + c];
      for (int c = 0; c < 2; ++c) t[(s * ldp + p) * 2 + c] = target[(s * P + p) * 2 + c];
    }
  CHECKED(M->g2.ensure(a.size() * sizeof(float)));
  hipStream_t st = nullptr;
  HIPOK(hipMemcpyAsync(M->g2.p, a.data(), a.size() * sizeof(float), hipMemcpyHostToDevice, st));
  launch_f32_to_bf16(M->g2.as<float>(), M->a0.as<__bf16>(), a.size(), st);
  HIPOK(hipMemcpyAsync(M->tgt.p, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice, st));
  CHECKED(net_fit_step(M, Nc, n, (float)lr, st));
  CHECKED(launch_check());
  if (loss) HIPOK(hipMemcpyAsync(loss, M->loss.p, n * sizeof(float), hipMemcpyDeviceToHost, st));
  if (grad) HIPOK(hipMemcpyAsync(grad, M->grad.p, stern_model::HEAD * sizeof(float), hipMemcpyDeviceToHost, st));
  if (out) {
    std::vector<float> o((size_t)n * ldp * C);
    HIPOK(hipMemcpyAsync(o.data(), M->out.p, o.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    for (size_t s = 0; s < (size_t)n; ++s)
      for (size_t p = 0; p < P; ++p)
        for (int c = 0; c < 2; ++c) out[(s * P + p) * 2 + c] = o[(s * ldp + p) * C + c];
  }
  HIPOK(hipStreamSynchronize(st));
  M->trained = true;
  return STERN_OK;
}

int stern_model_train(stern_model* M, int n_sys, stern_system* const* sys, const int* n_pert, const double* const* dv_r,
                      int mem_kind, const stern_train_opts* o, stern_train_stats* tstats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!M || n_sys <= 0 || !sys || !n_pert || !dv_r) return fail(STERN_ERR_INVALID_ARG, "bad arguments");
  if (mem_kind != STERN_MEM_HOST && mem_kind != STERN_MEM_DEVICE) return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  const int epochs = (o && o->epochs > 0) ? o->epochs : 4;
  const int B = (o && o->batch > 0) ? o->batch : 16;
  const float lr = (float)((o && o->lr > 0) ? o->lr : 1e-3);
  const int max_solves = (o && o->max_solves > 0) ? o->max_solves : 4096;
  const double tol = (o && o->tol > 0) ? o->tol : 1e-8;
  std::mt19937_64 rng(o ? o->seed : 0);
  int Nc = -1;
  long long total = 0;
  for (int k = 0; k < n_sys; ++k) {
    if (!sys[k] || !sys[k]->have_occ) return fail(STERN_ERR_STATE, "system %d is not ready", k);
    if (!sys[k]->have_coarse) return fail(STERN_ERR_UNSUPPORTED, "system %d has no coarse grid", k);
    if (sys[k]->device != M->device) return fail(STERN_ERR_INVALID_ARG, "system %d on another device", k);
    if (Nc < 0) Nc = sys[k]->hbc.N;
    if (sys[k]->hbc.N != Nc) return fail(STERN_ERR_INVALID_ARG, "training systems need the same coarse grid");
    if (n_pert[k] <= 0 || !dv_r[k]) return fail(STERN_ERR_INVALID_ARG, "system %d has no fields", k);
    total += (long long)n_pert[k] * sys[k]->n_occ;
  }
  for (int k = 0; k < n_sys; ++k) {  // no event profile during training
    sys[k]->prof_on = false;
    sys[k]->recs.clear();
    sys[k]->ev_used = 0;
  }
  Scope sc(M->device);
  const size_t ldp = (size_t)net_ldp(Nc), C = kNetChannels;
  const int nsamp_max = (int)std::min<long long>(total, max_solves);
  // which solves (global index) become training samples
  std::vector<long long> pick(total);
  std::iota(pick.begin(), pick.end(), 0LL);
  std::shuffle(pick.begin(), pick.end(), rng);
  std::vector<char> chosen(total, 0);
  for (int k = 0; k < nsamp_max; ++k) chosen[pick[k]] = 1;
  CHECKED(M->din.ensure((size_t)nsamp_max * ldp * C * sizeof(__bf16)));
  CHECKED(M->dtgt.ensure((size_t)nsamp_max * ldp * 2 * sizeof(float)));
  int nsamp = 0;
  long long base = 0;
  // ---- dataset: plain FP64 solutions of every system ----
  for (int k = 0; k < n_sys; ++k) {
    stern_system* S = sys[k];
    Scope ssc(S->device, &S->alloc);
    hipStream_t st = S->stream;
    const HostBasis& hb = S->hb;
    const size_t n3 = (size_t)hb.N * hb.N * hb.N;
    const int nb = S->n_occ;
    const double* dv_dev = dv_r[k];
    if (mem_kind == STERN_MEM_HOST) {
      CHECKED(S->dv_dev.ensure((size_t)n_pert[k] * n3 * sizeof(double)));
      HIPOK(hipMemcpyAsync(S->dv_dev.p, dv_r[k], (size_t)n_pert[k] * n3 * sizeof(double), hipMemcpyHostToDevice, st));
      dv_dev = S->dv_dev.as<double>();
    }
    size_t free_b = 0, total_b = 0;
    HIPOK(hipMemGetInfo(&free_b, &total_b));
    const size_t per_solve = (size_t)hb.npw_pad * sizeof(Z64) * 6 + (size_t)hb.N * hb.ncol_pad * sizeof(Z64) +
                             net_bytes_per_solve(S) + 1024;
    int per = (int)std::max<size_t>(1, (size_t)(0.4 * (double)free_b) / (per_solve * nb));
    per = std::min(per, n_pert[k]);
    CHECKED(ensure_workspace(S, per * nb));
    const CgState cs = cg_state(S);
    const double vecb = (double)hb.npw * sizeof(Z64);
    int n_restart = 0;
    const int chunk = std::min(per * nb, 512);
    CHECKED(S->c_pen.ensure((size_t)chunk * Nc * S->hbc.ncol_pad * sizeof(Z64)));
    CHECKED(S->c_field.ensure((size_t)chunk * Nc * Nc * Nc * sizeof(Z64)));
    CHECKED(S->net_a0.ensure((size_t)chunk * ldp * C * sizeof(__bf16)));
    CHECKED(S->net_out.ensure((size_t)chunk * ldp * C * sizeof(float)));
    for (int i0 = 0; i0 < n_pert[k]; i0 += per) {
      const int i1 = std::min(n_pert[k], i0 + per);
      const int ns = (i1 - i0) * nb;
      CHECKED(setup_batch(S, i0, i1, 0, nb, dv_dev, vecb));
      std::vector<int> all(ns);
      std::iota(all.begin(), all.end(), 0);
      CHECKED(run_pcg64(S, cs, all, tol, 1000, 1, n_restart, vecb, false));
      for (int s0 = 0; s0 < ns; s0 += chunk) {
        const int c = std::min(chunk, ns - s0);
        CHECKED(net_input(S, cs, s0, c, S->net_a0.as<__bf16>()));
        CHECKED(coarse_fields(S, cs.x, s0, c));
        launch_pack_target(S->c_field.as<Z64>(), cs.bb + s0, S->net_out.as<float>(), Nc, c, st);
        for (int t = 0; t < c; ++t) {
          if (!chosen[base + (long long)i0 * nb + s0 + t]) continue;
          HIPOK(hipMemcpyAsync(M->din.as<__bf16>() + (size_t)nsamp * ldp * C,
                               S->net_a0.as<__bf16>() + (size_t)t * ldp * C, ldp * C * sizeof(__bf16),
                               hipMemcpyDeviceToDevice, st));
          HIPOK(hipMemcpyAsync(M->dtgt.as<float>() + (size_t)nsamp * ldp * 2,
                               S->net_out.as<float>() + (size_t)t * ldp * 2, ldp * 2 * sizeof(float),
                               hipMemcpyDeviceToDevice, st));
          ++nsamp;
        }
      }
      CHECKED(launch_check());
      HIPOK(hipStreamSynchronize(st));
    }
    base += (long long)n_pert[k] * nb;
  }
  // ---- training: Adam on mini-batches of B solves ----
  hipStream_t st = sys[0]->stream;
  CHECKED(net_train_workspace(M, Nc, B));
  std::vector<int> order(nsamp);
  std::iota(order.begin(), order.end(), 0);
  std::vector<float> hl(B);
  double first = 0.0, last = 0.0;
  int steps = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    std::shuffle(order.begin(), order.end(), rng);
    double ep_loss = 0.0;
    int ep_n = 0;
    for (int b0 = 0; b0 + B <= std::max(nsamp, B) && b0 < nsamp; b0 += B) {
      const int nb_ = std::min(B, nsamp - b0);
      for (int t = 0; t < nb_; ++t) {
        const int id = order[b0 + t];
        HIPOK(hipMemcpyAsync(M->a0.as<__bf16>() + (size_t)t * ldp * C, M->din.as<__bf16>() + (size_t)id * ldp * C,
                             ldp * C * sizeof(__bf16), hipMemcpyDeviceToDevice, st));
        HIPOK(hipMemcpyAsync(M->tgt.as<float>() + (size_t)t * ldp * 2, M->dtgt.as<float>() + (size_t)id * ldp * 2,
                             ldp * 2 * sizeof(float), hipMemcpyDeviceToDevice, st));
      }
      CHECKED(net_fit_step(M, Nc, nb_, lr, st));
      HIPOK(hipMemcpyAsync(hl.data(), M->loss.p, nb_ * sizeof(float), hipMemcpyDeviceToHost, st));
      HIPOK(hipStreamSynchronize(st));
      for (int t = 0; t < nb_; ++t) ep_loss += hl[t];
      ep_n += nb_;
      ++steps;
    }
    const double mean = ep_n ? ep_loss / ep_n : 0.0;
    if (ep == 0) first = mean;
    last = mean;
  }
  M->trained = true;
  // ---- preconditioner head: r0, e0 and features from the trained guess ----
  const int prec_epochs = (o && o->prec_epochs != 0) ? o->prec_epochs : 4;
  const float prec_lr = (float)((o && o->prec_lr > 0) ? o->prec_lr : 1e-2);
  const int prec_cap = (o && o->prec_max_solves > 0) ? o->prec_max_solves : 1024;
  int nprec = 0;
  double pfirst = 0.0, plast = 0.0;
  if (prec_epochs > 0) {
    M->prec_trained = false;
    // per system: its sample rows in the shared r0 / e0 / feature sets
    std::vector<int> sys_begin(n_sys + 1, 0);
    std::vector<size_t> sys_off(n_sys + 1, 0);  // element offset of system k's rows (stride npw_pad of k)
    std::vector<std::vector<char>> pick2(n_sys);
    long long gbase = 0;
    int ld_max = 0;
    for (int k = 0; k < n_sys; ++k) ld_max = std::max(ld_max, sys[k]->hb.npw_pad);
    {
      std::vector<long long> ids(total);
      std::iota(ids.begin(), ids.end(), 0LL);
      std::shuffle(ids.begin(), ids.end(), rng);
      std::vector<char> ch(total, 0);
      for (long long k = 0; k < std::min<long long>(total, prec_cap); ++k) ch[ids[k]] = 1;
      for (int k = 0; k < n_sys; ++k) {
        const long long n = (long long)n_pert[k] * sys[k]->n_occ;
        pick2[k].assign(ch.begin() + gbase, ch.begin() + gbase + n);
        gbase += n;
      }
    }
    const int ncap = (int)std::min<long long>(total, prec_cap);
    CHECKED(M->r0set.ensure((size_t)ncap * ld_max * sizeof(Z64)));
    CHECKED(M->e0set.ensure((size_t)ncap * ld_max * sizeof(Z64)));
    CHECKED(M->fset.ensure((size_t)ncap * kPrecIn * sizeof(float)));
    for (int k = 0; k < n_sys; ++k) {
      stern_system* S = sys[k];
      Scope ssc(S->device, &S->alloc);
      hipStream_t st2 = S->stream;
      const HostBasis& hb = S->hb;
      const int nb = S->n_occ, K = hb.npw_pad;
      const size_t n3 = (size_t)hb.N * hb.N * hb.N;
      const double* dv_dev = mem_kind == STERN_MEM_HOST ? S->dv_dev.as<double>() : dv_r[k];
      if (mem_kind == STERN_MEM_HOST) {  // the dataset pass above may have used another system's upload
        CHECKED(S->dv_dev.ensure((size_t)n_pert[k] * n3 * sizeof(double)));
        HIPOK(hipMemcpyAsync(S->dv_dev.p, dv_r[k], (size_t)n_pert[k] * n3 * sizeof(double), hipMemcpyHostToDevice,
                             st2));
        dv_dev = S->dv_dev.as<double>();
      }
      const double vecb = (double)hb.npw * sizeof(Z64);
      const int per = std::max(1, std::min(n_pert[k], S->ws_solves / nb));
      CgState cs = cg_state(S);
      sys_begin[k] = nprec;
      if (k > 0) sys_off[k] = sys_off[k - 1] + (size_t)(sys_begin[k] - sys_begin[k - 1]) * sys[k - 1]->hb.npw_pad;
      int n_restart = 0, n_rej = 0;
      for (int i0 = 0; i0 < n_pert[k]; i0 += per) {
        const int i1 = std::min(n_pert[k], i0 + per);
        const int ns = (i1 - i0) * nb;
        std::vector<int> rows, slots;
        for (int s = 0; s < ns; ++s)
          if (pick2[k][(size_t)i0 * nb + s]) {
            rows.push_back(s);
            slots.push_back(nprec + (int)rows.size() - 1);
          }
        if (rows.empty()) continue;
        CHECKED(setup_batch(S, i0, i1, 0, nb, dv_dev, vecb));
        CHECKED(learned_guess(S, M, cs, ns, n_rej, false, true, true));  // x0, r0, features; K still Teter
        const int nr = (int)rows.size();
        CHECKED(M->idx.ensure((size_t)nr * sizeof(int)));
        HIPOK(hipMemcpyAsync(M->idx.p, rows.data(), nr * sizeof(int), hipMemcpyHostToDevice, st2));
        const size_t off = sys_off[k] + (size_t)(nprec - sys_begin[k]) * K;
        Z64* R0 = M->r0set.as<Z64>() + off;
        Z64* E0 = M->e0set.as<Z64>() + off;
        launch_gather_rows(R0, cs.r, M->idx.as<int>(), K, nr, false, st2);
        launch_gather_rows(E0, cs.x, M->idx.as<int>(), K, nr, false, st2);
        launch_gather_f32(M->fset.as<float>() + (size_t)nprec * kPrecIn, S->net_feat.as<float>(), M->idx.as<int>(),
                          kPrecIn, nr, st2);
        std::vector<int> all(ns);
        std::iota(all.begin(), all.end(), 0);
        CHECKED(run_pcg64(S, cs, all, tol, 1000, 1, n_restart, vecb, false, true));
        launch_gather_rows(E0, cs.x, M->idx.as<int>(), K, nr, true, st2);  // e0 = x* - x0
        CHECKED(launch_check());
        HIPOK(hipStreamSynchronize(st2));
        nprec += nr;
      }
    }
    sys_begin[n_sys] = nprec;
    // Adam on the head, mini-batches within one system (they share its P_c)
    const int Bp = B;
    CHECKED(M->fb.ensure((size_t)Bp * kPrecIn * sizeof(float)));
    CHECKED(M->coef.ensure((size_t)Bp * kPrecKnots * sizeof(float)));
    CHECKED(M->gc.ensure((size_t)Bp * kPrecKnots * sizeof(float)));
    CHECKED(M->kb.ensure((size_t)Bp * ld_max * sizeof(float)));
    CHECKED(M->idx.ensure((size_t)2 * Bp * sizeof(int)));
    std::vector<std::pair<int, int>> batches;  // (system, first sample)
    for (int k = 0; k < n_sys; ++k) {
      Scope ssc(sys[k]->device, &sys[k]->alloc);
      CHECKED(ensure_workspace(sys[k], std::max(sys[k]->ws_solves, Bp)));
      for (int j = sys_begin[k]; j < sys_begin[k + 1]; j += Bp) batches.push_back({k, j});
    }
    std::vector<float> hl(Bp);
    std::vector<int> hidx(2 * Bp);
    for (int ep = 0; ep < prec_epochs && nprec > 0; ++ep) {
      std::shuffle(batches.begin(), batches.end(), rng);
      double ep_loss = 0.0;
      int ep_n = 0;
      for (const auto& bt : batches) {
        stern_system* S = sys[bt.first];
        hipStream_t st2 = S->stream;
        const int K = S->hb.npw_pad;
        const int nbt = std::min(Bp, sys_begin[bt.first + 1] - bt.second);
        for (int t = 0; t < nbt; ++t) {
          hidx[t] = bt.second - sys_begin[bt.first] + t;  // row within the system's block
          hidx[Bp + t] = bt.second + t;                   // global sample (features)
        }
        HIPOK(hipMemcpyAsync(M->idx.p, hidx.data(), 2 * Bp * sizeof(int), hipMemcpyHostToDevice, st2));
        const CgState cs = cg_state(S);
        const Z64* R0 = M->r0set.as<Z64>() + sys_off[bt.first];
        const Z64* E0 = M->e0set.as<Z64>() + sys_off[bt.first];
        launch_gather_f32(M->fb.as<float>(), M->fset.as<float>(), M->idx.as<int>() + Bp, kPrecIn, nbt, st2);
        launch_prec_coef(M->head(), M->fb.as<float>(), M->coef.as<float>(), nbt, st2);
        launch_prec_build(M->coef.as<float>(), M->fb.as<float>(), cs.g2h, M->kb.as<float>(), K, nbt, st2);
        launch_prec_apply(M->kb.as<float>(), R0, M->idx.as<int>(), cs.z, K, nbt, st2);
        CHECKED(apply_pc_rows(S, cs.z, nullptr, nbt));
        launch_prec_grad(cs.z, R0, E0, M->idx.as<int>(), M->coef.as<float>(), M->fb.as<float>(), cs.g2h, S->hb.npw, K,
                         M->gc.as<float>(), M->loss.as<float>(), nbt, st2);
        launch_head_grad(M->gc.as<float>(), M->fb.as<float>(), nbt, M->grad.as<float>() + stern_model::HEAD, st2);
        ++M->prec_step;
        launch_adam(M->w.as<float>() + stern_model::HEAD, M->m.as<float>() + stern_model::HEAD,
                    M->v.as<float>() + stern_model::HEAD, M->grad.as<float>() + stern_model::HEAD, kPrecParams,
                    prec_lr, M->prec_step, 1.f / (float)nbt, st2);
        CHECKED(launch_check());
        HIPOK(hipMemcpyAsync(hl.data(), M->loss.p, nbt * sizeof(float), hipMemcpyDeviceToHost, st2));
        HIPOK(hipStreamSynchronize(st2));
        for (int t = 0; t < nbt; ++t) ep_loss += hl[t];
        ep_n += nbt;
      }
      const double mean = ep_n ? ep_loss / ep_n : 0.0;
      if (ep == 0) pfirst = mean;
      plast = mean;
    }
    M->prec_trained = nprec > 0;
  }
  if (tstats) {
    tstats->n_samples = nsamp;
    tstats->steps = steps;
    tstats->loss_first = std::sqrt(first);
    tstats->loss_last = std::sqrt(last);
    tstats->prec_samples = nprec;
    tstats->prec_loss_first = pfirst;
    tstats->prec_loss_last = plast;
    tstats->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return STERN_OK;
}

void stern_free(stern_system* S) {
  if (!S) return;
  {
    Scope sc(S->device, &S->alloc);
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    else (void)hipDeviceSynchronize();
    S->release_all();
  }
  delete S;
}

}  // extern "C"
