// C ABI of the Sternheimer chi0 library: system setup, occupied states, the
// batched projected-PCG driver and the density response.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stern.h"
#include "basis.hpp"
#include "kernels.hpp"

using namespace stern;

namespace {

thread_local std::string g_err;

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

// A device allocation that only grows.
struct DBuf {
  void* p = nullptr;
  size_t n = 0;
  int ensure(size_t bytes) {
    if (bytes <= n) return 0;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    if (bytes == 0) return 0;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(STERN_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    n = bytes;
    return 0;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
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

struct stern_system {
  int device = 0;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;  // non-blocking stream for graph capture (created on demand)
  CellParams cell;
  HostBasis hb;
  int n_atoms = 0, natoms_pad = 0;
  // static device data
  DBuf col_start, col_len, col_xmin, col_pos, zl, ycol, g2h, tw64, tw32, v_r, v_r32, kb, perm;
  // occupied states
  int n_occ = 0, nocc_pad = 0;
  bool have_occ = false;
  std::vector<double> eps, invT;
  DBuf psi, psi_r;
  // split BF16 copies of Psi and of the KB rows (row and transposed layouts)
  DBuf psi_hi, psi_lo, psiT_hi, psiT_lo, kb_hi, kb_lo, kbT_hi, kbT_lo;
  // workspace
  DBuf wx, wr, wp, wq, wz, wb, pen, cpart, cmat, sv_eps, sv_invT, sv_band, sv_pert, sv_bb, sv_rz, sv_rr, sv_flag,
      sv_iters, sv_tres, list_act, list_f, pert_out, dv_dev, dn_dev, tmp_in, tmp_out;
  DBuf m_d, m_r, m_p, m_q, m_z, m_rz, m_rr0, m_flag;  // mixed inner solve
  int ws_solves = 0, ws32_solves = 0;

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
    return g;
  }

  void release_all() {
    DBuf* all[] = {&ycol, &tw32, &v_r32, &col_start, &col_len,  &col_xmin, &col_pos, &zl,       &g2h,     &tw64,     &v_r,      &kb,
                   &perm,      &psi,      &psi_r,    &wx,      &wr,       &wp,      &wq,       &wz,       &wb,
                   &pen,       &cpart,    &cmat,     &sv_eps,  &sv_invT,  &sv_band, &sv_pert,  &sv_bb,    &sv_rz,
                   &sv_rr,     &sv_flag,  &sv_iters, &sv_tres, &list_act, &list_f,  &pert_out, &dv_dev,   &dn_dev,
                   &tmp_in,    &tmp_out,  &psi_hi,  &psi_lo,   &psiT_hi, &psiT_lo,  &kb_hi,    &kb_lo,
                   &kbT_hi,    &kbT_lo,   &m_d,     &m_r,      &m_p,     &m_q,      &m_z,      &m_rz,
                   &m_rr0,     &m_flag};
    for (DBuf* d : all) d->release();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    events.clear();
    if (own_stream) (void)hipStreamDestroy(own_stream);
    own_stream = nullptr;
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
  const int ns = choose_nsplit(S->nocc_pad, n, K);
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

// out = (H - eps_s) in on rows list (without projection); eps per row index
int apply_h_rows(stern_system* S, const Z64* in, Z64* out, const int* list, int n, const double* eps_rows) {
  if (n <= 0) return 0;
  const FftGeom g = S->geom();
  const int K = S->hb.npw_pad;
  const double zb = sizeof(Z64), npw = S->hb.npw, N = S->hb.N, pen = N * S->hb.ncol * zb;
  CHECKED(timed(S, STERN_K_XINV, n * (npw * zb + pen), 0.0,
                [&] { launch_xinv(g, in, list, n, S->pen.as<Z64>(), S->stream); }));
  CHECKED(timed(S, STERN_K_PLANE_H, n * 2.0 * pen + N * N * N * sizeof(double), 0.0,
                [&] { launch_plane_vloc(g, S->pen.as<Z64>(), list, n, S->v_r.as<double>(), S->stream); }));
  CHECKED(timed(S, STERN_K_XFWD, n * (pen + 2.0 * npw * zb), 0.0,
                [&] { launch_xfwd(g, S->pen.as<Z64>(), list, n, out, 1, in, eps_rows, 0.0, S->stream); }));
  if (S->n_atoms > 0) {
    const double na = S->n_atoms;
    const int ns = choose_nsplit(S->natoms_pad, n, K);
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
int apply_pc32_rows(stern_system* S, Z32* Y, const int* list, int n) {
  if (n <= 0) return 0;
  const int K = S->hb.npw_pad;
  const double npw = S->hb.npw, m = S->n_occ;
  const int ns = choose_nsplit_bf16(S->nocc_pad, n, K);
  Z32* cp = S->cpart.as<Z32>();
  Z32* cm = S->cmat.as<Z32>();
  CHECKED(timed(S, STERN_K_GEMM_BF16, 8.0 * npw * (n + m), 8.0 * m * npw * n, [&] {
    launch_reduce_bf16(S->psi_hi.as<__bf16>(), S->psi_lo.as<__bf16>(), S->nocc_pad, Y, K, list, n, K, cp, ns,
                       S->stream);
  }));
  CHECKED(timed(S, STERN_K_SUM_PARTS, 8.0 * m * n * (ns + 1), 0.0,
                [&] { launch_sum_parts32(cp, ns, n, S->nocc_pad, -1.f, cm, S->stream); }));
  CHECKED(timed(S, STERN_K_GEMM_BF16, 8.0 * npw * (2.0 * n + m), 8.0 * m * npw * n, [&] {
    launch_expand_bf16(S->psiT_hi.as<__bf16>(), S->psiT_lo.as<__bf16>(), S->nocc_pad, cm, Y, K, list, n, K,
                       S->stream);
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
  CHECKED(timed(S, STERN_K_PLANE_H32, n * 2.0 * pen + N * N * N * sizeof(float), 0.0,
                [&] { launch_plane_vloc<float>(g, pen32, list, n, S->v_r32.as<float>(), S->stream); }));
  CHECKED(timed(S, STERN_K_X32, n * (pen + 2.0 * npw * zb), 0.0,
                [&] { launch_xfwd<float>(g, pen32, list, n, out, 1, in, eps_rows, 0.0, S->stream); }));
  if (S->n_atoms > 0) {
    const double na = S->n_atoms;
    const int ns = choose_nsplit_bf16(S->natoms_pad, n, K);
    Z32* cp = S->cpart.as<Z32>();
    Z32* cm = S->cmat.as<Z32>();
    CHECKED(timed(S, STERN_K_GEMM_BF16, zb * npw * (n + na), 8.0 * na * npw * n, [&] {
      launch_reduce_bf16(S->kb_hi.as<__bf16>(), S->kb_lo.as<__bf16>(), S->natoms_pad, in, K, list, n, K, cp, ns,
                         S->stream);
    }));
    CHECKED(timed(S, STERN_K_SUM_PARTS, zb * na * n * (ns + 1), 0.0,
                  [&] { launch_sum_parts32(cp, ns, n, S->natoms_pad, (float)S->cell.D, cm, S->stream); }));
    CHECKED(timed(S, STERN_K_GEMM_BF16, zb * npw * (2.0 * n + na), 8.0 * na * npw * n, [&] {
      launch_expand_bf16(S->kbT_hi.as<__bf16>(), S->kbT_lo.as<__bf16>(), S->natoms_pad, cm, out, K, list, n, K,
                         S->stream);
    }));
  }
  return 0;
}

size_t cpart_capacity(int M_pad, int nmax, int K) {
  size_t best = 0;
  for (int n = 1; n <= nmax; ++n) {
    const size_t c = (size_t)choose_nsplit(M_pad, n, K) * n;
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
  CHECKED(S->cpart.ensure(std::max(cpart_capacity(std::max(S->nocc_pad, 64), ns, (int)K),
                                   cpart_capacity(S->natoms_pad, ns, (int)K)) * sizeof(Z64)));
  CHECKED(S->cmat.ensure((size_t)ns * mp * sizeof(Z64)));
  for (DBuf* d : {&S->sv_eps, &S->sv_invT, &S->sv_bb, &S->sv_rz, &S->sv_rr, &S->sv_tres})
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
  for (DBuf* d : {&S->m_rz, &S->m_rr0}) CHECKED(d->ensure((size_t)ns * sizeof(double)));
  CHECKED(S->m_flag.ensure((size_t)ns * sizeof(int)));
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
  c.flag = S->m_flag.as<int>();
  c.iters = iters;
  c.invT = S->sv_invT.as<double>();
  c.g2h = S->g2h.as<double>();
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

struct Scope {
  int dev_prev = -1;
  explicit Scope(int dev) {
    (void)hipGetDevice(&dev_prev);
    (void)hipSetDevice(dev);
  }
  ~Scope() {
    if (dev_prev >= 0) (void)hipSetDevice(dev_prev);
  }
};


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
              int check_every, int& n_restart, double vecb, bool use_graph) {
  hipStream_t st = S->stream;
  const int ns_all = S->ws_solves;
  std::vector<int> h_flag(ns_all), act, flist;
  if (list.empty()) return 0;
  const int n0 = (int)list.size();
  HIPOK(hipMemcpyAsync(S->list_act.p, list.data(), n0 * sizeof(int), hipMemcpyHostToDevice, st));
  {
    const int* L = S->list_act.as<int>();
    CHECKED(timed(S, STERN_K_CG, vecb * n0 * 4.0, 0.0, [&] { launch_cg_init(cs, L, n0, st); }));
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

// Mixed precision: FP64 defect correction around FP32/BF16 inner PCG solves.
//   repeat: solve A d = r to inner_tol with FP32 FFTs and split-BF16 MFMA GEMMs
//           (FP64 dots and scalars); x += d; x = P_c x (FP64); r = b - A x (FP64)
//   until ||r|| <= tol ||b||; solves still above tol after max_outer steps are
//   re-solved by FP64 PCG from zero.
int run_mixed(stern_system* S, const CgState& cs, const std::vector<int>& list, double tol, double inner_tol,
              int max_outer, int max_iter, int check_every, int& n_restart, int& n_fallback, double vecb,
              bool use_graph) {
  hipStream_t st = S->stream;
  const int ns_all = S->ws_solves;
  const int K = S->hb.npw_pad;
  const double vec32 = vecb / 2;
  const Cg32State c32 = cg32_state(S, cs.iters);
  std::vector<int> h_flag(ns_all), h_iflag(ns_all), act, iact;
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
    CHECKED(apply_pc32_rows(S, c32.z, L, na));
    CHECKED(timed(S, STERN_K_CG32, na * 3.0 * vec32, 0.0, [&] { launch_cg32_init2(c32, L, na, st); }));
    CHECKED(launch_check());
    HIPOK(hipMemcpyAsync(h_iflag.data(), c32.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    iact.clear();
    for (int s : act)
      if (h_iflag[s] == 0) iact.push_back(s);
    int it = 0;
    while (!iact.empty() && it < max_inner) {
      const int ni = (int)iact.size();
      HIPOK(hipMemcpyAsync(S->list_f.p, iact.data(), ni * sizeof(int), hipMemcpyHostToDevice, st));
      const int* F = S->list_f.as<int>();
      const int nsteps = std::min(check_every, max_inner - it);
      CHECKED(run_steps(S, nsteps, use_graph && (it > 0 || outer > 0), [&]() -> int {
        CHECKED(apply_h32_rows(S, c32.p, c32.q, F, ni, cs.eps));
        CHECKED(apply_pc32_rows(S, c32.q, F, ni));
        CHECKED(timed(S, STERN_K_CG32, vec32 * ni * 7.0, 0.0,
                      [&] { launch_cg32_alpha(c32, F, ni, inner_tol * inner_tol, st); }));
        CHECKED(apply_pc32_rows(S, c32.z, F, ni));
        CHECKED(timed(S, STERN_K_CG32, vec32 * ni * 4.0, 0.0, [&] { launch_cg32_beta(c32, F, ni, st); }));
        return 0;
      }));
      it += nsteps;
      CHECKED(launch_check());
      HIPOK(hipMemcpyAsync(h_iflag.data(), c32.flag, ns_all * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPOK(hipStreamSynchronize(st));
      std::vector<int> nxt;
      for (int s : iact)
        if (h_iflag[s] == 0) nxt.push_back(s);
      iact.swap(nxt);
    }
    // FP64 update, re-orthogonalisation and true residual
    CHECKED(timed(S, STERN_K_CG, na * (2.0 * vecb + vec32), 0.0, [&] { launch_add_d(cs.x, c32.d, K, L, na, st); }));
    CHECKED(apply_pc_rows(S, cs.x, L, na));
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
  if (!act.empty()) {
    n_fallback += (int)act.size();
    CHECKED(run_pcg64(S, cs, act, tol, max_iter, check_every, n_restart, vecb, use_graph));
  }
  return 0;
}

}  // namespace

// ============================================================== C ABI ======

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
  stern_system* S = new stern_system();
  S->device = rt ? rt->device : 0;
  S->stream = rt ? (hipStream_t)rt->stream : nullptr;
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
  Scope sc(S->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, S->device) != hipSuccess) {
    delete S;
    return fail(STERN_ERR_HIP, "hipGetDeviceProperties failed");
  }
  const size_t lds = plane_lds_bytes(hb.N, sizeof(Z64));
  if (lds > prop.sharedMemPerBlock && lds > (size_t)prop.maxSharedMemoryPerMultiProcessor) {
    delete S;
    return fail(STERN_ERR_UNSUPPORTED, "FP64 plane of grid %d needs %zu bytes of LDS", hb.N, lds);
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
    std::vector<std::complex<double>> B = kb_projectors(p, hb, S->natoms_pad);
    CHECKED(upload(S->kb, B.data(), B.size() * sizeof(Z64), st));
    const size_t kbn = (size_t)S->natoms_pad * hb.npw_pad * 2 * sizeof(__bf16);
    for (DBuf* d : {&S->kb_hi, &S->kb_lo, &S->kbT_hi, &S->kbT_lo}) CHECKED(d->ensure(kbn));
    launch_split_bf16(S->kb.as<Z64>(), S->natoms_pad, hb.npw_pad, S->kb_hi.as<__bf16>(), S->kb_lo.as<__bf16>(),
                      S->kbT_hi.as<__bf16>(), S->kbT_lo.as<__bf16>(), st);
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

int stern_set_occupied(stern_system* S, int n_occ, const double* psi, const double* eps, int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (n_occ <= 0 || !psi || !eps) return fail(STERN_ERR_INVALID_ARG, "need n_occ > 0, psi and eps");
  if (mem_kind != STERN_MEM_HOST && mem_kind != STERN_MEM_DEVICE) return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  Scope sc(S->device);
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
  CHECKED(S->psi.ensure((size_t)S->nocc_pad * K * sizeof(Z64)));
  launch_fill_zero(S->psi.as<Z64>(), (size_t)S->nocc_pad * K, st);
  CHECKED(S->tmp_in.ensure((size_t)n_occ * npw * sizeof(Z64)));
  HIPOK(hipMemcpyAsync(S->tmp_in.p, hp, (size_t)n_occ * npw * sizeof(Z64), hipMemcpyHostToDevice, st));
  launch_permute(S->tmp_in.as<Z64>(), npw, S->psi.as<Z64>(), K, S->perm.as<int>(), npw, n_occ, true, st);
  const size_t psn = (size_t)S->nocc_pad * K * 2 * sizeof(__bf16);
  for (DBuf* d : {&S->psi_hi, &S->psi_lo, &S->psiT_hi, &S->psiT_lo}) CHECKED(d->ensure(psn));
  launch_split_bf16(S->psi.as<Z64>(), S->nocc_pad, K, S->psi_hi.as<__bf16>(), S->psi_lo.as<__bf16>(),
                    S->psiT_hi.as<__bf16>(), S->psiT_lo.as<__bf16>(), st);
  // psi_v(r) on the grid (unnormalised sum_G c_G e^{iG.r}) for the RHS and dn
  CHECKED(S->psi_r.ensure((size_t)n_occ * N * N * N * sizeof(Z64)));
  CHECKED(S->pen.ensure((size_t)n_occ * N * hb.ncol_pad * sizeof(Z64)));
  const FftGeom g = S->geom();
  launch_xinv(g, S->psi.as<Z64>(), nullptr, n_occ, S->pen.as<Z64>(), st);
  launch_plane_full_inv(g, S->pen.as<Z64>(), n_occ, S->psi_r.as<Z64>(), st);
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
  Scope sc(S->device);
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

int stern_apply_pc(stern_system* S, int n_vec, const double* c, double* out, int mem_kind) {
  if (!S) return fail(STERN_ERR_INVALID_ARG, "system is NULL");
  if (!S->have_occ) return fail(STERN_ERR_STATE, "set_occupied has not been called");
  if (n_vec <= 0) return STERN_OK;
  if (!c || !out) return fail(STERN_ERR_INVALID_ARG, "NULL array");
  Scope sc(S->device);
  CHECKED(ensure_workspace(S, std::max(n_vec, S->ws_solves)));
  CHECKED(rows_in(S, n_vec, c, mem_kind, S->wp));
  CHECKED(apply_pc_rows(S, S->wp.as<Z64>(), nullptr, n_vec));
  CHECKED(launch_check());
  return rows_out(S, n_vec, S->wp.as<Z64>(), nullptr, out, mem_kind);
}

static int apply_chi0_impl(stern_system* S, int n_pert, const double* dv_r, double* dn_r, const stern_opts* opts,
                           stern_stats* stats);

int stern_apply_chi0(stern_system* S, int n_pert, const double* dv_r, double* dn_r, const stern_opts* opts,
                     stern_stats* stats) {
  if (!S || !opts || !opts->use_graph || opts->profile) return apply_chi0_impl(S, n_pert, dv_r, dn_r, opts, stats);
  // stream capture is not allowed on the legacy default stream: run on the system's own stream
  Scope sc(S->device);
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
  if (opts->guess != STERN_GUESS_ZERO) return fail(STERN_ERR_UNSUPPORTED, "only STERN_GUESS_ZERO is available");
  if (opts->mem_kind != STERN_MEM_HOST && opts->mem_kind != STERN_MEM_DEVICE)
    return fail(STERN_ERR_INVALID_ARG, "bad mem_kind");
  if (!(opts->tol > 0)) return fail(STERN_ERR_INVALID_ARG, "tol must be > 0");
  const int v0 = opts->band_begin;
  const int v1 = opts->band_end > 0 ? opts->band_end : S->n_occ;
  if (v0 < 0 || v1 > S->n_occ || v0 >= v1) return fail(STERN_ERR_INVALID_ARG, "bad band range [%d, %d)", v0, v1);
  if (opts->n_sample < 0 || (opts->n_sample > 0 && (!opts->sample_pairs || !opts->sample_x)))
    return fail(STERN_ERR_INVALID_ARG, "bad sample request");
  for (int k = 0; k < opts->n_sample; ++k) {
    const int v = opts->sample_pairs[2 * k], i = opts->sample_pairs[2 * k + 1];
    if (v < v0 || v >= v1 || i < 0 || i >= n_pert) return fail(STERN_ERR_INVALID_ARG, "sample pair %d out of range", k);
  }
  Scope sc(S->device);
  hipStream_t st = S->stream;
  const HostBasis& hb = S->hb;
  const int N = hb.N, K = hb.npw_pad;
  const size_t n3 = (size_t)N * N * N;
  const int nb = v1 - v0;
  const int max_iter = opts->max_iter > 0 ? opts->max_iter : 1000;
  const int check_every = opts->check_every > 0 ? opts->check_every : 4;
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
  const CgState cs = cg_state(S);
  const FftGeom g = S->geom();
  std::vector<int> all_iters, all_flag;
  std::vector<double> all_tres;
  all_iters.reserve((size_t)n_pert * nb);
  long long tot_iters = 0;
  int n_restart = 0, n_fallback = 0;

  std::vector<int> h_flag(max_ns), h_band(max_ns), h_pert(max_ns);
  std::vector<double> h_eps(max_ns), h_invT(max_ns);
  for (int i0 = 0; i0 < n_pert; i0 += per) {
    const int i1 = std::min(n_pert, i0 + per);
    const int ns = (i1 - i0) * nb;
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
    // b = -P_c [dV psi_v]
    CHECKED(timed(S, STERN_K_RHS, ns * ((double)n3 * 24.0 + (double)N * hb.ncol * 16.0), 0.0, [&] {
      launch_plane_rhs(g, S->psi_r.as<Z64>(), dv_dev, S->sv_band.as<int>(), S->sv_pert.as<int>(), ns,
                       S->pen.as<Z64>(), st);
    }));
    CHECKED(timed(S, STERN_K_XFWD, ns * ((double)N * hb.ncol * 16.0 + vecb), 0.0, [&] {
      launch_xfwd<double>(g, S->pen.as<Z64>(), nullptr, ns, cs.b, 2, nullptr, nullptr, -1.0 / (double)n3, st);
    }));
    CHECKED(apply_pc_rows(S, cs.b, nullptr, ns));
    launch_outer_init(cs, nullptr, ns, st);  // x = 0, r = b, ||b||, counters
    std::vector<int> all(ns);
    for (int s = 0; s < ns; ++s) all[s] = s;
    if (opts->precision == STERN_MIXED) {
      CHECKED(run_mixed(S, cs, all, tol, inner_tol, max_outer, max_iter, check_every, n_restart, n_fallback, vecb,
                        use_graph));
    } else {
      CHECKED(run_pcg64(S, cs, all, tol, max_iter, check_every, n_restart, vecb, use_graph));
    }
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
    Scope sc(sys[k]->device);
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

void stern_free(stern_system* S) {
  if (!S) return;
  {
    Scope sc(S->device);
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    else (void)hipDeviceSynchronize();
    S->release_all();
  }
  delete S;
}

}  // extern "C"
