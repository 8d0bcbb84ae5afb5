// Conjugate gradient on A = D^dagger D (the solve of Algorithm 1).
//
// Plain CG (inner_prec = F64) runs Algorithm 1's inner recurrence entirely
// in float64:  q = A p;  alpha = rho / <p, q>;  x += alpha p;  r -= alpha q;
// rho' = <r, r>;  p = r + (rho'/rho) p.  Per iteration this is three
// kernels:
//   1. t = D p, fused with |t|^2 = <p, A p>  -> alpha        (device)
//   2. r -= alpha D^dag t, fused with |r|^2  -> beta, rho    (device)
//      (A p itself is never stored)
//   3. x += alpha p;  p = r + beta p
// All scalars live in device memory (CgState), so a batch of iterations is
// enqueued without host round trips; the host checks convergence between
// batches.  Converged right-hand sides are gated off inside the kernels.
// When the recursive residual reaches the target, the true residual
// ||eta - A x|| is recomputed in float64 and the solve restarts from it if it
// is still above the tolerance.
//
// Mixed precision (inner_prec = F32 / F16S / BF16S) follows Algorithm 1:
// a float64 outer loop computes the true residual r = eta - A x, its norm
// s, and the normalised r0 = r / s in low precision; a low-precision inner
// CG (float32 arithmetic, float64 reductions) solves A psi = r0 until
// ||r_inner|| < delta; the solution is updated x += s psi in float64.  The
// search direction of the previous cycle is carried over after removing its
// component along the new r0 and rescaling by beta_0 = s_new / (s_old rho_k)
// (the reading of the carried direction p_0 = r0 + beta_0 p~).  The inner
// iteration count is open in the paper: the first cycle runs to ||r|| < delta
// (or inner_kmax); later cycles, which restart from a unit residual, may take
// at most twice the first cycle's count.  Two capped cycles in a row, or six
// cycles without progress, mean the low-precision operator cannot reach the
// target and the solve finishes in float64.
//
// The even-odd form (cg_solve_eo) runs the same machinery on the normal
// equations of the even-site Schur complement, D_hat^dagger D_hat x_e =
// D_hat^dagger b_hat, for the system D x = b: the two operator applications
// of an iteration become two half-lattice hops each, and the vector
// operations act on the even sites of the fields only.  The odd sites are
// reconstructed afterwards and the residual ||b - D x|| checked on the full
// lattice; if it is still above the target, the CG tolerance is tightened
// and the solve resumed from the current x.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "lib.h"

namespace dirac {

namespace {

// Lattices up to this many sites run their CG iterations in one launch by
// default (one workgroup per right-hand side): measured, the single launch
// is 2-4x faster on 4^4 and slower from about 2000 sites on, where one
// workgroup's latency chain outweighs the launches it saves.
constexpr int64_t kSingleLaunchSites = 1024;

struct Layout {
  int64_t state, partials, r, p, t, r0, psi, plo, tlo, eh, total;
  int64_t nparts;  // partial slots per right-hand side
};

Layout layout(const OpInfo& hi, int inner_prec, bool eo = false) {
  Layout L;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off += align256(bytes);
    return o;
  };
  const int nrhs = hi.nrhs;
  L.nparts = 2 * ((hi.g.Vh + 63) / 64);
  L.state = take(sizeof(CgState) * kMaxRhs);
  L.partials = take(L.nparts * nrhs * 2 * (int64_t)sizeof(double));
  const int64_t f64 = nrhs * align256(spinor_field_bytes(DIRAC_F64, hi.V));
  L.r = take(f64);
  L.p = take(f64);
  L.t = take(f64);
  if (inner_prec != DIRAC_F64) {
    const int64_t f32 = nrhs * align256(spinor_field_bytes(DIRAC_F32, hi.V));
    const int64_t flo = nrhs * align256(spinor_field_bytes(inner_prec, hi.V));
    L.r0 = take(f32);
    L.psi = take(f32);
    L.plo = take(flo);
    L.tlo = take(flo);
  } else {
    L.r0 = L.psi = L.plo = L.tlo = -1;
  }
  L.eh = eo ? take(f64) : -1;  // even-odd form: the source of the normal equations
  L.total = off;
  return L;
}

struct Ctx {
  OpInfo hi, lo;
  bool eo = false;  // operator: D_hat of the even-odd form instead of D
  int eo_dag = 0;   // even-odd form of D^dagger: D_hat^dagger, normal equations D_hat D_hat^dagger
  bool single = false;  // CG iterations in one launch (small lattices)
  Geom vg;          // geometry of the vector operations (even sites only when eo)
  const void* Uhi;
  const void* Ulo;
  char* work;
  Layout L;
  hipStream_t st;
  CgState* dstate;
  std::vector<CgState> hstate;
  RedTarget red(int kind) const {
    return RedTarget{(double*)(work + L.partials), dstate, kind};
  }
  FieldRef f(int64_t off, int prec) const { return field_as(hi, prec, work + off); }
  int pull() {
    int rc = hip_status(hipMemcpyAsync(hstate.data(), dstate, sizeof(CgState) * hi.nrhs, hipMemcpyDeviceToHost, st),
                        "state readback");
    if (rc != DIRAC_OK) return rc;
    return hip_status(hipStreamSynchronize(st), "solver sync");
  }
  int push() {
    int rc = hip_status(hipMemcpyAsync(dstate, hstate.data(), sizeof(CgState) * hi.nrhs, hipMemcpyHostToDevice, st),
                        "state upload");
    if (rc != DIRAC_OK) return rc;
    return hip_status(hipStreamSynchronize(st), "solver sync");
  }
};

RedArgs to_args(const RedTarget& t) { return RedArgs{t.partials, t.state, t.kind}; }

// sqrt of a reduced norm^2; NaN stays NaN (std::max would turn it into 0).
double norm_of(double v) { return std::isnan(v) ? v : std::sqrt(v > 0.0 ? v : 0.0); }

// Half-lattice hop: on the sites of parity par, out = cm * ctr + ch * K in
// (K of D^dagger when dag), with epilogue epi; src, use_alpha and the format
// of src / out (oprec, when it differs from o's) for the subtraction epilogue.
int hop(const Ctx& c, const OpInfo& o, const void* U, const void* in, const void* ctr, void* out, int par,
        int dag, double cm, double ch, int epi, int gate, int kind, const void* src = nullptr, int use_alpha = 0,
        int oprec = -1) {
  DslashArgs a = dslash_args(o, U, in, out);
  a.par = par;
  a.ctr = (const char*)ctr;
  a.ctr_stride = o.field_stride;
  a.mass4 = cm;
  a.hop_c = ch;
  a.gate = gate;
  a.red = to_args(c.red(kind));
  a.src = (const char*)src;
  a.src_stride = o.field_stride;
  a.sub_alpha = use_alpha;
  if (oprec >= 0 && oprec != o.prec) {
    const FieldRef d = field_as(c.hi, oprec, out);
    a.out_bytes = d.bytes;
    a.out_stride = d.stride;
    a.src_stride = d.stride;
  }
  return run_hop(o.prec, o.link, dag, epi, a, launch_cfg(o), c.st);
}

// t = D in (store + |t|^2 into `kind`), for precision op o.  Even-odd form:
// t_e = D_hat in_e (D_hat^dagger for the solve with D^dagger), with the odd
// plane of t holding the intermediate K_oe in_e.
int dslash_norm(const Ctx& c, const OpInfo& o, const void* U, const void* in, void* t, int gate, int kind) {
  if (c.eo) {
    const double A = o.m_q + 4.0;
    const int dag = c.eo_dag;
    int rc = hop(c, o, U, in, nullptr, t, 1, dag, 0.0, 1.0, kEpiStore, gate, kFinPlain);
    if (rc != DIRAC_OK) return rc;
    return hop(c, o, U, t, in, t, 0, dag, A, -1.0 / A, kEpiStoreNorm, gate, kind);
  }
  DslashArgs a = dslash_args(o, U, in, t);
  a.gate = gate;
  a.red = to_args(c.red(kind));
  return run_dslash(o.prec, o.prec, o.link, 0, kEpiStoreNorm, launch_cfg(o), a, c.st);
}

// dst = src - coef * D^dag in, |dst|^2 into `kind`; dst has precision dprec.
// Even-odd form: dst_e = src_e - coef * D_hat^dagger in_e (D_hat for the solve
// with D^dagger), and the odd plane of `in` (a workspace field) receives the
// intermediate.
int dslash_sub(const Ctx& c, const OpInfo& o, const void* U, const void* in, const void* src, void* dst, int dprec,
               int use_alpha, int gate, int kind) {
  if (c.eo) {
    const int want = (o.prec == DIRAC_F16S || o.prec == DIRAC_BF16S) ? DIRAC_F32 : o.prec;
    if (dprec != want) return set_error(DIRAC_EUNSUPPORTED, "even-odd residual update: format %d", dprec);
    const double A = o.m_q + 4.0;
    const int dag = 1 - c.eo_dag;
    int rc = hop(c, o, U, in, nullptr, (void*)in, 1, dag, 0.0, 1.0, kEpiStore, gate, kFinPlain);
    if (rc != DIRAC_OK) return rc;
    return hop(c, o, U, in, in, dst, 0, dag, A, -1.0 / A, kEpiSubNorm, gate, kind, src, use_alpha, dprec);
  }
  DslashArgs a = dslash_args(o, U, in, dst);
  const FieldRef d = field_as(c.hi, dprec, dst);
  a.out_bytes = d.bytes;
  a.out_stride = d.stride;
  a.src = (const char*)src;
  a.src_stride = d.stride;
  a.sub_alpha = use_alpha;
  a.gate = gate;
  a.red = to_args(c.red(kind));
  return run_dslash(o.prec, dprec, o.link, 1, kEpiSubNorm, launch_cfg(o), a, c.st);
}

// r = eta - A x (float64), |r|^2 into `kind`.
int true_residual(Ctx& c, const void* eta, const void* x, int kind) {
  int rc = dslash_norm(c, c.hi, c.Uhi, x, c.work + c.L.t, kGateNone, kFinPlain);
  if (rc != DIRAC_OK) return rc;
  return dslash_sub(c, c.hi, c.Uhi, c.work + c.L.t, eta, c.work + c.L.r, DIRAC_F64, 0, kGateNone, kind);
}

// Iterations enqueued between host convergence checks: about 600 us of work,
// at least 8 (an iteration past convergence is gated off inside its kernels
// and costs only the launches, cheaper than a host round trip).
int auto_check_every(const OpInfo& o) {
  const double iter_us = std::max(15.0, o.V * o.nrhs * 6e-4);
  return (int)std::min(64.0, std::max(8.0, std::round(600.0 / iter_us)));
}

// Run CG iterations on (x, p, r) with the given operator until every
// right-hand side is done; returns iterations done per RHS via hstate.
int run_iterations(Ctx& c, const OpInfo& o, const void* U, FieldRef x, FieldRef p, FieldRef r, FieldRef t,
                   int check_every) {
  if (c.single) {
    // about 2^18 site updates per launch (a few milliseconds), at most 1000 iterations
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(1000, (int64_t(1) << 18) / o.V));
    while (true) {
      int rc = cg_small_iterations(o, U, x, p, r, t, c.dstate, chunk, c.st);
      if (rc != DIRAC_OK) return rc;
      rc = c.pull();
      if (rc != DIRAC_OK) return rc;
      bool all = true;
      for (int k = 0; k < c.hi.nrhs; ++k) all &= c.hstate[k].done != 0;
      if (all) return DIRAC_OK;
    }
  }
  // Iterations are enqueued in batches between host checks.  An iteration
  // enqueued after its right-hand side is done still launches its kernels
  // (gated off, but every block starts), so each batch after the first is
  // sized from the convergence rate seen so far: the iterations the slowest
  // active right-hand side still needs to reach its stop2, plus one, at most
  // check_every.  An underestimate costs one more host check.
  const int n = c.hi.nrhs;
  std::vector<double> rho_prev(n, -1.0);
  int batch = check_every;
  while (true) {
    for (int k = 0; k < batch; ++k) {
      int rc = dslash_norm(c, o, U, p.ptr, t.ptr, kGateNotDone, kFinAlpha);
      if (rc != DIRAC_OK) return rc;
      rc = dslash_sub(c, o, U, t.ptr, r.ptr, r.ptr, r.prec, 1, kGateActive, kFinRho);
      if (rc != DIRAC_OK) return rc;
      rc = hip_status(cg_xp_update(c.vg, n, x, p, r, c.dstate, c.st), "cg update");
      if (rc != DIRAC_OK) return rc;
    }
    int rc = c.pull();
    if (rc != DIRAC_OK) return rc;
    bool all = true;
    double need = 0.0;
    for (int k = 0; k < n; ++k) {
      const CgState& S = c.hstate[k];
      if (S.done) continue;
      all = false;
      double est = check_every;  // no usable rate yet
      if (rho_prev[k] > 0.0 && S.rho > 0.0 && S.rho < rho_prev[k] && S.stop2 > 0.0) {
        const double rate = std::log(S.rho / rho_prev[k]) / batch;  // log decrease per iteration
        est = S.rho <= S.stop2 ? 1.0 : std::log(S.stop2 / S.rho) / rate;
      }
      est = std::min(est, (double)(S.kmax - S.iters));
      need = std::max(need, est);
      rho_prev[k] = S.rho;
    }
    if (all) return DIRAC_OK;
    batch = (int)std::min<double>(check_every, std::max(1.0, std::ceil(need) + 1.0));
  }
}

int eta_norms(Ctx& c, const void* eta, std::vector<double>& en) {
  int rc = hip_status(norm2(c.vg, c.hi.nrhs, field_of(c.hi, eta), c.red(kFinPlain), c.st), "norm");
  if (rc != DIRAC_OK) return rc;
  rc = c.pull();
  if (rc != DIRAC_OK) return rc;
  for (int k = 0; k < c.hi.nrhs; ++k) en[k] = std::sqrt(c.hstate[k].res[0]);
  return DIRAC_OK;
}

// Plain float64 CG starting from x (in place).
int cg_f64(Ctx& c, const void* eta, void* x, const cg_params& prm, const std::vector<double>& en,
           std::vector<cg_stats>& stats, int check_every) {
  const int n = c.hi.nrhs;
  FieldRef X = field_of(c.hi, x), P = c.f(c.L.p, DIRAC_F64), R = c.f(c.L.r, DIRAC_F64), T = c.f(c.L.t, DIRAC_F64);
  std::vector<int> used(n, 0);
  std::vector<bool> finished(n, false);
  for (int k = 0; k < n; ++k) {
    used[k] = stats[k].iters;
    if (en[k] == 0.0) finished[k] = true;
    if (!std::isfinite(en[k])) {
      stats[k].status = DIRAC_EBREAKDOWN;
      finished[k] = true;
    }
  }
  while (true) {
    int rc = true_residual(c, eta, x, kFinRhoSet);
    if (rc != DIRAC_OK) return rc;
    for (int k = 0; k < n; ++k) stats[k].dslash_hi += 2;
    rc = c.pull();
    if (rc != DIRAC_OK) return rc;
    bool any = false;
    for (int k = 0; k < n; ++k) {
      const double res = norm_of(c.hstate[k].rho);
      const double rel = en[k] > 0 ? res / en[k] : 0.0;
      if (!finished[k]) {
        stats[k].true_rel_res = rel;
        stats[k].outer += 1;
        if (!std::isfinite(rel)) {
          stats[k].status = DIRAC_EBREAKDOWN;
          finished[k] = true;
        } else if (rel < prm.tol) {
          stats[k].status = DIRAC_OK;
          finished[k] = true;
        } else if (used[k] >= prm.max_iter) {
          stats[k].status = DIRAC_ENOCONV;
          finished[k] = true;
        } else if (stats[k].status == DIRAC_EBREAKDOWN) {
          finished[k] = true;
        }
      }
      CgState& s = c.hstate[k];
      s.stop2 = std::pow(prm.tol * en[k], 2);
      s.kmax = std::max(0, prm.max_iter - used[k]);
      s.iters = 0;
      s.done = finished[k] ? 1 : 0;
      s.active = 0;
      s.status = DIRAC_OK;
      any |= !finished[k];
    }
    if (!any) return DIRAC_OK;
    rc = c.push();
    if (rc != DIRAC_OK) return rc;
    rc = hip_status(convert_scale(c.vg, n, R, P, nullptr, -1, nullptr, c.st), "copy");  // p = r
    if (rc != DIRAC_OK) return rc;
    rc = run_iterations(c, c.hi, c.Uhi, X, P, R, T, check_every);
    if (rc != DIRAC_OK) return rc;
    for (int k = 0; k < n; ++k) {
      if (finished[k]) continue;
      stats[k].iters += c.hstate[k].iters;
      stats[k].dslash_hi += 2 * c.hstate[k].iters;
      used[k] += c.hstate[k].iters;
      if (c.hstate[k].status == DIRAC_EBREAKDOWN) stats[k].status = DIRAC_EBREAKDOWN;
    }
  }
}

// Algorithm 1 with a low-precision inner CG.
int cg_mixed(Ctx& c, const void* eta, void* x, const cg_params& prm, const std::vector<double>& en,
             std::vector<cg_stats>& stats, int check_every, bool* fallback) {
  const int n = c.hi.nrhs;
  const int lp = c.lo.prec;
  FieldRef X = field_of(c.hi, x), R = c.f(c.L.r, DIRAC_F64);
  FieldRef R0 = c.f(c.L.r0, DIRAC_F32), PSI = c.f(c.L.psi, DIRAC_F32), PLO = c.f(c.L.plo, lp),
           TLO = c.f(c.L.tlo, lp);
  // Default inner target: 1e-3 for float32 and 0.1 for the 16-bit formats;
  // the better-conditioned even-odd system lets F16S reach 0.02, which saves
  // outer cycles (measured flat from 0.05 down to 0.005 on 32^3 x 64; BF16S
  // falls back to float64 below 0.1 there, as both formats do with D^dag D).
  const double delta = prm.inner_delta > 0 ? prm.inner_delta
                       : (lp == DIRAC_F32 ? 1e-3 : (c.eo && lp == DIRAC_F16S ? 0.02 : 0.1));
  const int kmax = prm.inner_kmax > 0 ? prm.inner_kmax : 10000;

  std::vector<double> s(n), s_prev(n, 0.0), s_best(n), rho_k(n, 0.0);
  std::vector<bool> have_p(n, false), conv(n, false);
  std::vector<int> stall(n, 0), used(n, 0), capped(n, 0), n_first(n, -1), n_cap(n, kmax);
  *fallback = false;

  int rc = hip_status(zero(c.vg, n, PLO, c.st), "zero");
  if (rc != DIRAC_OK) return rc;
  rc = true_residual(c, eta, x, kFinPlain);
  if (rc != DIRAC_OK) return rc;
  rc = c.pull();
  if (rc != DIRAC_OK) return rc;
  for (int k = 0; k < n; ++k) {
    stats[k].dslash_hi += 2;
    s[k] = norm_of(c.hstate[k].res[0]);
    s_best[k] = s[k];
    conv[k] = en[k] == 0.0 || s[k] < prm.tol * en[k] || !std::isfinite(en[k]);
    if (!std::isfinite(en[k])) stats[k].status = DIRAC_EBREAKDOWN;
    stats[k].true_rel_res = en[k] > 0 ? s[k] / en[k] : 0.0;
  }

  while (true) {
    bool any = false;
    for (int k = 0; k < n; ++k) {
      if (conv[k]) continue;
      if (!std::isfinite(s[k])) {
        stats[k].status = DIRAC_EBREAKDOWN;
        conv[k] = true;
        continue;
      }
      if (used[k] >= prm.max_iter) {
        stats[k].status = DIRAC_ENOCONV;
        conv[k] = true;
        continue;
      }
      any = true;
    }
    if (!any) return DIRAC_OK;

    // r0 = r / s in float32 (rho0 = |r0|^2 as stored), converged RHS scaled by 0
    for (int k = 0; k < n; ++k) c.hstate[k].coef[0] = conv[k] ? 0.0 : 1.0 / s[k];
    rc = c.push();
    if (rc != DIRAC_OK) return rc;
    RedTarget rt = c.red(kFinRhoSet);
    rc = hip_status(convert_scale(c.vg, n, R, R0, c.dstate, 0, &rt, c.st), "cast");
    if (rc != DIRAC_OK) return rc;
    // carried direction: <r0, p_k>
    rc = hip_status(dot(c.vg, n, R0, PLO, c.red(kFinPlain), c.st), "dot");
    if (rc != DIRAC_OK) return rc;
    rc = c.pull();
    if (rc != DIRAC_OK) return rc;
    for (int k = 0; k < n; ++k) {
      CgState& S = c.hstate[k];
      const double rho0 = S.rho;
      if (have_p[k] && !conv[k] && rho0 > 0) {
        // p0 = r0 + beta0 (p_k - (<r0,p_k>/rho0) r0) = (1 - beta0 c/rho0) r0 + beta0 p_k
        const double beta0 = s[k] / (s_prev[k] * rho_k[k]);
        S.coef[0] = 1.0 - beta0 * S.res[0] / rho0;
        S.coef[1] = -beta0 * S.res[1] / rho0;
        S.coef[2] = beta0;
        S.coef[3] = 0.0;
      } else {
        S.coef[0] = 1.0;
        S.coef[1] = 0.0;
        S.coef[2] = 0.0;
        S.coef[3] = 0.0;
      }
      const double stop_a = delta * delta;
      const double stop_b = std::pow(0.5 * prm.tol * en[k] / std::max(s[k], 1e-300), 2);
      S.stop2 = std::max(stop_a, stop_b);
      // every cycle after the first may take at most twice the first one's count
      n_cap[k] = n_first[k] < 0 ? kmax : std::min(kmax, std::max(2 * n_first[k], 50));
      S.kmax = std::max(1, std::min(n_cap[k], prm.max_iter - used[k]));
      S.iters = 0;
      S.done = conv[k] ? 1 : 0;
      S.active = 0;
      S.status = DIRAC_OK;
    }
    rc = c.push();
    if (rc != DIRAC_OK) return rc;
    rc = hip_status(axpby(c.vg, n, R0, PLO, c.dstate, 0, 0, 0, 0, c.st), "restart direction");
    if (rc != DIRAC_OK) return rc;
    rc = hip_status(zero(c.vg, n, PSI, c.st), "zero");
    if (rc != DIRAC_OK) return rc;

    rc = run_iterations(c, c.lo, c.Ulo, PSI, PLO, R0, TLO, check_every);
    if (rc != DIRAC_OK) return rc;
    for (int k = 0; k < n; ++k) {
      CgState& S = c.hstate[k];
      if (conv[k]) continue;
      stats[k].iters += S.iters;
      stats[k].dslash_lo += 2 * S.iters;
      used[k] += S.iters;
      rho_k[k] = S.rho;
      if (n_first[k] < 0) n_first[k] = S.iters;
      const bool hit_cap = S.iters >= n_cap[k] && S.rho >= S.stop2;
      capped[k] = hit_cap ? capped[k] + 1 : 0;
      // x += s psi
      S.coef[0] = s[k];
      S.coef[1] = 0.0;
      S.coef[2] = 1.0;
      S.coef[3] = 0.0;
    }
    for (int k = 0; k < n; ++k)
      if (conv[k]) {
        c.hstate[k].coef[0] = 0.0;
        c.hstate[k].coef[1] = 0.0;
        c.hstate[k].coef[2] = 1.0;
        c.hstate[k].coef[3] = 0.0;
      }
    rc = c.push();
    if (rc != DIRAC_OK) return rc;
    rc = hip_status(axpby(c.vg, n, PSI, X, c.dstate, 0, 0, 0, 0, c.st), "accumulate");
    if (rc != DIRAC_OK) return rc;
    rc = true_residual(c, eta, x, kFinPlain);
    if (rc != DIRAC_OK) return rc;
    rc = c.pull();
    if (rc != DIRAC_OK) return rc;
    bool stagnated = false;
    for (int k = 0; k < n; ++k) {
      if (conv[k]) continue;
      stats[k].dslash_hi += 2;
      stats[k].outer += 1;
      s_prev[k] = s[k];
      s[k] = norm_of(c.hstate[k].res[0]);
      stats[k].true_rel_res = s[k] / en[k];
      have_p[k] = true;
      if (s[k] < prm.tol * en[k]) {
        conv[k] = true;
        stats[k].status = DIRAC_OK;
        continue;
      }
      if (s[k] < s_best[k]) {
        s_best[k] = s[k];
        stall[k] = 0;
      } else if (++stall[k] >= 3) {
        have_p[k] = false;  // restart without the carried direction
      }
      // the low-precision operator is too far from the float64 one: six
      // cycles without progress, or two inner solves in a row that stopped at
      // their iteration cap
      if (stall[k] >= 6 || capped[k] >= 2) stagnated = true;
    }
    if (stagnated) {
      *fallback = true;  // finish in float64
      for (int k = 0; k < n; ++k)
        if (!conv[k]) stats[k].fallback = stats[k].outer;
      return DIRAC_OK;
    }
  }
}

// Validation and context of a solve (cg_solve and cg_solve_eo).
int prepare(const dirac_op* op_hi, const void* U_hi, const void* U_lo, const void* eta, void* x, void* work,
            int64_t work_bytes, const cg_params* params, cg_stats* stats_out, bool eo, const char* what, Ctx& c,
            cg_params& prm, void* stream) {
  OpInfo hi;
  int rc = check_op(op_hi, &hi, what);
  if (rc != DIRAC_OK) return rc;
  if (hi.prec != DIRAC_F64) return set_error(DIRAC_EINVAL, "%s: op_hi must be DIRAC_F64", what);
  if (params == nullptr || stats_out == nullptr) return set_error(DIRAC_EINVAL, "%s: NULL params/stats", what);
  prm = *params;
  if (!(prm.tol > 0) || !std::isfinite(prm.tol)) return set_error(DIRAC_EINVAL, "%s: tol must be > 0", what);
  if (prm.max_iter < 1) return set_error(DIRAC_EINVAL, "%s: max_iter must be >= 1", what);
  if (!std::isfinite(prm.inner_delta)) return set_error(DIRAC_EINVAL, "%s: inner_delta must be finite", what);
  if (prm.single_launch < -1 || prm.single_launch > 1 || prm.reserved != 0)
    return set_error(DIRAC_EINVAL, "%s: single_launch must be -1, 0 or 1 and reserved 0", what);
  const int ip = prm.inner_prec;
  if (ip != DIRAC_F64 && ip != DIRAC_F32 && ip != DIRAC_F16S && ip != DIRAC_BF16S)
    return set_error(DIRAC_EINVAL, "%s: unknown inner_prec %d", what, ip);
  if (!U_hi || !eta || !x || !work) return set_error(DIRAC_EINVAL, "%s: NULL buffer", what);
  if (ip != DIRAC_F64 && !U_lo) return set_error(DIRAC_EINVAL, "%s: U_lo is NULL for a mixed solve", what);
  if ((((uintptr_t)U_hi | (uintptr_t)eta | (uintptr_t)x | (uintptr_t)work | (uintptr_t)U_lo) & 255u) != 0)
    return set_error(DIRAC_EINVAL, "%s: buffers must be 256-byte aligned", what);
  Layout L = layout(hi, ip, eo);
  if (work_bytes < L.total)
    return set_error(DIRAC_EWORKSPACE, "%s: workspace needs %lld bytes, got %lld", what, (long long)L.total,
                     (long long)work_bytes);
  const int64_t sb = hi.nrhs * hi.field_stride;
  auto ov = [](const void* a, int64_t na, const void* b, int64_t nb) {
    const char* p = (const char*)a;
    const char* q = (const char*)b;
    return p < q + nb && q < p + na;
  };
  if (ov(eta, sb, x, sb) || ov(work, L.total, x, sb) || ov(work, L.total, eta, sb) ||
      ov(work, L.total, U_hi, hi.gauge_bytes))
    return set_error(DIRAC_EINVAL, "%s: buffers overlap", what);

  c.hi = hi;
  c.lo = hi;
  c.eo = eo;
  c.vg = hi.g;
  if (eo) c.vg.vpar = 0;  // vector operations on the even sites only
  c.single = !eo && (prm.single_launch > 0 || (prm.single_launch == 0 && hi.V <= kSingleLaunchSites));
  if (ip != DIRAC_F64) {
    dirac_op lo = *op_hi;
    lo.prec = ip;
    lo.link = (ip == DIRAC_F32) ? op_hi->link : DIRAC_LINK12;
    rc = check_op(&lo, &c.lo, what);
    if (rc != DIRAC_OK) return rc;
  }
  c.Uhi = U_hi;
  c.Ulo = U_lo;
  c.work = (char*)work;
  c.L = L;
  c.st = (hipStream_t)stream;
  c.dstate = (CgState*)(c.work + L.state);
  c.hstate.assign(kMaxRhs, CgState{});
  std::memset(c.hstate.data(), 0, sizeof(CgState) * kMaxRhs);
  return c.push();
}

// The solve proper on A x = eta (A = D^dag D, or D_hat^dag D_hat in the
// even-odd form): Algorithm 1 with a low-precision inner solve, finishing in
// float64 if that falls back, or plain float64 CG.
int solve_with(Ctx& c, const void* eta, void* x, const cg_params& prm, const std::vector<double>& en,
               std::vector<cg_stats>& stats) {
  const int ip = prm.inner_prec;
  const int check_every = prm.check_every > 0 ? prm.check_every : auto_check_every(ip == DIRAC_F64 ? c.hi : c.lo);
  bool fallback = false;
  int rc = DIRAC_OK;
  if (ip != DIRAC_F64) rc = cg_mixed(c, eta, x, prm, en, stats, check_every, &fallback);
  if (rc == DIRAC_OK && (ip == DIRAC_F64 || fallback)) {
    for (size_t k = 0; k < stats.size(); ++k)
      if (stats[k].status != DIRAC_EBREAKDOWN && en[k] != 0.0) stats[k].status = DIRAC_ENOCONV;
    rc = cg_f64(c, eta, x, prm, en, stats, check_every);
  }
  return rc;
}

}  // namespace

}  // namespace dirac

using namespace dirac;

extern "C" {

int64_t cg_workspace_bytes(const dirac_op* op_hi, const cg_params* params) {
  clear_error();
  OpInfo hi;
  int rc = check_op(op_hi, &hi, "cg_workspace_bytes");
  if (rc != DIRAC_OK) return rc;
  if (params == nullptr) return set_error(DIRAC_EINVAL, "cg_workspace_bytes: params is NULL");
  const int ip = params->inner_prec;
  if (ip != DIRAC_F64 && ip != DIRAC_F32 && ip != DIRAC_F16S && ip != DIRAC_BF16S)
    return set_error(DIRAC_EINVAL, "cg_workspace_bytes: unknown inner_prec %d", ip);
  return layout(hi, ip).total;
}

int cg_solve(const dirac_op* op_hi, const void* U_hi, const void* U_lo, const void* eta, void* x, void* work,
             int64_t work_bytes, const cg_params* params, cg_stats* stats_out, void* stream) {
  clear_error();
  const auto t0 = std::chrono::steady_clock::now();
  Ctx c;
  cg_params prm;
  int rc = prepare(op_hi, U_hi, U_lo, eta, x, work, work_bytes, params, stats_out, false, "cg_solve", c, prm, stream);
  if (rc != DIRAC_OK) return rc;
  const int n = c.hi.nrhs;
  std::vector<cg_stats> stats(n);
  for (auto& s : stats) {
    std::memset(&s, 0, sizeof(s));
    s.status = DIRAC_ENOCONV;
  }
  std::vector<double> en(n, 0.0);
  rc = eta_norms(c, eta, en);
  if (rc == DIRAC_OK) {
    for (int k = 0; k < n; ++k)
      if (!std::isfinite(en[k])) stats[k].status = DIRAC_EBREAKDOWN;
    rc = solve_with(c, eta, x, prm, en, stats);
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int overall = DIRAC_OK;
  for (int k = 0; k < n; ++k) {
    if (en[k] == 0.0 && stats[k].status != DIRAC_EBREAKDOWN) {
      stats[k].status = DIRAC_OK;
      stats[k].true_rel_res = 0.0;
    }
    stats[k].seconds = secs;
    stats_out[k] = stats[k];
    if (overall == DIRAC_OK && stats[k].status != DIRAC_OK) overall = stats[k].status;
  }
  if (rc != DIRAC_OK) return rc;
  if (overall != DIRAC_OK)
    set_error(overall, "cg_solve: not every right-hand side converged (first status %d)", overall);
  return overall;
}

int64_t cg_workspace_bytes_eo(const dirac_op* op_hi, const cg_params* params) {
  clear_error();
  OpInfo hi;
  int rc = check_op(op_hi, &hi, "cg_workspace_bytes_eo");
  if (rc != DIRAC_OK) return rc;
  if (params == nullptr) return set_error(DIRAC_EINVAL, "cg_workspace_bytes_eo: params is NULL");
  const int ip = params->inner_prec;
  if (ip != DIRAC_F64 && ip != DIRAC_F32 && ip != DIRAC_F16S && ip != DIRAC_BF16S)
    return set_error(DIRAC_EINVAL, "cg_workspace_bytes_eo: unknown inner_prec %d", ip);
  return layout(hi, ip, true).total;
}

int cg_solve_eo(const dirac_op* op_hi, const void* U_hi, const void* U_lo, const void* b, void* x, void* work,
                int64_t work_bytes, const cg_params* params, int32_t dagger, cg_stats* stats_out, void* stream) {
  clear_error();
  const auto t0 = std::chrono::steady_clock::now();
  Ctx c;
  cg_params prm;
  int rc = prepare(op_hi, U_hi, U_lo, b, x, work, work_bytes, params, stats_out, true, "cg_solve_eo", c, prm, stream);
  if (rc != DIRAC_OK) return rc;
  const int dag = dagger ? 1 : 0;  // D^dagger x = b: every hop below adjoint
  c.eo_dag = dag;
  const int n = c.hi.nrhs;
  const double A = c.hi.m_q + 4.0;
  void* T = c.work + c.L.t;
  void* EH = c.work + c.L.eh;
  std::vector<cg_stats> stats(n);
  for (auto& s : stats) {
    std::memset(&s, 0, sizeof(s));
    s.status = DIRAC_ENOCONV;
  }
  std::vector<double> bn(n, 0.0), en(n, 0.0), rel(n, std::nan(""));
  std::vector<bool> fin(n, false);

  // |b| on the full lattice
  rc = hip_status(norm2(c.hi.g, n, field_of(c.hi, b), c.red(kFinPlain), c.st), "norm");
  if (rc == DIRAC_OK) rc = c.pull();
  for (int k = 0; rc == DIRAC_OK && k < n; ++k) {
    bn[k] = std::sqrt(c.hstate[k].res[0]);
    if (!std::isfinite(bn[k])) {
      stats[k].status = DIRAC_EBREAKDOWN;
      fin[k] = true;
    } else if (bn[k] == 0.0) {
      stats[k].status = DIRAC_OK;
      fin[k] = true;
    }
  }
  // b_hat = b_e - K_eo b_o / A (even plane of T), then eta_hat = D_hat^dag b_hat
  // (for D^dagger: the adjoint hop, and eta_hat = D_hat b_hat)
  if (rc == DIRAC_OK) rc = hop(c, c.hi, U_hi, b, b, T, 0, dag, 1.0, -1.0 / A, kEpiStore, kGateNone, kFinPlain);
  if (rc == DIRAC_OK) rc = hop(c, c.hi, U_hi, T, nullptr, T, 1, 1 - dag, 0.0, 1.0, kEpiStore, kGateNone, kFinPlain);
  if (rc == DIRAC_OK) rc = hop(c, c.hi, U_hi, T, T, EH, 0, 1 - dag, A, -1.0 / A, kEpiStore, kGateNone, kFinPlain);
  if (rc == DIRAC_OK) rc = eta_norms(c, EH, en);

  // The CG stops on the residual of the normal equations; its tolerance
  // starts below the target (||b - D x|| usually ends a few times above
  // it) and is tightened, resuming from x, while a source misses the target.
  double tol_n = 0.25 * prm.tol;
  for (int pass = 0; rc == DIRAC_OK && pass < 6; ++pass) {
    std::vector<double> en_pass(n);
    for (int k = 0; k < n; ++k) en_pass[k] = fin[k] ? 0.0 : en[k];  // 0: nothing left to do
    cg_params pp = prm;
    pp.tol = tol_n;
    rc = solve_with(c, EH, x, pp, en_pass, stats);
    if (rc != DIRAC_OK) break;
    // x_o = (b_o - K_oe x_e) / A, then r = b - D x on the full lattice
    rc = hop(c, c.hi, U_hi, x, b, x, 1, dag, 1.0 / A, -1.0 / A, kEpiStore, kGateNone, kFinPlain);
    if (rc != DIRAC_OK) break;
    DslashArgs a = dslash_args(c.hi, U_hi, x, T);
    rc = run_dslash(DIRAC_F64, DIRAC_F64, c.hi.link, dag, kEpiStore, launch_cfg(c.hi), a, c.st);
    if (rc != DIRAC_OK) break;
    const FieldRef TR = field_of(c.hi, T);
    rc = hip_status(axpby(c.hi.g, n, field_of(c.hi, b), TR, nullptr, 1.0, 0.0, -1.0, 0.0, c.st), "residual");
    if (rc == DIRAC_OK) rc = hip_status(norm2(c.hi.g, n, TR, c.red(kFinPlain), c.st), "norm");
    if (rc == DIRAC_OK) rc = c.pull();
    if (rc != DIRAC_OK) break;
    double worst = 0.0;
    bool more = false;
    for (int k = 0; k < n; ++k) {
      if (fin[k]) continue;
      rel[k] = std::sqrt(c.hstate[k].res[0]) / bn[k];
      stats[k].true_rel_res = rel[k];
      if (!std::isfinite(rel[k]) || stats[k].status == DIRAC_EBREAKDOWN) {
        stats[k].status = DIRAC_EBREAKDOWN;
        fin[k] = true;
      } else if (rel[k] < prm.tol) {
        stats[k].status = DIRAC_OK;
        fin[k] = true;
      } else if (stats[k].iters >= prm.max_iter) {
        stats[k].status = DIRAC_ENOCONV;
        fin[k] = true;
      } else {
        stats[k].status = DIRAC_ENOCONV;
        worst = std::max(worst, rel[k] / prm.tol);
        more = true;
      }
    }
    if (!more) break;
    tol_n *= std::min(0.5, std::max(1e-4, 0.5 / worst));
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int overall = DIRAC_OK;
  for (int k = 0; k < n; ++k) {
    stats[k].true_rel_res = rel[k];  // the full-lattice residual (a later pass resets finished sources')
    if (bn[k] == 0.0 && stats[k].status != DIRAC_EBREAKDOWN) {
      stats[k].status = DIRAC_OK;
      stats[k].true_rel_res = 0.0;
    }
    stats[k].seconds = secs;
    stats_out[k] = stats[k];
    if (overall == DIRAC_OK && stats[k].status != DIRAC_OK) overall = stats[k].status;
  }
  if (rc != DIRAC_OK) return rc;
  if (overall != DIRAC_OK)
    set_error(overall, "cg_solve_eo: not every right-hand side converged (first status %d)", overall);
  return overall;
}

}  // extern "C"
