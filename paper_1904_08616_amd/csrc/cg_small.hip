// The CG iteration loop of small lattices in one launch.
//
// On a lattice of a few hundred sites an iteration of the multi-kernel CG
// (D with |Dp|^2, its finalize, D^dagger with the residual update, its
// finalize, the x / p update) is five dependent launches of almost no work,
// and the host polls the scalars between batches.  Here one workgroup runs
// every iteration of one right-hand side: the same three steps separated by
// workgroup barriers, the float64 reductions over the workgroup in a fixed
// order, the scalars in registers.  The recurrence and its stopping and
// breakdown rules are those of the multi-kernel path (cg_finalize): alpha =
// rho / |D p|^2, r -= alpha D^dagger D p, beta = rho' / rho, x += alpha p,
// p = r + beta p, until rho < stop2 or kmax iterations.  The vector formats
// are those of the solver's iteration: the operator's format for p and D p,
// float64 (float64 operator) or float32 (low-precision operator) for x and r.
//
// Nothing is shared between workgroups (each owns one right-hand side), so
// there is no grid-wide synchronisation; every wave leaves the loop at the
// same iteration because the loop condition is computed from the same
// workgroup-wide sums by every thread.  The scalars are never re-read from
// the CgState in memory inside the loop.  One launch runs at most `chunk`
// iterations (it then stores the state and the host launches again), so a
// launch stays short whatever the iteration cap.
#include "lib.h"

namespace dirac {

namespace {

constexpr int kSmallBlock = 512;

struct SmallCgArgs {
  Geom g;
  const char* U;
  uint32_t U_bytes;
  uint32_t op_bytes;   // one field in the operator's format (p, t)
  uint32_t vec_bytes;  // one field in the vector format (x, r)
  int64_t op_stride, vec_stride;
  char* x;
  char* p;
  char* r;
  char* t;
  double mass4;
  CgState* state;
  int chunk;  // iterations per launch at most
};

// Sum over the workgroup, the same value in every thread (fixed order).
__device__ __forceinline__ double wg_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kSmallBlock / 64; ++w) s += red[w];
  __syncthreads();  // red is reused by the next sum
  return s;
}

// D (or D^dagger) of `in` at site (p, i): (m_q + 4) in(n) + 1/2 sum of hops.
template <int P, int LK, bool DAG>
__device__ __forceinline__ void site_op(const DslashArgs& da, Rsrc Ur, Rsrc in, int p, int i,
                                        Cx<typename SpinFmt<P>::R> (&o)[12]) {
  using SF = SpinFmt<P>;
  using Rl = typename SF::R;
  const Coord c = cb_coords(da.g, p, i);
  const Rsrc inr[1] = {in};
  const bool on[1] = {true};
  Cx<Rl> acc[1][12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[0][k] = {Rl(0), Rl(0)};
  hop_dir<P, LK, DAG, 1, 0>(da, Ur, inr, c, p, i, on, acc);
  hop_dir<P, LK, DAG, 1, 1>(da, Ur, inr, c, p, i, on, acc);
  hop_dir<P, LK, DAG, 1, 2>(da, Ur, inr, c, p, i, on, acc);
  hop_dir<P, LK, DAG, 1, 3>(da, Ur, inr, c, p, i, on, acc);
  Cx<Rl> v[12];
  SF::load(in, da.g.Vh, p, i, v);
  const Rl m4 = (Rl)da.mass4, half = Rl(0.5);
#pragma unroll
  for (int k = 0; k < 12; ++k)
    o[k] = {fma(m4, v[k].re, half * acc[0][k].re), fma(m4, v[k].im, half * acc[0][k].im)};
}

template <int P, int LK>
__global__ void __launch_bounds__(kSmallBlock) k_cg_small(SmallCgArgs a) {
  using SO = SpinFmt<P>;                                      // p, t
  constexpr int PV = (P == DIRAC_F64) ? DIRAC_F64 : DIRAC_F32;  // x, r
  using SV = SpinFmt<PV>;
  using Ro = typename SO::R;
  using Rv = typename SV::R;
  __shared__ double red[kSmallBlock / 64];
  const int rhs = blockIdx.x;
  const int Vh = a.g.Vh;
  const int V = 2 * Vh;
  CgState S = a.state[rhs];
  if (S.done) {
    if (threadIdx.x == 0) {
      a.state[rhs].active = 0;
      a.state[rhs].alpha = 0.0;
    }
    return;
  }
  DslashArgs da{};
  da.g = a.g;
  da.mass4 = a.mass4;
  const Rsrc Ur = make_rsrc(a.U, a.U_bytes);
  const Rsrc xr = make_rsrc(a.x + (size_t)rhs * a.vec_stride, a.vec_bytes);
  const Rsrc rr = make_rsrc(a.r + (size_t)rhs * a.vec_stride, a.vec_bytes);
  const Rsrc pr = make_rsrc(a.p + (size_t)rhs * a.op_stride, a.op_bytes);
  const Rsrc tr = make_rsrc(a.t + (size_t)rhs * a.op_stride, a.op_bytes);
  double rho = S.rho, alpha = 0.0, beta = 0.0;
  int iters = S.iters, done = 0, status = S.status, active = 0;
  const int last = iters + a.chunk;

#pragma nounroll
  while (true) {
    // t = D p and <p, D^dag D p> = |t|^2 (the exact value paired with the stored one)
    double s = 0.0;
    for (int n = threadIdx.x; n < V; n += kSmallBlock) {
      const int p = n >= Vh ? 1 : 0, i = n - p * Vh;
      Cx<Ro> o[12];
      site_op<P, LK, false>(da, Ur, pr, p, i, o);
      Cx<Ro> q[12];  // the value as stored
      SO::store_q(tr, Vh, p, i, o, q);
#pragma unroll
      for (int k = 0; k < 12; ++k) s = fma((double)o[k].im, (double)q[k].im, fma((double)o[k].re, (double)q[k].re, s));
    }
    s = wg_sum(s, red);  // its barriers also publish t to the workgroup
    if (!(s > 0.0) || !isfinite(s) || !isfinite(rho)) {
      done = 1;
      status = DIRAC_EBREAKDOWN;
      active = 0;
      alpha = 0.0;
      break;
    }
    active = 1;
    alpha = rho / s;

    // r -= alpha D^dag t, rho' = |r|^2
    double s2 = 0.0;
    for (int n = threadIdx.x; n < V; n += kSmallBlock) {
      const int p = n >= Vh ? 1 : 0, i = n - p * Vh;
      Cx<Ro> w[12];
      site_op<P, LK, true>(da, Ur, tr, p, i, w);
      Cx<Rv> d[12];
      SV::load(rr, Vh, p, i, d);
      const Rv cf = (Rv)alpha;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        d[k].re = fma(-cf, (Rv)w[k].re, d[k].re);
        d[k].im = fma(-cf, (Rv)w[k].im, d[k].im);
        s2 = fma((double)d[k].im, (double)d[k].im, fma((double)d[k].re, (double)d[k].re, s2));
      }
      SV::store(rr, Vh, p, i, d);
    }
    s2 = wg_sum(s2, red);
    if (!isfinite(s2)) {
      done = 1;
      status = DIRAC_EBREAKDOWN;
      beta = 0.0;
    } else {
      beta = s2 / rho;
      rho = s2;
    }
    iters += 1;

    // x += alpha p; p = r + beta p (each thread its own sites)
    for (int n = threadIdx.x; n < V; n += kSmallBlock) {
      const int p = n >= Vh ? 1 : 0, i = n - p * Vh;
      Cx<Rv> xv[12], rv[12];
      Cx<Ro> pv[12];
      SV::load(xr, Vh, p, i, xv);
      SO::load(pr, Vh, p, i, pv);
      SV::load(rr, Vh, p, i, rv);
      const Rv al = (Rv)alpha;
      const Ro be = (Ro)beta;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        xv[k].re = fma(al, (Rv)pv[k].re, xv[k].re);
        xv[k].im = fma(al, (Rv)pv[k].im, xv[k].im);
        pv[k].re = fma(be, pv[k].re, (Ro)rv[k].re);
        pv[k].im = fma(be, pv[k].im, (Ro)rv[k].im);
      }
      SV::store(xr, Vh, p, i, xv);
      SO::store(pr, Vh, p, i, pv);
    }
    if (rho < S.stop2 || iters >= S.kmax) done = 1;
    if (done || iters >= last) break;
    __syncthreads();  // p complete before the next D p reads its neighbours
  }
  if (threadIdx.x == 0) {
    CgState& o = a.state[rhs];
    o.rho = rho;
    o.alpha = alpha;
    o.beta = beta;
    o.iters = iters;
    o.done = done;
    o.status = status;
    o.active = active;
  }
}

template <int P, int LK>
hipError_t launch_small(const SmallCgArgs& a, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_cg_small<P, LK>), dim3(nrhs), dim3(kSmallBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace

int cg_small_iterations(const OpInfo& o, const void* U, FieldRef x, FieldRef p, FieldRef r, FieldRef t,
                        CgState* state, int chunk, hipStream_t st) {
  const int pv = (o.prec == DIRAC_F64) ? DIRAC_F64 : DIRAC_F32;
  if (p.prec != o.prec || t.prec != o.prec || x.prec != pv || r.prec != pv)
    return set_error(DIRAC_EUNSUPPORTED, "single-launch CG: unexpected vector formats");
  SmallCgArgs a;
  a.g = o.g;
  a.U = (const char*)U;
  a.U_bytes = o.gauge_bytes;
  a.op_bytes = p.bytes;
  a.vec_bytes = x.bytes;
  a.op_stride = p.stride;
  a.vec_stride = x.stride;
  a.x = x.ptr;
  a.p = p.ptr;
  a.r = r.ptr;
  a.t = t.ptr;
  a.mass4 = o.m_q + 4.0;
  a.state = state;
  a.chunk = chunk;
  hipError_t e;
  if (o.prec == DIRAC_F64 && o.link == 18) e = launch_small<DIRAC_F64, 18>(a, o.nrhs, st);
  else if (o.prec == DIRAC_F64 && o.link == 12) e = launch_small<DIRAC_F64, 12>(a, o.nrhs, st);
  else if (o.prec == DIRAC_F32 && o.link == 18) e = launch_small<DIRAC_F32, 18>(a, o.nrhs, st);
  else if (o.prec == DIRAC_F32 && o.link == 12) e = launch_small<DIRAC_F32, 12>(a, o.nrhs, st);
  else if (o.prec == DIRAC_F16S && o.link == 12) e = launch_small<DIRAC_F16S, 12>(a, o.nrhs, st);
  else if (o.prec == DIRAC_BF16S && o.link == 12) e = launch_small<DIRAC_BF16S, 12>(a, o.nrhs, st);
  else return set_error(DIRAC_EUNSUPPORTED, "single-launch CG: no kernel for prec %d link %d", o.prec, o.link);
  return hip_status(e, "single-launch CG");
}

}  // namespace dirac
