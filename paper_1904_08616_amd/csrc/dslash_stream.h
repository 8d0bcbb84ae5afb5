// t-streaming variant of the eq. (1) stencil with LDS staging.
//
// A block owns a tile of (x, y, z) columns -- all of x, tile_y rows of y,
// tile_z planes of z -- one thread per column, and walks t_chunk consecutive
// time slices.  At each slice the block's spinors psi(t) sit in LDS, so the
// x, y and z neighbours of a site are read from LDS (only the y and z faces
// of the tile reach to global memory); the t neighbours never leave the
// thread: psi(t+1) is loaded one slice ahead and becomes the next slice's
// centre, and the backward-t hop U_t(n)^dag (1 +- gamma_t) psi(n) is formed
// while U_t(n) and psi(n) are in registers and carried to site n + t.
// Every spinor is therefore read from memory about once per sweep instead
// of up to nine times, and every U_t once instead of twice; the U_x, U_y,
// U_z of a site are read by its own thread and again (backward hop) by the
// neighbour thread a few instructions later, which the caches serve.  The
// walk can run downwards in t as well (mirror image), so that the two
// chunks on either side of a chunk boundary fetch the slices and links they
// share at the same moment and the L2 serves the second reader.
#pragma once

#include "dslash_impl.h"

namespace dirac {

// [12 components][NC columns] complex; NC is a compile-time constant so
// that the component stride is an immediate offset of the LDS instruction.
template <int PI, int NC>
struct StreamLds {
  using R = typename SpinFmt<PI>::R;
  Cx<R>* base;
  __device__ __forceinline__ void put(int col, const Cx<R> (&v)[12]) const {
    Cx<R>* b = base + col;
#pragma unroll
    for (int k = 0; k < 12; ++k) b[k * NC] = v[k];
  }
  __device__ __forceinline__ void get(int col, Cx<R> (&v)[12]) const {
    const Cx<R>* b = base + col;
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = b[k * NC];
  }
};

// Complete the accumulation up to this point and keep the scheduler from
// moving loads of later hops above it (bounds the registers in flight).
template <class R>
__device__ __forceinline__ void pin12(Cx<R> (&acc)[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(acc[k].re), "+v"(acc[k].im));
  __builtin_amdgcn_sched_barrier(0);
}

// One hop of eq. (1) from an already loaded neighbour spinor v:
// FWD: acc += U (1 - S gamma_mu) v;  backward: acc += U^dag (1 + S gamma_mu) v.
// MIX (links held as decoded 16-bit values): the colour products as chains
// of fused multiply-adds from an opaque zero, which read the 16-bit link
// entries directly.
template <int MU, bool DAG, bool FWD, bool MIX = false, class R>
__device__ __forceinline__ void hop_apply(const M3<R>& u, const Cx<R> (&v)[12], Cx<R> (&acc)[12]) {
  constexpr int S = DAG ? -1 : 1;
  Cx<R> h[2][3], w[2][3];
  R zero = R(0);
  if constexpr (MIX) asm("" : "+v"(zero));
  if constexpr (FWD) {
    project<MU, -S>(v, h);
    if constexpr (MIX)
      su3_mul_fma(u, h, w, zero);
    else
      su3_mul(u, h, w);
    reconstruct_add<MU, -S>(acc, w);
  } else {
    project<MU, S>(v, h);
    if constexpr (MIX)
      su3_dag_mul_fma(u, h, w, zero);
    else
      su3_dag_mul(u, h, w);
    reconstruct_add<MU, S>(acc, w);
  }
}

#ifndef DIRAC_STREAM_WAVES_F32
#define DIRAC_STREAM_WAVES_F32 3
#endif

// LDS bytes of the streaming kernel per block of NC threads: two slice
// buffers and, in float64, the carried hops.
template <int PI, int NC>
constexpr size_t stream_lds_bytes() {
  using R = typename SpinFmt<PI>::R;
  return (size_t)NC * (PI == DIRAC_F64 ? 30 : 24) * sizeof(Cx<R>);
}

// Launch-order flags of the streaming kernel (DslashArgs::remap bits).
constexpr int kStreamXcd = 1;   // XCD-contiguous block order
constexpr int kStreamTFast = 2; // t-chunks fastest in the block order
constexpr int kStreamAlt = 4;   // odd t-chunks walk downwards
constexpr int kStreamPipe = 8;  // float64: loads one direction ahead (stream_walk's PIPE)
constexpr int kStreamAhead = 16; // float64: face spinors loaded one slice ahead (stream_walk's AHEAD)

// Store the output o of site (p, i) of right-hand side rhs, with the
// epilogue EPI: plain store, store and |o|^2 (of the value as stored), or
// dst = src - c o and |dst|^2 (c = the CG step alpha or 1).
template <int PO, int EPI>
__device__ __forceinline__ void stream_epilogue(const DslashArgs& a, int rhs, int p, int i,
                                                const Cx<typename SpinFmt<PO>::R> (&o)[12], double& val) {
  using SO = SpinFmt<PO>;
  using Ro = typename SO::R;
  const int Vh = a.g.Vh;
  const Rsrc orsrc = make_rsrc(a.out + (size_t)rhs * a.out_stride, a.out_bytes);
  if constexpr (EPI == kEpiStore || EPI == kEpiStoreNorm) {
    Cx<Ro> q[12];  // the value as stored
    if (a.nt_store)
      SO::template store_q<2>(orsrc, Vh, p, i, o, q);
    else
      SO::template store_q<0>(orsrc, Vh, p, i, o, q);
    if constexpr (EPI == kEpiStoreNorm) {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < 12; ++k) sum = fma((double)o[k].im, (double)q[k].im, fma((double)o[k].re, (double)q[k].re, sum));
      val += sum;
    }
  } else {
    const Ro cf = a.sub_alpha ? (Ro)a.red.state[rhs].alpha : Ro(1);
    Cx<Ro> d[12];
    SO::load(make_rsrc(a.src + (size_t)rhs * a.src_stride, a.out_bytes), Vh, p, i, d);
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      d[k].re = fma(-cf, o[k].re, d[k].re);
      d[k].im = fma(-cf, o[k].im, d[k].im);
      sum = fma((double)d[k].im, (double)d[k].im, fma((double)d[k].re, (double)d[k].re, sum));
    }
    SO::template store<0>(orsrc, Vh, p, i, d);
    val += sum;
  }
}

// One block's walk over the slices [t0, t1) of its tile, upwards (DOWN =
// false) or downwards.  The t-link between the centre slice t and the next
// slice tn = t +- 1 is loaded once per step: walking up it is U_t(n), giving
// the forward hop U (1 - S gamma_t) psi(n + t) of site n and the backward
// hop U^dag (1 + S gamma_t) psi(n) carried into n + t; walking down it is
// U_t(n - t), giving the backward hop of n and the forward hop
// U (1 - S gamma_t) psi(n) carried into n - t.  Neighbouring chunks that walk
// in opposite directions read their shared halo slice and link at the same
// time (both at the start, or both at the end of the walk).
//
// AHEAD: a thread's y and z neighbours outside the tile (at most one of each
// when tile_y and tile_z are at least 2) are requested one slice ahead, at
// the start of the step, next to psi(tn), and carried in registers into the
// next step.  The neighbouring tile requests the same spinors as its own
// psi(tn) at the start of that step, so the second request finds them in the
// L2; requested in the step that uses them they come a whole step (more than
// an XCD's L2 of traffic) after the first.
template <int PI, int PO, int LK, bool DAG, int EPI, int NC, bool DOWN, bool AHEAD = false>
__device__ __forceinline__ void stream_walk(const DslashArgs& a, int rhs, bool act, int x, int y, int z, int yl,
                                            int zl, int t0, int t1, char* lds_raw, double& val) {
  using SI = SpinFmt<PI>;
  using SO = SpinFmt<PO>;
  using LF = LinkFmt<PI, LK>;
  using Rl = typename SI::R;
  using Ro = typename SO::R;
  constexpr int S = DAG ? -1 : 1;
  constexpr int SC = DOWN ? -S : S;  // projector sign of the carried hop
  const Geom g = a.g;
  const int Vh = g.Vh;
  const int BY = a.sy, BZ = a.sz;
  const int tid = threadIdx.x;
  const Rsrc Ur = make_rsrc(a.U, a.U_bytes);
  const Rsrc in = make_rsrc(a.in + (size_t)rhs * a.in_stride, a.field_bytes);
  const int xp = (x + 1 == g.X) ? 0 : x + 1, xm = (x == 0) ? g.X - 1 : x - 1;
  const int yp = (y + 1 == g.Y) ? 0 : y + 1, ym = (y == 0) ? g.Y - 1 : y - 1;
  const int zp = (z + 1 == g.Z) ? 0 : z + 1, zm = (z == 0) ? g.Z - 1 : z - 1;
  const int col_xp = tid - x + xp, col_xm = tid - x + xm;
  const bool in_yp = yl + 1 < BY, in_ym = yl > 0, in_zp = zl + 1 < BZ, in_zm = zl > 0;
  // Lexicographic offsets of this thread's (x, y, z) column and of its
  // spatial neighbours within one time slice; a site's index is then
  // (t * X*Y*Z + column) / 2, with t uniform over the block.  Every +-1
  // neighbour has the other parity (all extents are even).
  const int cpar = (x + y + z) & 1;
  const int ccol = (z * g.Y + y) * g.X + x;
  const int ccol_xm = ccol - x + xm;
  const int ccol_yp = ccol + (yp - y) * g.X, ccol_ym = ccol + (ym - y) * g.X;
  const int ccol_zp = ccol + (zp - z) * g.X * g.Y, ccol_zm = ccol + (zm - z) * g.X * g.Y;
  const int slice = g.X * g.Y * g.Z;
  // AHEAD: the one y and one z neighbour column outside the tile, if any
  const int ccol_fy = in_yp ? ccol_ym : ccol_yp, ccol_fz = in_zp ? ccol_zm : ccol_zp;
  const bool has_fy = !(in_yp && in_ym), has_fz = !(in_zp && in_zm);
  Cx<Rl> fy[12], fz[12];
  auto at = [&](int col, int par, int t, int& p, int& i) {
    p = (par + t) & 1;
    i = (t * slice + col) >> 1;
  };
  // LDS: two slice buffers [2][12][NC] (slice t is read while the next one
  // is written) and, in float64, a private slot per thread for the carried hop.
  Cx<Rl>* const lbase = reinterpret_cast<Cx<Rl>*>(lds_raw);
  Cx<Rl>* const wslot = lbase + 24 * NC + tid;
  constexpr bool kWtInLds = (PI == DIRAC_F64);
  const int ts = DOWN ? t1 - 1 : t0;  // first centre slice
  const int nsteps = t1 - t0;

  // prologue: centre psi(ts) into buffer 0 and the hop carried into ts from
  // the slice before it in walking order, kept as w = U^(dag) h (12 reals)
  Cx<Rl> Wt[2][3];
  if (act) {
    int p, i;
    at(ccol, cpar, ts, p, i);
    Cx<Rl> v[12];
    SI::load(in, Vh, p, i, v);
    StreamLds<PI, NC>{lbase}.put(tid, v);
    const int tq = DOWN ? ((ts + 1 == g.T) ? 0 : ts + 1) : ((ts == 0) ? g.T - 1 : ts - 1);
    int pq, iq;
    at(ccol, cpar, tq, pq, iq);
    SI::load(in, Vh, pq, iq, v);
    M3<Rl> u;
    Cx<Rl> h[2][3];
    project<3, SC>(v, h);
    if constexpr (DOWN) {
      LF::load(Ur, Vh, p, 3, i, u);  // U_t(ts) links ts and ts + 1
      su3_mul(u, h, Wt);
    } else {
      LF::load(Ur, Vh, pq, 3, iq, u);  // U_t(ts - 1) links ts - 1 and ts
      su3_dag_mul(u, h, Wt);
    }
    if constexpr (kWtInLds) {
#pragma unroll
      for (int k = 0; k < 6; ++k) wslot[k * NC] = Wt[k / 3][k % 3];
    }
    if constexpr (AHEAD) {
      int pf, jf;
      if (has_fy) {
        at(ccol_fy, cpar ^ 1, ts, pf, jf);
        SI::load(in, Vh, pf, jf, fy);
      }
      if (has_fz) {
        at(ccol_fz, cpar ^ 1, ts, pf, jf);
        SI::load(in, Vh, pf, jf, fz);
      }
    }
  }
  __syncthreads();

#pragma nounroll
  for (int s = 0; s < nsteps; ++s) {
    const int t = DOWN ? ts - s : ts + s;
    const int b = s & 1;
    const StreamLds<PI, NC> cur_s{lbase + b * 12 * NC};        // slice t
    const StreamLds<PI, NC> nxt_s{lbase + (b ^ 1) * 12 * NC};  // slice tn
    if (act) {
    int p, i;
    at(ccol, cpar, t, p, i);
    const int tn = DOWN ? ((t == 0) ? g.T - 1 : t - 1) : ((t + 1 == g.T) ? 0 : t + 1);
    int pn, in_;
    at(ccol, cpar, tn, pn, in_);
    Cx<Rl> nxt[12];
    SI::load(in, Vh, pn, in_, nxt);
    Cx<Rl> fyn[12], fzn[12];  // AHEAD: the faces of slice tn
    if constexpr (AHEAD) {
      if (s + 1 < nsteps) {
        int pf, jf;
        if (has_fy) {
          at(ccol_fy, cpar ^ 1, tn, pf, jf);
          SI::load(in, Vh, pf, jf, fyn);
        }
        if (has_fz) {
          at(ccol_fz, cpar ^ 1, tn, pf, jf);
          SI::load(in, Vh, pf, jf, fzn);
        }
      }
    }

    Cx<Rl> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {Rl(0), Rl(0)};
    if constexpr (kWtInLds) {
#pragma unroll
      for (int k = 0; k < 6; ++k) Wt[k / 3][k % 3] = wslot[k * NC];
    }
    reconstruct_add<3, SC>(acc, Wt);  // the t hop carried from the previous slice
    {
      M3<Rl> u;
      Cx<Rl> v[12];
      // x: both neighbours are in the tile (it spans all of x)
      LF::load(Ur, Vh, p, 0, i, u);
      cur_s.get(col_xp, v);
      hop_apply<0, DAG, true, SI::kScaled>(u, v, acc);
      {
        int pb, ib;
        at(ccol_xm, cpar ^ 1, t, pb, ib);
        LF::load(Ur, Vh, pb, 0, ib, u);
      }
      cur_s.get(col_xm, v);
      hop_apply<0, DAG, false, SI::kScaled>(u, v, acc);
      nxt_s.put(tid, nxt);  // psi(tn) waits in LDS for the t hop and the next step
      pin12(acc);
      // y
      LF::load(Ur, Vh, p, 1, i, u);
      if (in_yp) {
        cur_s.get(tid + g.X, v);
      } else if constexpr (AHEAD) {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = fy[k];
      } else {
        int pf, jf;
        at(ccol_yp, cpar ^ 1, t, pf, jf);
        SI::load(in, Vh, pf, jf, v);
      }
      hop_apply<1, DAG, true, SI::kScaled>(u, v, acc);
      {
        int pb, ib;
        at(ccol_ym, cpar ^ 1, t, pb, ib);
        LF::load(Ur, Vh, pb, 1, ib, u);
        if (in_ym) {
          cur_s.get(tid - g.X, v);
        } else if constexpr (AHEAD) {
#pragma unroll
          for (int k = 0; k < 12; ++k) v[k] = fy[k];
        } else {
          SI::load(in, Vh, pb, ib, v);
        }
      }
      hop_apply<1, DAG, false, SI::kScaled>(u, v, acc);
      pin12(acc);
      // z
      LF::load(Ur, Vh, p, 2, i, u);
      if (in_zp) {
        cur_s.get(tid + g.X * BY, v);
      } else if constexpr (AHEAD) {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = fz[k];
      } else {
        int pf, jf;
        at(ccol_zp, cpar ^ 1, t, pf, jf);
        SI::load(in, Vh, pf, jf, v);
      }
      hop_apply<2, DAG, true, SI::kScaled>(u, v, acc);
      {
        int pb, ib;
        at(ccol_zm, cpar ^ 1, t, pb, ib);
        LF::load(Ur, Vh, pb, 2, ib, u);
        if (in_zm) {
          cur_s.get(tid - g.X * BY, v);
        } else if constexpr (AHEAD) {
#pragma unroll
          for (int k = 0; k < 12; ++k) v[k] = fz[k];
        } else {
          SI::load(in, Vh, pb, ib, v);
        }
      }
      hop_apply<2, DAG, false, SI::kScaled>(u, v, acc);
      pin12(acc);
      // t: the hop from psi(tn) now, and the hop from psi(t) carried to tn
      if constexpr (DOWN)
        LF::load(Ur, Vh, pn, 3, in_, u);  // U_t(n - t)
      else
        LF::load(Ur, Vh, p, 3, i, u);  // U_t(n)
      nxt_s.get(tid, v);
      hop_apply<3, DAG, !DOWN, SI::kScaled>(u, v, acc);
      cur_s.get(tid, v);
      Cx<Rl> h[2][3];
      project<3, SC>(v, h);
      if constexpr (DOWN)
        su3_mul(u, h, Wt);
      else
        su3_dag_mul(u, h, Wt);
      if constexpr (kWtInLds) {
#pragma unroll
        for (int k = 0; k < 6; ++k) wslot[k * NC] = Wt[k / 3][k % 3];
      }
    }

    if constexpr (AHEAD) {
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        fy[k] = fyn[k];
        fz[k] = fzn[k];
      }
    }
    // epilogue at site (p, i) with centre psi(t)
    Cx<Rl> cur[12];
    cur_s.get(tid, cur);
    const Rl m4 = (Rl)a.mass4;
    Cx<Ro> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
      o[k] = {(Ro)fma(m4, cur[k].re, Rl(0.5) * acc[k].re), (Ro)fma(m4, cur[k].im, Rl(0.5) * acc[k].im)};
    stream_epilogue<PO, EPI>(a, rhs, p, i, o, val);
    }  // act
    __syncthreads();  // slice tn complete; slice t no longer read
  }
}

// Links and face spinors of one direction's two hops, loaded one direction
// ahead of the hops that use them (see stream_walk).
template <int PI, int LK>
struct DirLoads {
  using Rl = typename SpinFmt<PI>::R;
  M3<Rl> uf, ub;          // U_mu(n) and U_mu(n - mu)
  Cx<Rl> vf[12], vb[12];  // psi(n + mu), psi(n - mu) where they lie outside the tile
};

// stream_walk with each step as a software pipeline over the directions:
// the links of direction mu + 1 (and its neighbour spinors outside the tile)
// are requested before the hops of direction mu are computed, so that two
// directions' loads are in flight while the wave computes, instead of one
// round trip to memory per direction.  It needs about twice the registers
// (float64: VGPRs and AGPRs of a wave running alone on its SIMD, which the
// LDS of a float64 walk imposes anyway).  AHEAD as in stream_walk: the face
// spinors then come one slice ahead and a direction's requests are its links.
template <int PI, int PO, int LK, bool DAG, int EPI, int NC, bool DOWN, bool AHEAD = false>
__device__ __forceinline__ void stream_walk_pipe(const DslashArgs& a, int rhs, bool act, int x, int y, int z, int yl,
                                            int zl, int t0, int t1, char* lds_raw, double& val) {
  using SI = SpinFmt<PI>;
  using SO = SpinFmt<PO>;
  using LF = LinkFmt<PI, LK>;
  using Rl = typename SI::R;
  using Ro = typename SO::R;
  constexpr int S = DAG ? -1 : 1;
  constexpr int SC = DOWN ? -S : S;  // projector sign of the carried hop
  const Geom g = a.g;
  const int Vh = g.Vh;
  const int BY = a.sy, BZ = a.sz;
  const int tid = threadIdx.x;
  const Rsrc Ur = make_rsrc(a.U, a.U_bytes);
  const Rsrc in = make_rsrc(a.in + (size_t)rhs * a.in_stride, a.field_bytes);
  const int xp = (x + 1 == g.X) ? 0 : x + 1, xm = (x == 0) ? g.X - 1 : x - 1;
  const int yp = (y + 1 == g.Y) ? 0 : y + 1, ym = (y == 0) ? g.Y - 1 : y - 1;
  const int zp = (z + 1 == g.Z) ? 0 : z + 1, zm = (z == 0) ? g.Z - 1 : z - 1;
  const int col_xp = tid - x + xp, col_xm = tid - x + xm;
  const bool in_yp = yl + 1 < BY, in_ym = yl > 0, in_zp = zl + 1 < BZ, in_zm = zl > 0;
  // Lexicographic offsets of this thread's (x, y, z) column and of its
  // spatial neighbours within one time slice; a site's index is then
  // (t * X*Y*Z + column) / 2, with t uniform over the block.  Every +-1
  // neighbour has the other parity (all extents are even).
  const int cpar = (x + y + z) & 1;
  const int ccol = (z * g.Y + y) * g.X + x;
  const int ccol_xm = ccol - x + xm;
  const int ccol_yp = ccol + (yp - y) * g.X, ccol_ym = ccol + (ym - y) * g.X;
  const int ccol_zp = ccol + (zp - z) * g.X * g.Y, ccol_zm = ccol + (zm - z) * g.X * g.Y;
  const int slice = g.X * g.Y * g.Z;
  const int ccol_fy = in_yp ? ccol_ym : ccol_yp, ccol_fz = in_zp ? ccol_zm : ccol_zp;
  const bool has_fy = !(in_yp && in_ym), has_fz = !(in_zp && in_zm);
  Cx<Rl> fy[12], fz[12];
  auto at = [&](int col, int par, int t, int& p, int& i) {
    p = (par + t) & 1;
    i = (t * slice + col) >> 1;
  };
  // LDS: two slice buffers [2][12][NC] (slice t is read while the next one
  // is written) and, in float64, a private slot per thread for the carried hop.
  Cx<Rl>* const lbase = reinterpret_cast<Cx<Rl>*>(lds_raw);
  Cx<Rl>* const wslot = lbase + 24 * NC + tid;
  constexpr bool kWtInLds = (PI == DIRAC_F64);
  const int ts = DOWN ? t1 - 1 : t0;  // first centre slice
  const int nsteps = t1 - t0;

  // prologue: centre psi(ts) into buffer 0 and the hop carried into ts from
  // the slice before it in walking order, kept as w = U^(dag) h (12 reals)
  Cx<Rl> Wt[2][3];
  if (act) {
    int p, i;
    at(ccol, cpar, ts, p, i);
    Cx<Rl> v[12];
    SI::load(in, Vh, p, i, v);
    StreamLds<PI, NC>{lbase}.put(tid, v);
    const int tq = DOWN ? ((ts + 1 == g.T) ? 0 : ts + 1) : ((ts == 0) ? g.T - 1 : ts - 1);
    int pq, iq;
    at(ccol, cpar, tq, pq, iq);
    SI::load(in, Vh, pq, iq, v);
    M3<Rl> u;
    Cx<Rl> h[2][3];
    project<3, SC>(v, h);
    if constexpr (DOWN) {
      LF::load(Ur, Vh, p, 3, i, u);  // U_t(ts) links ts and ts + 1
      su3_mul(u, h, Wt);
    } else {
      LF::load(Ur, Vh, pq, 3, iq, u);  // U_t(ts - 1) links ts - 1 and ts
      su3_dag_mul(u, h, Wt);
    }
    if constexpr (kWtInLds) {
#pragma unroll
      for (int k = 0; k < 6; ++k) wslot[k * NC] = Wt[k / 3][k % 3];
    }
    if constexpr (AHEAD) {
      int pf, jf;
      if (has_fy) {
        at(ccol_fy, cpar ^ 1, ts, pf, jf);
        SI::load(in, Vh, pf, jf, fy);
      }
      if (has_fz) {
        at(ccol_fz, cpar ^ 1, ts, pf, jf);
        SI::load(in, Vh, pf, jf, fz);
      }
    }
  }
  __syncthreads();

#pragma nounroll
  for (int s = 0; s < nsteps; ++s) {
    const int t = DOWN ? ts - s : ts + s;
    const int b = s & 1;
    const StreamLds<PI, NC> cur_s{lbase + b * 12 * NC};        // slice t
    const StreamLds<PI, NC> nxt_s{lbase + (b ^ 1) * 12 * NC};  // slice tn
    if (act) {
    int p, i;
    at(ccol, cpar, t, p, i);
    const int tn = DOWN ? ((t == 0) ? g.T - 1 : t - 1) : ((t + 1 == g.T) ? 0 : t + 1);
    int pn, in_;
    at(ccol, cpar, tn, pn, in_);
    int pxb, ixb, pyf, iyf, pyb, iyb, pzf, izf, pzb, izb;
    at(ccol_xm, cpar ^ 1, t, pxb, ixb);
    at(ccol_yp, cpar ^ 1, t, pyf, iyf);
    at(ccol_ym, cpar ^ 1, t, pyb, iyb);
    at(ccol_zp, cpar ^ 1, t, pzf, izf);
    at(ccol_zm, cpar ^ 1, t, pzb, izb);

    // requests of one direction: its two links and its neighbour spinors
    // outside the tile
    auto req_y = [&](DirLoads<PI, LK>& d) {
      LF::load(Ur, Vh, p, 1, i, d.uf);
      LF::load(Ur, Vh, pyb, 1, iyb, d.ub);
      if constexpr (!AHEAD) {
        if (!in_yp) SI::load(in, Vh, pyf, iyf, d.vf);
        if (!in_ym) SI::load(in, Vh, pyb, iyb, d.vb);
      }
    };
    auto req_z = [&](DirLoads<PI, LK>& d) {
      LF::load(Ur, Vh, p, 2, i, d.uf);
      LF::load(Ur, Vh, pzb, 2, izb, d.ub);
      if constexpr (!AHEAD) {
        if (!in_zp) SI::load(in, Vh, pzf, izf, d.vf);
        if (!in_zm) SI::load(in, Vh, pzb, izb, d.vb);
      }
    };
    auto req_t = [&](M3<Rl>& u) {  // U_t(n - t) walking down, U_t(n) walking up
      if constexpr (DOWN)
        LF::load(Ur, Vh, pn, 3, in_, u);
      else
        LF::load(Ur, Vh, p, 3, i, u);
    };
    // psi(tn) and the x links first
    Cx<Rl> nxt[12];
    SI::load(in, Vh, pn, in_, nxt);
    Cx<Rl> fyn[12], fzn[12];  // AHEAD: the faces of slice tn
    if constexpr (AHEAD) {
      if (s + 1 < nsteps) {
        int pf, jf;
        if (has_fy) {
          at(ccol_fy, cpar ^ 1, tn, pf, jf);
          SI::load(in, Vh, pf, jf, fyn);
        }
        if (has_fz) {
          at(ccol_fz, cpar ^ 1, tn, pf, jf);
          SI::load(in, Vh, pf, jf, fzn);
        }
      }
    }
    M3<Rl> uxf, uxb;
    LF::load(Ur, Vh, p, 0, i, uxf);
    LF::load(Ur, Vh, pxb, 0, ixb, uxb);
    DirLoads<PI, LK> dy, dz;
    M3<Rl> ut;
    req_y(dy);

    Cx<Rl> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {Rl(0), Rl(0)};
    if constexpr (kWtInLds) {
#pragma unroll
      for (int k = 0; k < 6; ++k) Wt[k / 3][k % 3] = wslot[k * NC];
    }
    reconstruct_add<3, SC>(acc, Wt);  // the t hop carried from the previous slice
    {
      Cx<Rl> v[12];
      // x: both neighbours are in the tile (it spans all of x)
      cur_s.get(col_xp, v);
      hop_apply<0, DAG, true, SI::kScaled>(uxf, v, acc);
      cur_s.get(col_xm, v);
      hop_apply<0, DAG, false, SI::kScaled>(uxb, v, acc);
      nxt_s.put(tid, nxt);  // psi(tn) waits in LDS for the t hop and the next step
      pin12(acc);
      req_z(dz);
      // y
      if (in_yp) {
        cur_s.get(tid + g.X, v);
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = AHEAD ? fy[k] : dy.vf[k];
      }
      hop_apply<1, DAG, true, SI::kScaled>(dy.uf, v, acc);
      if (in_ym) {
        cur_s.get(tid - g.X, v);
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = AHEAD ? fy[k] : dy.vb[k];
      }
      hop_apply<1, DAG, false, SI::kScaled>(dy.ub, v, acc);
      pin12(acc);
      req_t(ut);
      // z
      if (in_zp) {
        cur_s.get(tid + g.X * BY, v);
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = AHEAD ? fz[k] : dz.vf[k];
      }
      hop_apply<2, DAG, true, SI::kScaled>(dz.uf, v, acc);
      if (in_zm) {
        cur_s.get(tid - g.X * BY, v);
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = AHEAD ? fz[k] : dz.vb[k];
      }
      hop_apply<2, DAG, false, SI::kScaled>(dz.ub, v, acc);
      pin12(acc);
      // t: the hop from psi(tn) now, and the hop from psi(t) carried to tn
      nxt_s.get(tid, v);
      hop_apply<3, DAG, !DOWN, SI::kScaled>(ut, v, acc);
      cur_s.get(tid, v);
      Cx<Rl> h[2][3];
      project<3, SC>(v, h);
      if constexpr (DOWN)
        su3_mul(ut, h, Wt);
      else
        su3_dag_mul(ut, h, Wt);
      if constexpr (kWtInLds) {
#pragma unroll
        for (int k = 0; k < 6; ++k) wslot[k * NC] = Wt[k / 3][k % 3];
      }
    }

    if constexpr (AHEAD) {
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        fy[k] = fyn[k];
        fz[k] = fzn[k];
      }
    }
    // output of site (p, i) with centre psi(t)
    Cx<Rl> cur[12];
    cur_s.get(tid, cur);
    const Rl m4 = (Rl)a.mass4;
    Cx<Ro> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
      o[k] = {(Ro)fma(m4, cur[k].re, Rl(0.5) * acc[k].re), (Ro)fma(m4, cur[k].im, Rl(0.5) * acc[k].im)};
    stream_epilogue<PO, EPI>(a, rhs, p, i, o, val);
    }  // act
    __syncthreads();  // slice tn complete; slice t no longer read
  }
}

template <int PI, int PO, int LK, bool DAG, int EPI, int NC, bool PIPE = false, bool AHEAD = false>
__global__ void __launch_bounds__(NC)
__attribute__((amdgpu_waves_per_eu(PI == DIRAC_F64 ? (PIPE || AHEAD ? 1 : 2) : DIRAC_STREAM_WAVES_F32)))
k_dslash_stream(DslashArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  const Geom g = a.g;
  const int BY = a.sy, BZ = a.sz;
  const int tid = threadIdx.x;
  // threads past the tile's X * BY * BZ columns only take part in barriers
  const bool act = tid < g.X * BY * BZ;
  const int x = tid % g.X;
  const int yl = (tid / g.X) % BY;
  const int zl = tid / (g.X * BY);
  const int nty = g.Y / BY, ntz = g.Z / BZ;
  const int ntt = a.ntiles / (nty * ntz);
  // blocks = tiles x right-hand sides, the right-hand side fastest: the
  // blocks of one tile run side by side and share its link loads in the L2
  const int lb = xcd_tile(blockIdx.x, a.ntiles * a.nrhs, a.remap & kStreamXcd);
  const int rhs = lb % a.nrhs;
  const int l = lb / a.nrhs;
  int ty, tz, tt;
  if (a.remap & kStreamTFast) {
    tt = l % ntt;
    ty = (l / ntt) % nty;
    tz = l / (ntt * nty);
  } else {
    ty = l % nty;
    tz = (l / nty) % ntz;
    tt = l / (nty * ntz);
  }
  const int y = ty * BY + yl, z = tz * BZ + zl;
  const int t0 = tt * a.tc;
  const int t1 = min(t0 + a.tc, g.T);

  bool on = true;
  if (a.gate == kGateNotDone) on = !a.red.state[rhs].done;
  if (a.gate == kGateActive) on = a.red.state[rhs].active != 0;
  double vals[1][1] = {{0.0}};
  if (on) {
    const bool down = (a.remap & kStreamAlt) && (tt & 1);
    if constexpr (PIPE) {
      if (down)
        stream_walk_pipe<PI, PO, LK, DAG, EPI, NC, true, AHEAD>(a, rhs, act, x, y, z, yl, zl, t0, t1, lds_raw,
                                                                vals[0][0]);
      else
        stream_walk_pipe<PI, PO, LK, DAG, EPI, NC, false, AHEAD>(a, rhs, act, x, y, z, yl, zl, t0, t1, lds_raw,
                                                                 vals[0][0]);
    } else {
      if (down)
        stream_walk<PI, PO, LK, DAG, EPI, NC, true, AHEAD>(a, rhs, act, x, y, z, yl, zl, t0, t1, lds_raw, vals[0][0]);
      else
        stream_walk<PI, PO, LK, DAG, EPI, NC, false, AHEAD>(a, rhs, act, x, y, z, yl, zl, t0, t1, lds_raw,
                                                            vals[0][0]);
    }
  }
  if constexpr (EPI != kEpiStore) block_reduce_store<1, 1>(a.red, vals, rhs, a.nrhs, l, a.ntiles);
}

// Tile/geometry check of the streaming kernel (host): the tile's y and z
// extents divide the lattice's, and its X * tile_y * tile_z columns fit a
// block of 128, 192, 256, 384 or 512 threads (32 to 512 columns, spare
// threads idle; blocks of 192 and 384 fit tiles of a lattice 24 or 48 wide
// in x without idle waves).  Float64 takes up to 256 columns in blocks of
// 128 or 256: the two slice buffers of more would not fit the LDS of a CU.
inline int stream_max_columns(int prec) { return prec == DIRAC_F64 ? 256 : 512; }
inline int stream_columns(const Geom& g, int sy, int sz) { return g.X * sy * sz; }
inline int stream_block(const Geom& g, int sy, int sz, int prec) {
  const int n = stream_columns(g, sy, sz);
  if (prec == DIRAC_F64) return n <= 128 ? 128 : 256;
  for (int b : {128, 192, 256, 384})
    if (n <= b) return b;
  return 512;
}
inline bool stream_fits(const Geom& g, int sy, int sz, int tc, int prec) {
  if (sy < 1 || sz < 1 || tc < 1) return false;
  if (g.Y % sy || g.Z % sz) return false;
  const int n = stream_columns(g, sy, sz);
  return n >= 32 && n <= stream_max_columns(prec);
}
// The walk with faces one slice ahead carries one y and one z face per
// thread: tiles at least 2 deep in y and z.
inline bool stream_ahead_fits(int sy, int sz) { return sy >= 2 && sz >= 2; }

template <int PI, int PO, int LK, bool DAG, int EPI, int NC, bool PIPE, bool AHEAD>
void launch_stream_nc(const DslashArgs& a, dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_dslash_stream<PI, PO, LK, DAG, EPI, NC, PIPE, AHEAD>), grid, dim3(NC),
                     (stream_lds_bytes<PI, NC>()), st, a);
}

template <int PI, int PO, int LK, bool DAG, int EPI>
hipError_t launch_dslash_stream(DslashArgs a, int, hipStream_t st) {
  if (!stream_fits(a.g, a.sy, a.sz, a.tc, PI) || a.nrhs < 1) return hipErrorInvalidValue;
  const int nty = a.g.Y / a.sy, ntz = a.g.Z / a.sz, ntt = (a.g.T + a.tc - 1) / a.tc;
  a.ntiles = nty * ntz * ntt;
  a.ngroups = 1;
  const int nc = stream_block(a.g, a.sy, a.sz, PI);
  const dim3 grid(a.ntiles * a.nrhs);
  if constexpr (PI != DIRAC_F64) {
    if (nc != 128 && nc != 256) {
      if (nc == 192)
        hipLaunchKernelGGL((k_dslash_stream<PI, PO, LK, DAG, EPI, 192>), grid, dim3(192),
                           (stream_lds_bytes<PI, 192>()), st, a);
      else if (nc == 384)
        hipLaunchKernelGGL((k_dslash_stream<PI, PO, LK, DAG, EPI, 384>), grid, dim3(384),
                           (stream_lds_bytes<PI, 384>()), st, a);
      else
        hipLaunchKernelGGL((k_dslash_stream<PI, PO, LK, DAG, EPI, 512>), grid, dim3(512),
                           (stream_lds_bytes<PI, 512>()), st, a);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess || EPI == kEpiStore) return e;
      return launch_finalize(a.red, a.ntiles, a.nrhs, 1, st);
    }
  }
  // float64 walks: bit 3 pipelined, bit 4 faces one slice ahead
  constexpr bool F = PI == DIRAC_F64;
  const bool pipe = F && (a.remap & kStreamPipe);
  const bool ahead = F && (a.remap & kStreamAhead);
  if (ahead && !stream_ahead_fits(a.sy, a.sz)) return hipErrorInvalidValue;
  if (nc == 256) {
    if (pipe && ahead)
      launch_stream_nc<PI, PO, LK, DAG, EPI, 256, F, F>(a, grid, st);
    else if (pipe)
      launch_stream_nc<PI, PO, LK, DAG, EPI, 256, F, false>(a, grid, st);
    else if (ahead)
      launch_stream_nc<PI, PO, LK, DAG, EPI, 256, false, F>(a, grid, st);
    else
      launch_stream_nc<PI, PO, LK, DAG, EPI, 256, false, false>(a, grid, st);
  } else {
    if (pipe && ahead)
      launch_stream_nc<PI, PO, LK, DAG, EPI, 128, F, F>(a, grid, st);
    else if (pipe)
      launch_stream_nc<PI, PO, LK, DAG, EPI, 128, F, false>(a, grid, st);
    else if (ahead)
      launch_stream_nc<PI, PO, LK, DAG, EPI, 128, false, F>(a, grid, st);
    else
      launch_stream_nc<PI, PO, LK, DAG, EPI, 128, false, false>(a, grid, st);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || EPI == kEpiStore) return e;
  return launch_finalize(a.red, a.ntiles, a.nrhs, 1, st);
}

#define DIRAC_DSLASH_STREAM_ENTRY(PI, PO, LK, DAG, EPI) \
  DslashEntry{PI, PO, LK, DAG, EPI, 0, &launch_dslash_stream<PI, PO, LK, DAG, EPI>}

}  // namespace dirac
