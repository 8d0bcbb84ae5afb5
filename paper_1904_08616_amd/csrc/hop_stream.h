// t-streaming form of the half-lattice hop (the even-odd form of eq. (1)).
//
// The hop writes the sites of one parity P and reads `in` on the other.  In
// one x row at one time slice the two parities alternate, so a thread owns a
// pair of x columns (2 xh, 2 xh + 1) of a tile (all of x, tile_y rows,
// tile_z planes) and walks t: at slice t one site of its pair, x_o, has
// parity P and is the output, the other, x_i = x_o ^ 1, is an input site.
// Each step the block stages the input sites of slice t in LDS, one per
// thread, so that
//   * the x neighbours of x_o are the input sites of the same pair and of the
//     pair on the side x_o faces (x_o even: pairs xh and xh - 1; odd: xh + 1
//     and xh);
//   * its y and z neighbours are the input sites of the same pair in the
//     neighbouring rows and planes (the parity flips with y and z), read from
//     LDS inside the tile and from memory at its faces;
//   * its t neighbours (x_o, t +- 1) are this thread's own input sites of the
//     next and the previous slice: psi(x_o, t + 1) is loaded one step ahead
//     (it becomes the next slice's LDS entry), and the backward t hop of the
//     next step's output x_i is formed while U_t(x_i, t) and psi(x_i, t) are
//     at hand and carried over.
// Every input spinor is read from memory once per sweep (plus the tile
// faces), every link once, as in the per-site hop.  When the tile is at
// least 2 deep in y and z (one y and one z face per thread), the face
// spinors of the next slice are requested at the start of a step, when the
// neighbouring tile requests the same spinors as its next slice, and carried
// in registers (AHEAD): the second request then finds them in the L2.
#pragma once

#include "dslash_stream.h"

namespace dirac {

// The tile of the streaming D (tile_y, tile_z, t_chunk) taken by the hop:
// its (X / 2) * tile_y * tile_z column pairs fill a block of 128 or 256
// threads (float32 also 512; spare threads only join the barriers), at least
// 32 of them.
inline int hop_stream_threads(const Geom& g, int sy, int sz) { return g.X / 2 * sy * sz; }
inline bool hop_stream_fits(const Geom& g, int sy, int sz, int tc, int prec) {
  if (prec != DIRAC_F64 && prec != DIRAC_F32) return false;
  if (sy < 1 || sz < 1 || tc < 1 || g.Y % sy || g.Z % sz) return false;
  const int n = hop_stream_threads(g, sy, sz);
  return n >= 32 && n <= (prec == DIRAC_F64 ? 256 : 512);
}
inline int hop_stream_block(const Geom& g, int sy, int sz) {
  const int n = hop_stream_threads(g, sy, sz);
  return n <= 128 ? 128 : (n <= 256 ? 256 : 512);
}
// The hop's tile, from the launch's: a tile of X * tile_y * tile_z columns
// has half as many column pairs, so it is doubled in z, else in y (while it
// divides the lattice and fits the largest block), until its pairs fill at
// least 3/4 of their block.
inline void hop_stream_tile(const Geom& g, int prec, int& sy, int& sz) {
  const int cap = prec == DIRAC_F64 ? 256 : 512;
  while (4 * hop_stream_threads(g, sy, sz) < 3 * hop_stream_block(g, sy, sz)) {
    if (g.Z % (2 * sz) == 0 && hop_stream_threads(g, sy, 2 * sz) <= cap)
      sz *= 2;
    else if (g.Y % (2 * sy) == 0 && hop_stream_threads(g, 2 * sy, sz) <= cap)
      sy *= 2;
    else
      break;
  }
}

// The hop's t_chunk: its blocks hold half the threads and LDS of the D's, so
// several share a CU and the hop wants more of them; it walks the D's
// t_chunk, at most 8 slices (on 32^3 x 64 the D's 32-slice chunks fill one
// block per CU, the hop's 8-slice ones two rounds of two).
inline int hop_stream_chunk(int tc) { return tc < 8 ? tc : 8; }

// out = mass4 * ctr + (hop_c / 2) * acc at output site (P, i) of right-hand
// side rhs, then the epilogue EPI: store, store and the norm pairing the
// exact result with the value as stored (the two differ for the scaled
// 16-bit formats), or dst = src - c out and |dst|^2 (c = alpha or 1).  Both
// hop kernels end with it.
template <int PI, int PO, int EPI>
__device__ __forceinline__ void hop_epilogue(const DslashArgs& a, int rhs, int P, int i,
                                                    const Cx<typename SpinFmt<PI>::R> (&acc)[12], double& val) {
  using SI = SpinFmt<PI>;
  using SO = SpinFmt<PO>;
  using Rl = typename SI::R;
  using Ro = typename SO::R;
  const int Vh = a.g.Vh;
  const Rl ch = (Rl)(0.5 * a.hop_c);
  Cx<Ro> o[12];
  if (a.ctr != nullptr) {
    Cx<Rl> v[12];
    SI::load(make_rsrc(a.ctr + (size_t)rhs * a.ctr_stride, a.field_bytes), Vh, P, i, v);
    const Rl cm = (Rl)a.mass4;
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = {(Ro)fma(cm, v[k].re, ch * acc[k].re), (Ro)fma(cm, v[k].im, ch * acc[k].im)};
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = {(Ro)(ch * acc[k].re), (Ro)(ch * acc[k].im)};
  }
  if constexpr (EPI == kEpiStore || EPI == kEpiStoreNorm) {
    Cx<Ro> q[12];
    SO::store_q(make_rsrc(a.out + (size_t)rhs * a.out_stride, a.out_bytes), Vh, P, i, o, q);
    if constexpr (EPI == kEpiStoreNorm) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 12; ++k) s = fma((double)o[k].im, (double)q[k].im, fma((double)o[k].re, (double)q[k].re, s));
      val += s;
    }
  } else {
    const Ro cf = a.sub_alpha ? (Ro)a.red.state[rhs].alpha : Ro(1);
    Cx<Ro> d[12];
    SO::load(make_rsrc(a.src + (size_t)rhs * a.src_stride, a.out_bytes), Vh, P, i, d);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      d[k].re = fma(-cf, o[k].re, d[k].re);
      d[k].im = fma(-cf, o[k].im, d[k].im);
      s = fma((double)d[k].im, (double)d[k].im, fma((double)d[k].re, (double)d[k].re, s));
    }
    SO::store(make_rsrc(a.out + (size_t)rhs * a.out_stride, a.out_bytes), Vh, P, i, d);
    val += s;
  }
}

// One block's walk over the slices [t0, t1) of its tile (upwards).
template <int PI, int PO, int LK, bool DAG, int EPI, int NC, bool AHEAD>
__device__ __forceinline__ void hop_stream_walk(const DslashArgs& a, int rhs, bool act, int xh, int y, int z, int yl,
                                                int zl, int t0, int t1, char* lds_raw, double& val) {
  using SI = SpinFmt<PI>;
  using LF = LinkFmt<PI, LK>;
  using Rl = typename SI::R;
  constexpr int S = DAG ? -1 : 1;
  const Geom g = a.g;
  const int Vh = g.Vh;
  const int XH = g.X / 2, BY = a.sy, BZ = a.sz;
  const int P = a.par;
  const int tid = threadIdx.x;
  const Rsrc Ur = make_rsrc(a.U, a.U_bytes);
  const Rsrc in = make_rsrc(a.in + (size_t)rhs * a.in_stride, a.field_bytes);
  const int yp = (y + 1 == g.Y) ? 0 : y + 1, ym = (y == 0) ? g.Y - 1 : y - 1;
  const int zp = (z + 1 == g.Z) ? 0 : z + 1, zm = (z == 0) ? g.Z - 1 : z - 1;
  const bool in_yp = yl + 1 < BY, in_ym = yl > 0, in_zp = zl + 1 < BZ, in_zm = zl > 0;
  // LDS slots of the pairs xh + 1 and xh - 1 of this row (periodic in x)
  const int slot_xp = tid + ((xh + 1 == XH) ? 1 - XH : 1), slot_xm = tid + ((xh == 0) ? XH - 1 : -1);
  const int slice = g.X * g.Y * g.Z;
  // index of site (x, yy, zz, t) in its parity plane; its plane is (x + yy + zz + t) & 1
  auto idx = [&](int x, int yy, int zz, int t) { return (t * slice + (zz * g.Y + yy) * g.X + x) >> 1; };
  auto x_out = [&](int t) { return 2 * xh + ((P + y + z + t) & 1); };
  // LDS: two input half-slices [2][12][NC] and, in float64, a slot per
  // thread for the carried hop
  Cx<Rl>* const lbase = reinterpret_cast<Cx<Rl>*>(lds_raw);
  Cx<Rl>* const wslot = lbase + 24 * NC + tid;
  constexpr bool kWtInLds = (PI == DIRAC_F64);
  const int nsteps = t1 - t0;
  // AHEAD: the one y and one z face spinor of the output of each slice,
  // requested a step ahead (tile_y, tile_z >= 2)
  const bool has_fy = !(in_yp && in_ym), has_fz = !(in_zp && in_zm);
  const int fyy = in_yp ? ym : yp, fzz = in_zp ? zm : zp;
  Cx<Rl> fy[12], fz[12];

  // prologue: the input site of slice t0 into buffer 0, and the backward t
  // hop of the first output (x_o, t0) from (x_o, t0 - 1)
  Cx<Rl> Wt[2][3];
  if (act) {
    const int xo = x_out(t0);
    Cx<Rl> v[12];
    SI::load(in, Vh, P ^ 1, idx(xo ^ 1, y, z, t0), v);
    StreamLds<PI, NC>{lbase}.put(tid, v);
    const int tq = (t0 == 0) ? g.T - 1 : t0 - 1;
    const int iq = idx(xo, y, z, tq);
    SI::load(in, Vh, P ^ 1, iq, v);
    M3<Rl> u;
    LF::load(Ur, Vh, P ^ 1, 3, iq, u);  // U_t(x_o, t0 - 1)
    Cx<Rl> h[2][3];
    project<3, S>(v, h);
    su3_dag_mul(u, h, Wt);
    if constexpr (kWtInLds) {
#pragma unroll
      for (int k = 0; k < 6; ++k) wslot[k * NC] = Wt[k / 3][k % 3];
    }
    if constexpr (AHEAD) {
      if (has_fy) SI::load(in, Vh, P ^ 1, idx(xo, fyy, z, t0), fy);
      if (has_fz) SI::load(in, Vh, P ^ 1, idx(xo, y, fzz, t0), fz);
    }
  }
  __syncthreads();

#pragma nounroll
  for (int s = 0; s < nsteps; ++s) {
    const int t = t0 + s;
    const int b = s & 1;
    const StreamLds<PI, NC> cur_s{lbase + b * 12 * NC};        // input sites of slice t
    const StreamLds<PI, NC> nxt_s{lbase + (b ^ 1) * 12 * NC};  // input sites of slice tn
    if (act) {
      const int tn = (t + 1 == g.T) ? 0 : t + 1;
      const int xo = x_out(t), xi = xo ^ 1;
      const bool odd = xo & 1;
      const int io = idx(xo, y, z, t);
      // psi(x_o, tn): the forward t neighbour now, this pair's input site of slice tn next
      Cx<Rl> nxt[12];
      SI::load(in, Vh, P ^ 1, idx(xo, y, z, tn), nxt);
      Cx<Rl> fyn[12], fzn[12];  // AHEAD: the faces of the output (x_i, tn)
      if constexpr (AHEAD) {
        if (s + 1 < nsteps) {
          if (has_fy) SI::load(in, Vh, P ^ 1, idx(xi, fyy, z, tn), fyn);
          if (has_fz) SI::load(in, Vh, P ^ 1, idx(xi, y, fzz, tn), fzn);
        }
      }

      Cx<Rl> acc[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = {Rl(0), Rl(0)};
      if constexpr (kWtInLds) {
#pragma unroll
        for (int k = 0; k < 6; ++k) Wt[k / 3][k % 3] = wslot[k * NC];
      }
      reconstruct_add<3, S>(acc, Wt);  // the backward t hop carried from the previous step
      {
        M3<Rl> u;
        Cx<Rl> v[12];
        // x: forward neighbour x_o + 1, backward x_o - 1 (link of that site)
        LF::load(Ur, Vh, P, 0, io, u);
        cur_s.get(odd ? slot_xp : tid, v);
        hop_apply<0, DAG, true>(u, v, acc);
        {
          const int xb = (xo == 0) ? g.X - 1 : xo - 1;
          LF::load(Ur, Vh, P ^ 1, 0, idx(xb, y, z, t), u);
        }
        cur_s.get(odd ? tid : slot_xm, v);
        hop_apply<0, DAG, false>(u, v, acc);
        nxt_s.put(tid, nxt);
        pin12(acc);
        // y
        LF::load(Ur, Vh, P, 1, io, u);
        if (in_yp) {
          cur_s.get(tid + XH, v);
        } else if constexpr (AHEAD) {
#pragma unroll
          for (int k = 0; k < 12; ++k) v[k] = fy[k];
        } else {
          SI::load(in, Vh, P ^ 1, idx(xo, yp, z, t), v);
        }
        hop_apply<1, DAG, true>(u, v, acc);
        {
          const int ib = idx(xo, ym, z, t);
          LF::load(Ur, Vh, P ^ 1, 1, ib, u);
          if (in_ym) {
            cur_s.get(tid - XH, v);
          } else if constexpr (AHEAD) {
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] = fy[k];
          } else {
            SI::load(in, Vh, P ^ 1, ib, v);
          }
        }
        hop_apply<1, DAG, false>(u, v, acc);
        pin12(acc);
        // z
        LF::load(Ur, Vh, P, 2, io, u);
        if (in_zp) {
          cur_s.get(tid + XH * BY, v);
        } else if constexpr (AHEAD) {
#pragma unroll
          for (int k = 0; k < 12; ++k) v[k] = fz[k];
        } else {
          SI::load(in, Vh, P ^ 1, idx(xo, y, zp, t), v);
        }
        hop_apply<2, DAG, true>(u, v, acc);
        {
          const int ib = idx(xo, y, zm, t);
          LF::load(Ur, Vh, P ^ 1, 2, ib, u);
          if (in_zm) {
            cur_s.get(tid - XH * BY, v);
          } else if constexpr (AHEAD) {
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] = fz[k];
          } else {
            SI::load(in, Vh, P ^ 1, ib, v);
          }
        }
        hop_apply<2, DAG, false>(u, v, acc);
        pin12(acc);
        // t: the forward hop from psi(x_o, tn), and the backward hop of the
        // next output (x_i, tn) from (x_i, t), carried over
        LF::load(Ur, Vh, P, 3, io, u);  // U_t(x_o, t)
        nxt_s.get(tid, v);               // psi(x_o, tn), back from LDS (not kept in registers)
        hop_apply<3, DAG, true>(u, v, acc);
        LF::load(Ur, Vh, P ^ 1, 3, idx(xi, y, z, t), u);  // U_t(x_i, t)
        cur_s.get(tid, v);
        Cx<Rl> h[2][3];
        project<3, S>(v, h);
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
      hop_epilogue<PI, PO, EPI>(a, rhs, P, io, acc, val);
    }  // act
    __syncthreads();  // slice tn complete; slice t no longer read
  }
}

template <int PI, int PO, int LK, bool DAG, int EPI, int NC, bool AHEAD = false>
__global__ void __launch_bounds__(NC)
__attribute__((amdgpu_waves_per_eu(PI == DIRAC_F64 ? (AHEAD ? 1 : 2) : (AHEAD ? 2 : DIRAC_STREAM_WAVES_F32))))
k_hop_stream(DslashArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  const Geom g = a.g;
  const int XH = g.X / 2, BY = a.sy, BZ = a.sz;
  const int tid = threadIdx.x;
  const bool act = tid < XH * BY * BZ;
  const int xh = tid % XH;
  const int yl = (tid / XH) % BY;
  const int zl = tid / (XH * BY);
  const int nty = g.Y / BY, ntz = g.Z / BZ;
  const int ntt = a.ntiles / (nty * ntz);
  // blocks = tiles x right-hand sides, the right-hand side fastest
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
  const int t0 = tt * a.tc;
  const int t1 = min(t0 + a.tc, g.T);
  bool on = true;
  if (a.gate == kGateNotDone) on = !a.red.state[rhs].done;
  if (a.gate == kGateActive) on = a.red.state[rhs].active != 0;
  double vals[1][1] = {{0.0}};
  if (on)
    hop_stream_walk<PI, PO, LK, DAG, EPI, NC, AHEAD>(a, rhs, act, xh, ty * BY + yl, tz * BZ + zl, yl, zl, t0, t1,
                                                     lds_raw, vals[0][0]);
  if constexpr (EPI != kEpiStore) block_reduce_store<1, 1>(a.red, vals, rhs, a.nrhs, l, a.ntiles);
}

// Launch over the tile (a.sy, a.sz, a.tc) that hop_stream_fits accepts.
template <int PI, int PO, int LK, bool DAG, int EPI>
hipError_t launch_hop_stream(DslashArgs a, hipStream_t st) {
  if (!hop_stream_fits(a.g, a.sy, a.sz, a.tc, PI) || a.nrhs < 1) return hipErrorInvalidValue;
  a.ntiles = (a.g.Y / a.sy) * (a.g.Z / a.sz) * ((a.g.T + a.tc - 1) / a.tc);
  a.ngroups = a.nrhs;
  const dim3 grid(a.ntiles * a.nrhs);
  const int nb = hop_stream_block(a.g, a.sy, a.sz);
  const bool ahead = a.sy >= 2 && a.sz >= 2;  // faces one slice ahead (one y and one z face per thread)
  if (nb == 128 && ahead)
    hipLaunchKernelGGL((k_hop_stream<PI, PO, LK, DAG, EPI, 128, true>), grid, dim3(128),
                       (stream_lds_bytes<PI, 128>()), st, a);
  else if (nb == 256 && ahead)
    hipLaunchKernelGGL((k_hop_stream<PI, PO, LK, DAG, EPI, 256, true>), grid, dim3(256),
                       (stream_lds_bytes<PI, 256>()), st, a);
  else if (nb == 128)
    hipLaunchKernelGGL((k_hop_stream<PI, PO, LK, DAG, EPI, 128>), grid, dim3(128), (stream_lds_bytes<PI, 128>()),
                       st, a);
  else if (nb == 256)
    hipLaunchKernelGGL((k_hop_stream<PI, PO, LK, DAG, EPI, 256>), grid, dim3(256), (stream_lds_bytes<PI, 256>()),
                       st, a);
  else if constexpr (PI != DIRAC_F64)
    hipLaunchKernelGGL((k_hop_stream<PI, PO, LK, DAG, EPI, 512>), grid, dim3(512), (stream_lds_bytes<PI, 512>()),
                       st, a);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || EPI == kEpiStore) return e;
  return launch_finalize(a.red, a.ntiles, a.nrhs, 1, st);
}

}  // namespace dirac
