// The Wilson-Dirac stencil of eq. (1) as a HIP kernel template.
//
// One thread computes the full output spinor of one lattice site (both
// parities are covered by one launch, so a link read as U_mu(n) by site n is
// read again as U_mu(n)^dag by site n+mu while it is still in cache), for R
// right-hand sides at once: each of the 8 links is loaded and (for 12-real
// storage) rebuilt once per site and applied to all R half spinors.
//
// Per site and hop the steps follow the paper's stencil stages (Kernel
// Description): gather the neighbour spinor, project it to a half spinor
// (the "8 additions and 8 subtractions of vector type"), multiply by the
// link or its adjoint (the SU(3) matrix-vector stage, two products per hop),
// reconstruct the lower spin pair and accumulate; finally scale by 1/2 and
// add (m_q + 4) psi(n).
//
// Epilogues: plain store; store plus the float64 norm^2 of the result
// (CG: <p, D^dag D p> = |D p|^2); or dst = src - c * result plus |dst|^2
// with c = 1 or the CG step alpha (CG: r -= alpha D^dag D p without ever
// storing D^dag D p; true residual: r = eta - D^dag D x).
#pragma once

#include "common.h"

namespace dirac {

enum Epi : int { kEpiStore = 0, kEpiStoreNorm = 1, kEpiSubNorm = 2 };

// Second reduction stage (field.hip): sums partials[rhs][nparts][nc] per
// right-hand side in a fixed order and applies cg_finalize.
hipError_t launch_finalize(const RedArgs& ra, int nparts, int nrhs, int nc, hipStream_t st);
enum Gate : int { kGateNone = 0, kGateNotDone = 1, kGateActive = 2 };

struct DslashArgs {
  Geom g;
  const char* U;
  uint32_t U_bytes;
  uint32_t field_bytes;  // bytes of one spinor field of the input format
  uint32_t out_bytes;    // bytes of one field of the output format
  const char* in;    // input spinor(s), rhs stride in_stride bytes
  int64_t in_stride;
  char* out;         // output (kEpiStore*) or dst (kEpiSubNorm)
  int64_t out_stride;
  const char* src;   // kEpiSubNorm: src of dst = src - c * D in (output format)
  int64_t src_stride;
  double mass4;      // m_q + 4
  int nrhs;
  int remap;         // XCD-aware tile order
  int ntiles;        // 2 * ceil(Vh / blockDim.x)
  int ngroups;       // ceil(nrhs / R)
  int sub_alpha;     // kEpiSubNorm: c = state.alpha (1) or 1 (0)
  int gate;          // Gate
  int nt_store;      // non-temporal output stores (kEpiStore / kEpiStoreNorm)
  int sy, sz, tc;    // streaming kernel: tile rows in y, planes in z, t slices per block
  RedArgs red;
  // half-lattice hop (even-odd form): output parity, centre field and the
  // hop coefficient of out = mass4 * ctr + hop_c * (1/2) sum of hops
  int par;
  const char* ctr;   // null: no centre term
  int64_t ctr_stride;
  double hop_c;
};

template <class To, class From>
__device__ __forceinline__ void convert12(const Cx<From> (&a)[12], Cx<To> (&b)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) b[c] = {(To)a[c].re, (To)a[c].im};
}

// Pin the accumulators at this point of the program: the hop's arithmetic
// must complete here, so the compiler cannot defer every hop's arithmetic to
// the end (which would keep all 8 hops' loaded data live and spill).
template <class Rl, int R>
__device__ __forceinline__ void pin_acc(Cx<Rl> (&acc)[R][12]) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(acc[r][k].re), "+v"(acc[r][k].im));
}

template <int PI, int LK, bool DAG, int R, int MU>
__device__ __forceinline__ void hop_dir(const DslashArgs& a, Rsrc Ur, const Rsrc (&in)[R],
                                        const Coord& c, int p, int i, const bool (&on)[R],
                                        Cx<typename SpinFmt<PI>::R> (&acc)[R][12]) {
  using SI = SpinFmt<PI>;
  using LF = LinkFmt<PI, LK>;
  using Rl = typename SI::R;
  constexpr int S = DAG ? -1 : 1;  // D^dag = eq. (1) with the projectors swapped
  const int Vh = a.g.Vh;
  const int q = p ^ 1;
  {  // forward hop: U_mu(n) (1 - S gamma_mu) psi(n + mu)
    const int j = nb_fwd<MU>(a.g, c, i);
    M3<Rl> u;
    LF::load(Ur, Vh, p, MU, i, u);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!on[r]) continue;
      Cx<Rl> v[12];
      Cx<Rl> h[2][3], w[2][3];
      if constexpr (SI::kScaled) {
        float sc;
        SI::load_raw(in[r], Vh, q, j, v, sc);
        float one = 1.f, zero = 0.f;
        asm("" : "+v"(one), "+v"(zero));
        project_fma1<MU, -S>(v, h, one);
        su3_mul_fma(u, h, w, zero);
        reconstruct_fma<MU, -S>(acc[r], w, sc);
      } else {
        SI::load(in[r], Vh, q, j, v);
        project<MU, -S>(v, h);
        su3_mul(u, h, w);
        reconstruct_add<MU, -S>(acc[r], w);
      }
    }
  }
  pin_acc<Rl, R>(acc);
  {  // backward hop: U_mu(n - mu)^dag (1 + S gamma_mu) psi(n - mu)
    const int j = nb_bwd<MU>(a.g, c, i);
    M3<Rl> u;
    LF::load(Ur, Vh, q, MU, j, u);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!on[r]) continue;
      Cx<Rl> v[12];
      Cx<Rl> h[2][3], w[2][3];
      if constexpr (SI::kScaled) {
        float sc;
        SI::load_raw(in[r], Vh, q, j, v, sc);
        float one = 1.f, zero = 0.f;
        asm("" : "+v"(one), "+v"(zero));
        project_fma1<MU, S>(v, h, one);
        su3_dag_mul_fma(u, h, w, zero);
        reconstruct_fma<MU, S>(acc[r], w, sc);
      } else {
        SI::load(in[r], Vh, q, j, v);
        project<MU, S>(v, h);
        su3_dag_mul(u, h, w);
        reconstruct_add<MU, S>(acc[r], w);
      }
    }
  }
  pin_acc<Rl, R>(acc);
}

// Site work of one thread: (parity p, checkerboard index i), right-hand
// sides rhs0 .. rhs0+R-1 that are switched on.
template <int PI, int PO, int LK, bool DAG, int EPI, int R>
__device__ __forceinline__ void dslash_site(const DslashArgs& a, int p, int i, int rhs0,
                                            const bool (&on)[R], double (&vals)[R][1]) {
  using SI = SpinFmt<PI>;
  using SO = SpinFmt<PO>;
  using Rl = typename SI::R;
  using Ro = typename SO::R;
  const int Vh = a.g.Vh;
  const Coord c = cb_coords(a.g, p, i);
  const Rsrc Ur = make_rsrc(a.U, a.U_bytes);
  Rsrc in[R];
#pragma unroll
  for (int r = 0; r < R; ++r) in[r] = make_rsrc(a.in + (size_t)(rhs0 + r) * a.in_stride, a.field_bytes);
  Cx<Rl> acc[R][12];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r][k] = {Rl(0), Rl(0)};

  hop_dir<PI, LK, DAG, R, 0>(a, Ur, in, c, p, i, on, acc);
  hop_dir<PI, LK, DAG, R, 1>(a, Ur, in, c, p, i, on, acc);
  hop_dir<PI, LK, DAG, R, 2>(a, Ur, in, c, p, i, on, acc);
  hop_dir<PI, LK, DAG, R, 3>(a, Ur, in, c, p, i, on, acc);

  const Rl m4 = (Rl)a.mass4;
  const Rl half = Rl(0.5);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!on[r]) continue;
    const int rhs = rhs0 + r;
    Cx<Rl> v[12];
    SI::load(in[r], Vh, p, i, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      acc[r][k].re = fma(m4, v[k].re, half * acc[r][k].re);
      acc[r][k].im = fma(m4, v[k].im, half * acc[r][k].im);
    }
    Cx<Ro> o[12];
    convert12(acc[r], o);
    if constexpr (EPI == kEpiStore || EPI == kEpiStoreNorm) {
      const Rsrc orsrc = make_rsrc(a.out + (size_t)rhs * a.out_stride, a.out_bytes);
      Cx<Ro> q[12];  // the value as stored
      if (a.nt_store)
        SO::template store_q<2>(orsrc, Vh, p, i, o, q);
      else
        SO::template store_q<0>(orsrc, Vh, p, i, o, q);
      if constexpr (EPI == kEpiStoreNorm) {
        // <p, D^dag t_stored> = Re <D p, t_stored>: pair the exact result with
        // the value as stored, so that the CG step matches the vector the
        // next kernel actually applies D^dag to (they differ for scaled
        // 16-bit formats).
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) s = fma((double)o[k].im, (double)q[k].im, fma((double)o[k].re, (double)q[k].re, s));
        vals[r][0] = s;
      }
    } else {
      const Ro cf = a.sub_alpha ? (Ro)a.red.state[rhs].alpha : Ro(1);
      Cx<Ro> d[12];
      SO::load(make_rsrc(a.src + (size_t)rhs * a.src_stride, a.out_bytes), Vh, p, i, d);
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        d[k].re = fma(-cf, o[k].re, d[k].re);
        d[k].im = fma(-cf, o[k].im, d[k].im);
        s = fma((double)d[k].im, (double)d[k].im, fma((double)d[k].re, (double)d[k].re, s));
      }
      SO::store(make_rsrc(a.out + (size_t)rhs * a.out_stride, a.out_bytes), Vh, p, i, d);
      vals[r][0] = s;
    }
  }
}

// Waves per SIMD the register allocation is sized for (the kernel is bound
// by memory traffic, so occupancy hides latency; more waves than this would
// force spills of the accumulators).
template <int PI, int R>
constexpr int dslash_waves() {
#ifdef DIRAC_DSLASH_WPE
  return DIRAC_DSLASH_WPE;
#else
  return PI == DIRAC_F64 ? (R == 1 ? 3 : 2) : (R == 1 ? 4 : 3);
#endif
}

template <int PI, int PO, int LK, bool DAG, int EPI, int R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(dslash_waves<PI, R>())))
k_dslash(DslashArgs a) {
  const int nblocks = a.ntiles * a.ngroups;
  const int l = xcd_tile(blockIdx.x, nblocks, a.remap);
  const int grp = l % a.ngroups;
  const int tile = l / a.ngroups;
  const int p = tile & 1;
  const int i = (tile >> 1) * blockDim.x + threadIdx.x;
  const int rhs0 = grp * R;

  bool on[R];
  bool any = false;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int rhs = rhs0 + r;
    bool v = rhs < a.nrhs && i < a.g.Vh;
    if (v && a.gate == kGateNotDone) v = !a.red.state[rhs].done;
    if (v && a.gate == kGateActive) v = a.red.state[rhs].active != 0;
    on[r] = v;
    any |= v;
  }
  double vals[R][1];
#pragma unroll
  for (int r = 0; r < R; ++r) vals[r][0] = 0.0;
  if (any) dslash_site<PI, PO, LK, DAG, EPI, R>(a, p, i, rhs0, on, vals);
  if constexpr (EPI != kEpiStore) {
    block_reduce_store<R, 1>(a.red, vals, rhs0, a.nrhs, tile, a.ntiles);
  }
}

// Direction-split variant for lattices too small to fill the device with one
// thread per site: NS waves share a block of 64 sites, wave w applies the
// hops of directions {w} (NS = 4) or {2w, 2w+1} (NS = 2) to all 64 sites,
// the NS partial spinors meet in LDS, and each wave finishes (mass term,
// epilogue, store) its share of the output storage vectors.  NS times more
// waves are in flight for the same lattice, each with a shorter dependency
// chain.  One right-hand side.
template <int PI, int PO, int LK, bool DAG, int EPI, int NS>
__global__ void __launch_bounds__(64 * NS) __attribute__((amdgpu_waves_per_eu(dslash_waves<PI, 1>())))
k_dslash_split(DslashArgs a) {
  using SI = SpinFmt<PI>;
  using SO = SpinFmt<PO>;
  using Rl = typename SI::R;
  using Ro = typename SO::R;
  __shared__ Rl part[NS][24][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int Vh = a.g.Vh;
  const int tile = xcd_tile(blockIdx.x, a.ntiles, a.remap);
  const int p = tile & 1;
  const int i = (tile >> 1) * 64 + lane;
  bool on = i < Vh;
  if (on && a.gate == kGateNotDone) on = !a.red.state[0].done;
  if (on && a.gate == kGateActive) on = a.red.state[0].active != 0;
  Cx<Rl> acc[1][12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[0][k] = {Rl(0), Rl(0)};
  const Rsrc in[1] = {make_rsrc(a.in, a.field_bytes)};
  if (on) {
    const bool onr[1] = {true};
    const Coord c = cb_coords(a.g, p, i);
    const Rsrc Ur = make_rsrc(a.U, a.U_bytes);
    if constexpr (NS == 4) {
      if (wave == 0) hop_dir<PI, LK, DAG, 1, 0>(a, Ur, in, c, p, i, onr, acc);
      else if (wave == 1) hop_dir<PI, LK, DAG, 1, 1>(a, Ur, in, c, p, i, onr, acc);
      else if (wave == 2) hop_dir<PI, LK, DAG, 1, 2>(a, Ur, in, c, p, i, onr, acc);
      else hop_dir<PI, LK, DAG, 1, 3>(a, Ur, in, c, p, i, onr, acc);
    } else {
      if (wave == 0) {
        hop_dir<PI, LK, DAG, 1, 0>(a, Ur, in, c, p, i, onr, acc);
        hop_dir<PI, LK, DAG, 1, 1>(a, Ur, in, c, p, i, onr, acc);
      } else {
        hop_dir<PI, LK, DAG, 1, 2>(a, Ur, in, c, p, i, onr, acc);
        hop_dir<PI, LK, DAG, 1, 3>(a, Ur, in, c, p, i, onr, acc);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    part[wave][2 * k][lane] = acc[0][k].re;
    part[wave][2 * k + 1][lane] = acc[0][k].im;
  }
  __syncthreads();

  // Output storage vectors [v0, v1) of this wave (scaled formats need the
  // whole site for the scale: wave 0 takes all of them).
  constexpr int NVO = SO::NV;
  constexpr int CPV = 12 / NVO;
  const int v0 = SO::kScaled ? (wave == 0 ? 0 : NVO) : wave * NVO / NS;
  const int v1 = SO::kScaled ? NVO : (wave + 1) * NVO / NS;
  double vals[1][1] = {{0.0}};
  if (on && v0 < v1) {
    const int c0 = v0 * CPV, c1 = v1 * CPV;
    Cx<Rl> ctr[12];
    if constexpr (SI::kScaled || SpinFmt<PI>::NV != NVO)
      SI::load(in[0], Vh, p, i, ctr);
    else
      SI::load_range(in[0], Vh, p, i, ctr, v0, v1);
    const Rl m4 = (Rl)a.mass4;
    Cx<Ro> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      o[k] = {Ro(0), Ro(0)};
      if (k >= c0 && k < c1) {
        Rl re = 0, im = 0;
#pragma unroll
        for (int d = 0; d < NS; ++d) {
          re += part[d][2 * k][lane];
          im += part[d][2 * k + 1][lane];
        }
        o[k] = {(Ro)fma(m4, ctr[k].re, Rl(0.5) * re), (Ro)fma(m4, ctr[k].im, Rl(0.5) * im)};
      }
    }
    if constexpr (EPI == kEpiStore || EPI == kEpiStoreNorm) {
      const Rsrc orsrc = make_rsrc(a.out, a.out_bytes);
      if constexpr (SO::kScaled) {
        if (a.nt_store)
          SO::template store<2>(orsrc, Vh, p, i, o);
        else
          SO::template store<0>(orsrc, Vh, p, i, o);
      } else {
        if (a.nt_store)
          SO::template store_range<2>(orsrc, Vh, p, i, o, v0, v1);
        else
          SO::template store_range<0>(orsrc, Vh, p, i, o, v0, v1);
      }
      if constexpr (EPI == kEpiStoreNorm) {
        Cx<Ro> q[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = o[k];
        SO::round(q);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) s = fma((double)o[k].im, (double)q[k].im, fma((double)o[k].re, (double)q[k].re, s));
        vals[0][0] = s;
      }
    } else {
      static_assert(!SO::kScaled, "subtraction epilogue writes float32/float64");
      const Ro cf = a.sub_alpha ? (Ro)a.red.state[0].alpha : Ro(1);
      const Rsrc sr = make_rsrc(a.src, a.out_bytes);
      Cx<Ro> dd[12];
      SO::load_range(sr, Vh, p, i, dd, v0, v1);
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        dd[k].re = fma(-cf, o[k].re, dd[k].re);
        dd[k].im = fma(-cf, o[k].im, dd[k].im);
        s = fma((double)dd[k].im, (double)dd[k].im, fma((double)dd[k].re, (double)dd[k].re, s));
      }
      SO::template store_range<0>(make_rsrc(a.out, a.out_bytes), Vh, p, i, dd, v0, v1);
      vals[0][0] = s;
    }
  }
  if constexpr (EPI != kEpiStore) block_reduce_store<1, 1>(a.red, vals, 0, 1, tile, a.ntiles);
}

template <int PI, int PO, int LK, bool DAG, int EPI, int NS>
hipError_t launch_dslash_split(DslashArgs a, hipStream_t st) {
  a.ngroups = 1;
  a.ntiles = 2 * ((a.g.Vh + 63) / 64);
  hipLaunchKernelGGL((k_dslash_split<PI, PO, LK, DAG, EPI, NS>), dim3(a.ntiles), dim3(64 * NS), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || EPI == kEpiStore) return e;
  return launch_finalize(a.red, a.ntiles, 1, 1, st);
}

typedef hipError_t (*DslashLaunchFn)(DslashArgs, int block_sites, hipStream_t);

template <int PI, int PO, int LK, bool DAG, int EPI, int R>
hipError_t launch_dslash(DslashArgs a, int S, hipStream_t st) {
  a.ngroups = (a.nrhs + R - 1) / R;
  a.ntiles = 2 * ((a.g.Vh + S - 1) / S);
  const int nblocks = a.ntiles * a.ngroups;
  hipLaunchKernelGGL((k_dslash<PI, PO, LK, DAG, EPI, R>), dim3(nblocks), dim3(S), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || EPI == kEpiStore) return e;
  return launch_finalize(a.red, a.ntiles, a.nrhs, 1, st);
}

template <int PI, int PO, int LK, bool DAG, int EPI, int NS>
hipError_t launch_split_entry(DslashArgs a, int, hipStream_t st) {
  return launch_dslash_split<PI, PO, LK, DAG, EPI, NS>(a, st);
}

// rpt > 0: one-thread-per-site kernel with rpt right-hand sides per thread;
// rpt = -NS: direction-split kernel with NS waves per block of 64 sites.
struct DslashEntry {
  int pin, pout, link, dag, epi, rpt;
  DslashLaunchFn fn;
};

#define DIRAC_DSLASH_ENTRY(PI, PO, LK, DAG, EPI, R) \
  DslashEntry{PI, PO, LK, DAG, EPI, R, &launch_dslash<PI, PO, LK, DAG, EPI, R>}
#define DIRAC_DSLASH_SPLIT_ENTRY(PI, PO, LK, DAG, EPI, NS) \
  DslashEntry{PI, PO, LK, DAG, EPI, -NS, &launch_split_entry<PI, PO, LK, DAG, EPI, NS>}

}  // namespace dirac
