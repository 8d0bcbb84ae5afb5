// Half-lattice hops: the even-odd (Schur complement) form of D.
//
// Every hop of eq. (1) joins sites of opposite parity and the mass term stays
// on its site, so in (even, odd) blocks D = [[A, K_eo], [K_oe, A]] with
// A = m_q + 4 and K the hopping sum (its factor 1/2 included).  One launch
// here computes, on the sites of one parity p only,
//     out(n) = mass4 * ctr(n) + hop_c * (K in)(n),
// reading `in` on the other parity (the hops of eq. (1), projectors swapped
// for the adjoint) and the centre field `ctr` on p; with ctr null there is no
// centre term.  Two launches make the Schur complement
//     D_hat = A - K_eo K_oe / A
// (bare hop into the odd sites, then centre A and hop coefficient -1/A on the
// even sites), and with the adjoint hop D_hat^dagger.  Fields keep the full
// layout; a launch touches only the plane of its output parity, so one
// buffer can hold an even vector and the odd intermediate of the same
// operator.  Epilogues as in the full stencil: store, store plus |out|^2, or
// dst = src - alpha out plus |dst|^2 (dst in float32 for the scaled 16-bit
// formats).
//
// One thread per output site and right-hand side (the per-site stencil's
// hop code); the grid covers one parity only.  When the operator's launch
// configuration is the t-streaming one and its tile suits the hop (float64
// and float32), the streaming form of hop_stream.h runs instead.
#include "lib.h"
#include "hop_stream.h"

namespace dirac {

namespace {

constexpr int kHopBlock = 128;

template <int PI, int PO, int LK, bool DAG, int EPI>
__global__ void __launch_bounds__(kHopBlock) __attribute__((amdgpu_waves_per_eu(dslash_waves<PI, 1>())))
k_hop(DslashArgs a) {
  using Rl = typename SpinFmt<PI>::R;
  const int Vh = a.g.Vh;
  const int l = xcd_tile(blockIdx.x, a.ntiles * a.ngroups, a.remap);
  const int rhs = l % a.ngroups;  // right-hand sides of one tile side by side
  const int tile = l / a.ngroups;
  const int p = a.par;
  const int i = tile * kHopBlock + threadIdx.x;
  bool on = i < Vh;
  if (on && a.gate == kGateNotDone) on = !a.red.state[rhs].done;
  if (on && a.gate == kGateActive) on = a.red.state[rhs].active != 0;
  double vals[1][1] = {{0.0}};
  if (on) {
    const Coord c = cb_coords(a.g, p, i);
    const Rsrc Ur = make_rsrc(a.U, a.U_bytes);
    const Rsrc in[1] = {make_rsrc(a.in + (size_t)rhs * a.in_stride, a.field_bytes)};
    const bool onr[1] = {true};
    Cx<Rl> acc[1][12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[0][k] = {Rl(0), Rl(0)};
    hop_dir<PI, LK, DAG, 1, 0>(a, Ur, in, c, p, i, onr, acc);
    hop_dir<PI, LK, DAG, 1, 1>(a, Ur, in, c, p, i, onr, acc);
    hop_dir<PI, LK, DAG, 1, 2>(a, Ur, in, c, p, i, onr, acc);
    hop_dir<PI, LK, DAG, 1, 3>(a, Ur, in, c, p, i, onr, acc);
    hop_epilogue<PI, PO, EPI>(a, rhs, p, i, acc[0], vals[0][0]);
  }
  if constexpr (EPI != kEpiStore) block_reduce_store<1, 1>(a.red, vals, rhs, a.nrhs, tile, a.ntiles);
}

template <int PI, int PO, int LK, bool DAG, int EPI>
hipError_t launch_hop(DslashArgs a, hipStream_t st) {
  a.ngroups = a.nrhs;
  a.ntiles = (a.g.Vh + kHopBlock - 1) / kHopBlock;
  hipLaunchKernelGGL((k_hop<PI, PO, LK, DAG, EPI>), dim3(a.ntiles * a.ngroups), dim3(kHopBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || EPI == kEpiStore) return e;
  return launch_finalize(a.red, a.ntiles, a.nrhs, 1, st);
}

// The residual update of a scaled 16-bit operator writes float32 (as in the
// full stencil); everything else keeps the input format.
template <int P, int LK>
hipError_t hop_dispatch(int dag, int epi, const DslashArgs& a, hipStream_t st) {
  constexpr int PS = (P == DIRAC_F16S || P == DIRAC_BF16S) ? DIRAC_F32 : P;
  if (dag) {
    if (epi == kEpiStore) return launch_hop<P, P, LK, true, kEpiStore>(a, st);
    if (epi == kEpiStoreNorm) return launch_hop<P, P, LK, true, kEpiStoreNorm>(a, st);
    return launch_hop<P, PS, LK, true, kEpiSubNorm>(a, st);
  }
  if (epi == kEpiStore) return launch_hop<P, P, LK, false, kEpiStore>(a, st);
  if (epi == kEpiStoreNorm) return launch_hop<P, P, LK, false, kEpiStoreNorm>(a, st);
  return launch_hop<P, PS, LK, false, kEpiSubNorm>(a, st);
}

template <int P, int LK>
hipError_t hop_stream_dispatch(int dag, int epi, const DslashArgs& a, hipStream_t st) {
  if (dag) {
    if (epi == kEpiStore) return launch_hop_stream<P, P, LK, true, kEpiStore>(a, st);
    if (epi == kEpiStoreNorm) return launch_hop_stream<P, P, LK, true, kEpiStoreNorm>(a, st);
    return launch_hop_stream<P, P, LK, true, kEpiSubNorm>(a, st);
  }
  if (epi == kEpiStore) return launch_hop_stream<P, P, LK, false, kEpiStore>(a, st);
  if (epi == kEpiStoreNorm) return launch_hop_stream<P, P, LK, false, kEpiStoreNorm>(a, st);
  return launch_hop_stream<P, P, LK, false, kEpiSubNorm>(a, st);
}

}  // namespace

int hop_partials(const Geom& g) { return (g.Vh + kHopBlock - 1) / kHopBlock; }

int run_hop(int prec, int link, int dag, int epi, DslashArgs a, const LaunchCfg& c, hipStream_t st) {
  if (a.par != 0 && a.par != 1) return set_error(DIRAC_EINVAL, "half-lattice hop: parity must be 0 or 1");
  if (epi != kEpiStore && epi != kEpiStoreNorm && epi != kEpiSubNorm)
    return set_error(DIRAC_EINVAL, "half-lattice hop: unknown epilogue %d", epi);
  hipError_t e;
  int sy = c.sy, sz = c.sz;
  if (c.lds) hop_stream_tile(a.g, prec, sy, sz);
  if (c.lds && hop_stream_fits(a.g, sy, sz, c.tc, prec)) {
    // the operator's streaming tile grown to fill the hop's block, in
    // XCD-contiguous order (t-chunks fastest, which suits some D launches,
    // made the hop slower)
    a.sy = sy;
    a.sz = sz;
    a.tc = hop_stream_chunk(c.tc);
    a.remap = kStreamXcd;
    if (prec == DIRAC_F64 && link == 18) e = hop_stream_dispatch<DIRAC_F64, 18>(dag, epi, a, st);
    else if (prec == DIRAC_F64 && link == 12) e = hop_stream_dispatch<DIRAC_F64, 12>(dag, epi, a, st);
    else if (prec == DIRAC_F32 && link == 18) e = hop_stream_dispatch<DIRAC_F32, 18>(dag, epi, a, st);
    else e = hop_stream_dispatch<DIRAC_F32, 12>(dag, epi, a, st);
    return hip_status(e, "half-lattice hop launch");
  }
  a.remap = 1;
  if (prec == DIRAC_F64 && link == 18) e = hop_dispatch<DIRAC_F64, 18>(dag, epi, a, st);
  else if (prec == DIRAC_F64 && link == 12) e = hop_dispatch<DIRAC_F64, 12>(dag, epi, a, st);
  else if (prec == DIRAC_F32 && link == 18) e = hop_dispatch<DIRAC_F32, 18>(dag, epi, a, st);
  else if (prec == DIRAC_F32 && link == 12) e = hop_dispatch<DIRAC_F32, 12>(dag, epi, a, st);
  else if (prec == DIRAC_F16S && link == 12) e = hop_dispatch<DIRAC_F16S, 12>(dag, epi, a, st);
  else if (prec == DIRAC_BF16S && link == 12) e = hop_dispatch<DIRAC_BF16S, 12>(dag, epi, a, st);
  else return set_error(DIRAC_EUNSUPPORTED, "half-lattice hop: no kernel for prec %d link %d", prec, link);
  return hip_status(e, "half-lattice hop launch");
}

}  // namespace dirac
