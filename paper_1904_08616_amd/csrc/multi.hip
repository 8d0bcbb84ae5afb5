// Several independent lattices in one persistent kernel launch.
//
// Small lattices (8^4 is 4096 sites, a few microseconds of HBM traffic)
// cannot fill 256 compute units on their own and are dominated by launch
// latency; one launch over a work list of (lattice, tile) items removes the
// gaps between lattices.  Two forms share the work-list idea:
//   - per site: a grid of a few workgroups per CU walks (lattice, parity,
//     block of sites) tiles in order, each workgroup taking every
//     gridDim-th tile, with the per-site stencil;
//   - t-streaming: one 256-thread workgroup per (lattice, streaming tile),
//     each lattice with its own tile (all of x times tile_y times tile_z,
//     the largest that fits 256 threads) and a common t_chunk; odd chunks
//     walk down in t, and the tiles are dealt to the XCDs in contiguous runs.
// The whole launch can be captured in a hipGraph (dirac_multi_plan_create),
// which first times the candidate forms on the caller's buffers.
#include "dslash_stream.h"
#include "lib.h"

namespace dirac {

namespace {

constexpr int kMaxLat = 8;
constexpr int kMultiBlock = 128;
constexpr int kMultiStreamNC = 256;

struct MultiLat {
  Geom g;
  const char* U;
  const char* in;
  char* out;
  uint32_t U_bytes;
  uint32_t field_bytes;
  double mass4;
  int tile_begin;  // first global tile of this lattice
  int ntiles;      // per site: 2 * ceil(Vh / kMultiBlock); streaming: tiles
  int sy, sz, tc;  // streaming tile
  int nty, ntz, ntt;
};

struct MultiArgs {
  MultiLat lat[kMaxLat];
  int n;
  int total_tiles;
  int xcd;  // XCD-contiguous tile order (streaming form)
};

__device__ __forceinline__ int multi_lattice(const MultiArgs& m, int t) {
  int L = 0;
#pragma unroll
  for (int k = 1; k < kMaxLat; ++k)
    if (k < m.n && t >= m.lat[k].tile_begin) L = k;
  return L;
}

template <int P, int LK, bool DAG>
__global__ void __launch_bounds__(kMultiBlock) __attribute__((amdgpu_waves_per_eu(dslash_waves<P, 1>())))
k_multi(MultiArgs m) {
  for (int t = blockIdx.x; t < m.total_tiles; t += gridDim.x) {
    const MultiLat& lt = m.lat[multi_lattice(m, t)];
    const int tile = t - lt.tile_begin;
    const int p = tile & 1;
    const int i = (tile >> 1) * kMultiBlock + threadIdx.x;
    if (i >= lt.g.Vh) continue;
    DslashArgs a{};  // every field defined (reading an undefined one is UB)
    a.g = lt.g;
    a.U = lt.U;
    a.U_bytes = lt.U_bytes;
    a.field_bytes = lt.field_bytes;
    a.out_bytes = lt.field_bytes;
    a.in = lt.in;
    a.in_stride = 0;
    a.out = lt.out;
    a.out_stride = 0;
    a.src = nullptr;
    a.src_stride = 0;
    a.mass4 = lt.mass4;
    a.nrhs = 1;
    a.gate = kGateNone;
    a.nt_store = 0;
    bool on[1] = {true};
    double vals[1][1] = {{0.0}};
    dslash_site<P, P, LK, DAG, kEpiStore, 1>(a, p, i, 0, on, vals);
  }
}

template <int P, int LK, bool DAG>
__global__ void __launch_bounds__(kMultiStreamNC)
__attribute__((amdgpu_waves_per_eu(P == DIRAC_F64 ? 2 : DIRAC_STREAM_WAVES_F32)))
k_multi_stream(MultiArgs m) {
  extern __shared__ __align__(16) char lds_raw[];
  const int gt = xcd_tile(blockIdx.x, m.total_tiles, m.xcd);
  const MultiLat& lt = m.lat[multi_lattice(m, gt)];
  const int l = gt - lt.tile_begin;
  DslashArgs a{};
  a.g = lt.g;
  a.U = lt.U;
  a.U_bytes = lt.U_bytes;
  a.field_bytes = lt.field_bytes;
  a.out_bytes = lt.field_bytes;
  a.in = lt.in;
  a.out = lt.out;
  a.mass4 = lt.mass4;
  a.nrhs = 1;
  a.gate = kGateNone;
  a.nt_store = 1;
  a.sy = lt.sy;
  a.sz = lt.sz;
  a.tc = lt.tc;
  a.ntiles = lt.ntiles;
  const Geom g = lt.g;
  const int tid = threadIdx.x;
  const bool act = tid < g.X * lt.sy * lt.sz;
  const int x = tid % g.X;
  const int yl = (tid / g.X) % lt.sy;
  const int zl = tid / (g.X * lt.sy);
  // t-chunks fastest within a lattice, so a tile's chunks run side by side
  const int tt = l % lt.ntt;
  const int ty = (l / lt.ntt) % lt.nty;
  const int tz = l / (lt.ntt * lt.nty);
  const int y = ty * lt.sy + yl, z = tz * lt.sz + zl;
  const int t0 = tt * lt.tc;
  const int t1 = min(t0 + lt.tc, g.T);
  double v = 0.0;
  if (tt & 1)
    stream_walk<P, P, LK, DAG, kEpiStore, kMultiStreamNC, true>(a, 0, act, x, y, z, yl, zl, t0, t1, lds_raw, v);
  else
    stream_walk<P, P, LK, DAG, kEpiStore, kMultiStreamNC, false>(a, 0, act, x, y, z, yl, zl, t0, t1, lds_raw, v);
}

template <int P, int LK>
hipError_t launch_multi(const MultiArgs& m, int dag, int grid, hipStream_t st) {
  if (dag)
    hipLaunchKernelGGL((k_multi<P, LK, true>), dim3(grid), dim3(kMultiBlock), 0, st, m);
  else
    hipLaunchKernelGGL((k_multi<P, LK, false>), dim3(grid), dim3(kMultiBlock), 0, st, m);
  return hipGetLastError();
}

template <int P, int LK>
hipError_t launch_multi_stream(const MultiArgs& m, int dag, hipStream_t st) {
  const size_t lds = (size_t)kMultiStreamNC * (P == DIRAC_F64 ? 30 : 24) * sizeof(Cx<typename SpinFmt<P>::R>);
  if (dag)
    hipLaunchKernelGGL((k_multi_stream<P, LK, true>), dim3(m.total_tiles), dim3(kMultiStreamNC), lds, st, m);
  else
    hipLaunchKernelGGL((k_multi_stream<P, LK, false>), dim3(m.total_tiles), dim3(kMultiStreamNC), lds, st, m);
  return hipGetLastError();
}

}  // namespace

// Largest streaming tile of at most 256 columns for this lattice (the most
// columns, then the squarest); false if none has at least 32.
bool multi_stream_tile(const Geom& g, int* sy, int* sz) {
  int best = 0, bsy = 0, bsz = 0;
  for (int a = 1; a <= g.Y; ++a) {
    if (g.Y % a) continue;
    for (int b = 1; b <= g.Z; ++b) {
      if (g.Z % b) continue;
      const int n = stream_columns(g, a, b);
      if (n > kMultiStreamNC || n < 32) continue;
      if (n > best || (n == best && std::abs(a - b) < std::abs(bsy - bsz))) {
        best = n;
        bsy = a;
        bsz = b;
      }
    }
  }
  *sy = bsy;
  *sz = bsz;
  return best > 0;
}

int multi_apply(int n, const OpInfo* infos, const void* const* U, const void* const* psi, void* const* chi,
                int dagger, const MultiCfg& cfg, hipStream_t st) {
  MultiArgs m;
  m.n = n;
  m.xcd = cfg.xcd;
  const bool stream = cfg.stream != 0;
  int tiles = 0;
  for (int k = 0; k < n; ++k) {
    MultiLat& l = m.lat[k];
    l.g = infos[k].g;
    l.U = (const char*)U[k];
    l.in = (const char*)psi[k];
    l.out = (char*)chi[k];
    l.U_bytes = infos[k].gauge_bytes;
    l.field_bytes = infos[k].field_bytes;
    l.mass4 = infos[k].m_q + 4.0;
    l.tile_begin = tiles;
    if (stream) {
      if (!multi_stream_tile(l.g, &l.sy, &l.sz))
        return set_error(DIRAC_EUNSUPPORTED, "multi launch: no streaming tile fits lattice %d", k);
      l.tc = std::min(std::max(cfg.tc, 1), l.g.T);
      l.nty = l.g.Y / l.sy;
      l.ntz = l.g.Z / l.sz;
      l.ntt = (l.g.T + l.tc - 1) / l.tc;
      l.ntiles = l.nty * l.ntz * l.ntt;
    } else {
      l.sy = l.sz = l.tc = l.nty = l.ntz = l.ntt = 1;
      l.ntiles = 2 * ((l.g.Vh + kMultiBlock - 1) / kMultiBlock);
    }
    tiles += l.ntiles;
  }
  for (int k = n; k < kMaxLat; ++k) m.lat[k] = m.lat[0];
  m.total_tiles = tiles;
  const int prec = infos[0].prec, link = infos[0].link;
  hipError_t e;
  if (stream) {
#define MS(P, LK) launch_multi_stream<P, LK>(m, dagger, st)
    if (prec == DIRAC_F64 && link == 18) e = MS(DIRAC_F64, 18);
    else if (prec == DIRAC_F64 && link == 12) e = MS(DIRAC_F64, 12);
    else if (prec == DIRAC_F32 && link == 18) e = MS(DIRAC_F32, 18);
    else if (prec == DIRAC_F32 && link == 12) e = MS(DIRAC_F32, 12);
    else if (prec == DIRAC_F16S && link == 12) e = MS(DIRAC_F16S, 12);
    else if (prec == DIRAC_BF16S && link == 12) e = MS(DIRAC_BF16S, 12);
    else return set_error(DIRAC_EUNSUPPORTED, "dirac_multi_apply: unsupported precision/link");
#undef MS
    return hip_status(e, "multi stream launch");
  }
  // Persistent grid: a few workgroups per CU, never more than the tiles.
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  }
  const int grid = std::min(tiles, cus * 8);
  if (prec == DIRAC_F64 && link == 18) e = launch_multi<DIRAC_F64, 18>(m, dagger, grid, st);
  else if (prec == DIRAC_F64 && link == 12) e = launch_multi<DIRAC_F64, 12>(m, dagger, grid, st);
  else if (prec == DIRAC_F32 && link == 18) e = launch_multi<DIRAC_F32, 18>(m, dagger, grid, st);
  else if (prec == DIRAC_F32 && link == 12) e = launch_multi<DIRAC_F32, 12>(m, dagger, grid, st);
  else if (prec == DIRAC_F16S && link == 12) e = launch_multi<DIRAC_F16S, 12>(m, dagger, grid, st);
  else if (prec == DIRAC_BF16S && link == 12) e = launch_multi<DIRAC_BF16S, 12>(m, dagger, grid, st);
  else return set_error(DIRAC_EUNSUPPORTED, "dirac_multi_apply: unsupported precision/link");
  return hip_status(e, "multi launch");
}

}  // namespace dirac
