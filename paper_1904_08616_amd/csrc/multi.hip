// Several independent lattices in one persistent launch.
//
// Small lattices (8^4 is 4096 sites, a few microseconds of HBM traffic) cannot
// fill 256 compute units on their own and are dominated by launch latency.
// Here one grid of a few workgroups per CU walks a work list of
// (lattice, parity, block of sites) tiles in order, each workgroup taking
// every gridDim-th tile, and applies the same per-site stencil as the
// single-lattice kernel to each.  The whole launch can be captured in a
// hipGraph (dirac_multi_plan_create) and replayed.
#include "lib.h"

namespace dirac {

namespace {

constexpr int kMaxLat = 8;
constexpr int kMultiBlock = 128;

struct MultiLat {
  Geom g;
  const char* U;
  const char* in;
  char* out;
  uint32_t U_bytes;
  uint32_t field_bytes;
  double mass4;
  int tile_begin;  // first global tile of this lattice
  int ntiles;      // 2 * ceil(Vh / kMultiBlock)
};

struct MultiArgs {
  MultiLat lat[kMaxLat];
  int n;
  int total_tiles;
};

template <int P, int LK, bool DAG>
__global__ void __launch_bounds__(kMultiBlock) __attribute__((amdgpu_waves_per_eu(dslash_waves<P, 1>())))
k_multi(MultiArgs m) {
  for (int t = blockIdx.x; t < m.total_tiles; t += gridDim.x) {
    int L = 0;
#pragma unroll
    for (int k = 1; k < kMaxLat; ++k)
      if (k < m.n && t >= m.lat[k].tile_begin) L = k;
    const MultiLat& lt = m.lat[L];
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

template <int P, int LK>
hipError_t launch_multi(const MultiArgs& m, int dag, int grid, hipStream_t st) {
  if (dag)
    hipLaunchKernelGGL((k_multi<P, LK, true>), dim3(grid), dim3(kMultiBlock), 0, st, m);
  else
    hipLaunchKernelGGL((k_multi<P, LK, false>), dim3(grid), dim3(kMultiBlock), 0, st, m);
  return hipGetLastError();
}

}  // namespace

int multi_apply(int n, const OpInfo* infos, const void* const* U, const void* const* psi, void* const* chi,
                int dagger, hipStream_t st) {
  MultiArgs m;
  m.n = n;
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
    l.ntiles = 2 * ((l.g.Vh + kMultiBlock - 1) / kMultiBlock);
    l.tile_begin = tiles;
    tiles += l.ntiles;
  }
  for (int k = n; k < kMaxLat; ++k) m.lat[k] = m.lat[0];
  m.total_tiles = tiles;
  // Persistent grid: a few workgroups per CU, never more than the tiles.
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  }
  const int grid = std::min(tiles, cus * 8);
  const int prec = infos[0].prec, link = infos[0].link;
  hipError_t e;
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
