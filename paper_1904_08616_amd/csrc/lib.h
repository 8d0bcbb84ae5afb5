// Internal host-side interfaces shared by the C ABI (api.cpp), the solver
// (solver.cpp) and the batched launches (multi.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "dirac.h"
#include "common.h"
#include "dslash_impl.h"
#include "dslash_stream.h"
#include "field.h"

namespace dirac {

// Validated view of a dirac_op.
struct OpInfo {
  Geom g;
  int prec, link, nrhs;
  double m_q;
  int64_t V;
  uint32_t field_bytes;   // one field of this precision
  int64_t field_stride;   // distance between right-hand sides (256-byte aligned)
  uint32_t gauge_bytes;
};

int set_error(int code, const char* fmt, ...);
void clear_error();
int check_op(const dirac_op* op, OpInfo* out, const char* what);
int hip_status(hipError_t e, const char* what);

inline int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

FieldRef field_of(const OpInfo& o, const void* p);
FieldRef field_as(const OpInfo& o, int prec, const void* p);  // same geometry, other precision

// Launch configuration of the Dslash kernels.
struct LaunchCfg {
  int S;      // one-thread-per-site kernel: threads (sites) per block
  int R;      // right-hand sides per thread (> 0) or direction split (-2, -4)
  int remap;  // XCD-aware tile order
  int lds;    // 1: t-streaming kernel with the current slice staged in LDS
  int nt;     // non-temporal output stores
  int sy, sz, tc;  // streaming kernel tile: y rows, z planes, t slices per block
  int tuned;
};
LaunchCfg launch_cfg(const OpInfo& o);

// Run one Dslash instance; returns DIRAC_EUNSUPPORTED if no such instance.
int run_dslash(int pin, int pout, int link, int dag, int epi, const LaunchCfg& c, DslashArgs a,
               hipStream_t st);

DslashArgs dslash_args(const OpInfo& o, const void* U, const void* in, void* out);

// Half-lattice hop of the even-odd form (hop.hip): on the sites of parity
// a.par, out = a.mass4 * ctr + a.hop_c * (K in) with the epilogue `epi`;
// F64 and F32 with either link storage.  A streaming configuration c (lds)
// whose tile suits the hop selects its t-streaming form.  hop_partials:
// reduction partials per right-hand side of one per-site launch (the
// streaming form needs fewer).
int run_hop(int prec, int link, int dag, int epi, DslashArgs a, const LaunchCfg& c, hipStream_t st);
int hop_partials(const Geom& g);

// CG iterations of every right-hand side of op in one launch (cg_small.hip):
// at most `chunk` iterations each, from and back to the CgState scalars.
int cg_small_iterations(const OpInfo& o, const void* U, FieldRef x, FieldRef p, FieldRef r, FieldRef t,
                        CgState* state, int chunk, hipStream_t st);

// Multi-lattice persistent launch (multi.hip): per-site form, or t-streaming
// tiles with a common t_chunk (optionally dealt to XCDs in contiguous runs).
struct MultiCfg {
  int stream;
  int tc;
  int xcd;
};
bool multi_stream_tile(const Geom& g, int* sy, int* sz);
int multi_apply(int n, const OpInfo* infos, const void* const* U, const void* const* psi, void* const* chi,
                int dagger, const MultiCfg& cfg, hipStream_t st);

}  // namespace dirac
