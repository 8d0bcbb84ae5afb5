// Host-side declarations of the site-wise field kernels (layout conversion
// and the fused BLAS-1 operations of the CG).
#pragma once

#include "common.h"

namespace dirac {

// A spinor buffer: nrhs fields of one format, `stride` bytes apart.
struct FieldRef {
  char* ptr;
  int prec;
  int64_t stride;
  uint32_t bytes;  // bytes of one field
};

// Reduction target of a launch: partial sums go to `partials`, and a second
// one-block-per-RHS kernel applies `kind` to state[rhs] (see cg_finalize).
struct RedTarget {
  double* partials;
  CgState* state;
  int kind;
};

// Canonical complex128 <-> internal.
hipError_t pack_spinor(const Geom& g, int nrhs, const void* src_c128, FieldRef dst, hipStream_t st);
hipError_t unpack_spinor(const Geom& g, int nrhs, FieldRef src, void* dst_c128, hipStream_t st);
hipError_t pack_gauge(const Geom& g, int prec, int link, const void* U_c128, void* U_int,
                      hipStream_t st);

// dst = c * src with per-RHS real factor c = state[rhs].coef[coef_idx] (coef_idx >= 0)
// or 1 (coef_idx < 0); optional |dst|^2 reduction.
hipError_t convert_scale(const Geom& g, int nrhs, FieldRef src, FieldRef dst, const CgState* coef_state,
                         int coef_idx, const RedTarget* red, hipStream_t st);

// <a, b> per RHS (complex) into red (NC = 2).
hipError_t dot(const Geom& g, int nrhs, FieldRef a, FieldRef b, const RedTarget& red, hipStream_t st);

// |a|^2 per RHS into red (NC = 1).
hipError_t norm2(const Geom& g, int nrhs, FieldRef a, const RedTarget& red, hipStream_t st);

// y = a x + b y, complex a, b.  Per RHS from state[rhs].coef[0..3] =
// (a_re, a_im, b_re, b_im) when state != nullptr, else the given constants.
hipError_t axpby(const Geom& g, int nrhs, FieldRef x, FieldRef y, const CgState* state,
                 double a_re, double a_im, double b_re, double b_im, hipStream_t st);

// CG update after the residual step: where state[rhs].active,
//   x += alpha p;  p = r + beta p.
hipError_t cg_xp_update(const Geom& g, int nrhs, FieldRef x, FieldRef p, FieldRef r,
                        const CgState* state, hipStream_t st);

// Fill with zeros (a kernel, so it can sit inside a captured graph).
hipError_t zero(const Geom& g, int nrhs, FieldRef f, hipStream_t st);

// Link gradient (see dirac_force).
hipError_t force(const Geom& g, int prec, const void* gin, const void* psi, uint32_t field_bytes,
                 void* F_c128, double coeff, int accumulate, hipStream_t st);

}  // namespace dirac
