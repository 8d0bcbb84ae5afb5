// Shared device-side building blocks of libdirac: lattice geometry and the
// even-odd site map, complex arithmetic, the internal storage formats of
// spinors and links, SU(3) row reconstruction, the per-direction spin
// projections of eq. (1), and a deterministic float64 grid reduction.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstddef>

#include "dirac.h"

namespace dirac {

constexpr int kNumXcd = 8;       // MI355X: 8 XCDs, 32 CUs each
constexpr int kMaxRhs = 12;

// --------------------------------------------------------------- geometry --
// Sites are split by parity p = (x+y+z+t) & 1; within a parity the
// checkerboard index is i = n >> 1 where n = ((t*Z + z)*Y + y)*X + x is the
// lexicographic site number (x fastest).  X even makes this a bijection.
struct Geom {
  int X, Y, Z, T;
  int Xh;  // X / 2
  int Vh;  // sites per parity
  int sZ;  // checkerboard stride of z: Xh * Y
  int sT;  // checkerboard stride of t: Xh * Y * Z
  int vpar;  // site-wise field operations: -1 both parities, 0 / 1 that parity only
};

inline Geom make_geom(const int L[4]) {
  Geom g;
  g.vpar = -1;
  g.X = L[0]; g.Y = L[1]; g.Z = L[2]; g.T = L[3];
  g.Xh = g.X / 2;
  g.sZ = g.Xh * g.Y;
  g.sT = g.sZ * g.Z;
  g.Vh = g.sT * g.T;
  return g;
}

struct Coord { int x, y, z, t; };

__device__ __forceinline__ Coord cb_coords(const Geom& g, int p, int i) {
  Coord c;
  int xh = i % g.Xh;
  int r = i / g.Xh;
  c.y = r % g.Y;
  r /= g.Y;
  c.z = r % g.Z;
  c.t = r / g.Z;
  c.x = 2 * xh + ((p + c.y + c.z + c.t) & 1);
  return c;
}

// Checkerboard index (in the opposite parity) of the forward / backward
// neighbour of site (c, i) in direction MU.
template <int MU>
__device__ __forceinline__ int nb_fwd(const Geom& g, const Coord& c, int i) {
  if constexpr (MU == 0) {
    int xn = (c.x + 1 == g.X) ? 0 : c.x + 1;
    return i - (c.x >> 1) + (xn >> 1);
  } else if constexpr (MU == 1) {
    return (c.y + 1 == g.Y) ? i - (g.Y - 1) * g.Xh : i + g.Xh;
  } else if constexpr (MU == 2) {
    return (c.z + 1 == g.Z) ? i - (g.Z - 1) * g.sZ : i + g.sZ;
  } else {
    return (c.t + 1 == g.T) ? i - (g.T - 1) * g.sT : i + g.sT;
  }
}

template <int MU>
__device__ __forceinline__ int nb_bwd(const Geom& g, const Coord& c, int i) {
  if constexpr (MU == 0) {
    int xn = (c.x == 0) ? g.X - 1 : c.x - 1;
    return i - (c.x >> 1) + (xn >> 1);
  } else if constexpr (MU == 1) {
    return (c.y == 0) ? i + (g.Y - 1) * g.Xh : i - g.Xh;
  } else if constexpr (MU == 2) {
    return (c.z == 0) ? i + (g.Z - 1) * g.sZ : i - g.sZ;
  } else {
    return (c.t == 0) ? i + (g.T - 1) * g.sT : i - g.sT;
  }
}

// Block index -> logical tile index so that each XCD (blocks are handed to
// the 8 XCDs round-robin) walks one contiguous range of tiles: neighbouring
// tiles then share that XCD's L2.  A bijection on [0, nblocks).
__device__ __forceinline__ int xcd_tile(int b, int nblocks, int remap) {
  if (!remap) return b;
  int q = nblocks / kNumXcd, rem = nblocks % kNumXcd;
  int xcd = b % kNumXcd, slot = b / kNumXcd;
  return (xcd < rem) ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

// ---------------------------------------------------------------- complex --
template <class R> struct Cx { R re, im; };

template <class R> __device__ __forceinline__ Cx<R> cx(R a, R b) { return Cx<R>{a, b}; }
template <class R> __device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <class R> __device__ __forceinline__ Cx<R> mul_i(Cx<R> a) { return {-a.im, a.re}; }    // i a
template <class R> __device__ __forceinline__ Cx<R> mul_mi(Cx<R> a) { return {a.im, -a.re}; }   // -i a
template <class R> __device__ __forceinline__ Cx<R> neg(Cx<R> a) { return {-a.re, -a.im}; }
template <class R> __device__ __forceinline__ Cx<R> conj(Cx<R> a) { return {a.re, -a.im}; }
// a * b, each component one product and one fused multiply-add in a fixed
// order, so that every kernel instance rounds it the same way (left to the
// compiler, which product is fused may differ between instances)
template <class R> __device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
// acc + a * b
template <class R> __device__ __forceinline__ Cx<R> cmadd(Cx<R> acc, Cx<R> a, Cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc + conj(a) * b
template <class R> __device__ __forceinline__ Cx<R> cjmadd(Cx<R> acc, Cx<R> a, Cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}

template <class R> struct M3 { Cx<R> e[3][3]; };

// Row 2 of an SU(3) matrix from rows 0 and 1: conj(row0 x row1).
template <class R> __device__ __forceinline__ void su3_row2(M3<R>& u) {
  auto cr = [](Cx<R> a, Cx<R> b, Cx<R> c, Cx<R> d) {  // conj(a*b - c*d)
    Cx<R> v = cmul(a, b) - cmul(c, d);
    return conj(v);
  };
  u.e[2][0] = cr(u.e[0][1], u.e[1][2], u.e[0][2], u.e[1][1]);
  u.e[2][1] = cr(u.e[0][2], u.e[1][0], u.e[0][0], u.e[1][2]);
  u.e[2][2] = cr(u.e[0][0], u.e[1][1], u.e[0][1], u.e[1][0]);
}

// su3_row2 for rows held as decoded 16-bit values: each component is one
// chain of four fused multiply-adds from `zero` (= 0, kept opaque to the
// compiler), so that every product reads its 16-bit operands directly
// (mixed-precision FMA) instead of converting them first.
template <class R> __device__ __forceinline__ void su3_row2_fma(M3<R>& u, R zero) {
  auto cr = [zero](Cx<R> a, Cx<R> b, Cx<R> c, Cx<R> d) {  // conj(a*b - c*d)
    R re = fma(a.re, b.re, zero);
    re = fma(-a.im, b.im, re);
    re = fma(-c.re, d.re, re);
    re = fma(c.im, d.im, re);
    R im = fma(a.re, b.im, zero);
    im = fma(a.im, b.re, im);
    im = fma(-c.re, d.im, im);
    im = fma(-c.im, d.re, im);
    return Cx<R>{re, -im};
  };
  u.e[2][0] = cr(u.e[0][1], u.e[1][2], u.e[0][2], u.e[1][1]);
  u.e[2][1] = cr(u.e[0][2], u.e[1][0], u.e[0][0], u.e[1][2]);
  u.e[2][2] = cr(u.e[0][0], u.e[1][1], u.e[0][1], u.e[1][0]);
}

// Squared modulus of a complex entry, evaluated the same way by the link
// packer and the 10-real rebuild (their pivot choices must agree).
template <class R> __device__ __forceinline__ R abs2_exact(Cx<R> a) { return fma(a.re, a.re, a.im * a.im); }

// Rows 1 and 2 of an SU(3) matrix from row 0 (in u.e[0]) and, for the pivot
// column k, the entries b0 = U_1k and c0 = U_2k (the 10-real link form; the
// paper streams a 10-parameter link and trades the two extra words against
// trigonometric functions, Larger Lattice Streamed from the DDR Memory).
// The pivot is the column whose row-0 entry has the smallest modulus (lowest
// index on ties).  Rotating the columns cyclically by k gives V = U P, still
// special unitary, whose entries satisfy conj(V_ij) = cofactor_ij; solved
// for the four entries outside V's row 0 and column 0 they divide by
// n = |V_01|^2 + |V_02|^2 = 1 - |V_00|^2 >= 2/3, and no modulus is taken
// from a difference.
template <class R>
__device__ __forceinline__ void su3_from_row_pivot(M3<R>& u, Cx<R> b0, Cx<R> c0) {
  const Cx<R> e0 = u.e[0][0], e1 = u.e[0][1], e2 = u.e[0][2];
  const R m0 = abs2_exact(e0), m1 = abs2_exact(e1), m2 = abs2_exact(e2);
  const bool k0 = m0 <= m1 && m0 <= m2;
  const bool k1 = !k0 && m1 <= m2;
  auto sel = [k0, k1](Cx<R> x0, Cx<R> x1, Cx<R> x2) { return k0 ? x0 : (k1 ? x1 : x2); };
  const Cx<R> a0 = sel(e0, e1, e2), a1 = sel(e1, e2, e0), a2 = sel(e2, e0, e1);
  const R n = k0 ? m1 + m2 : (k1 ? m2 + m0 : m0 + m1);
  const R inv = R(1) / n;
  // V_11 = -(conj(a0) a1 b0 + conj(a2) conj(c0)) / n
  Cx<R> t = cmul(cmul(conj(a0), a1), b0);
  t = cmadd(t, conj(a2), conj(c0));
  const Cx<R> b1 = (-inv) * t;
  // V_12 = (conj(a1) conj(c0) - conj(a0) a2 b0) / n
  const Cx<R> b2 = inv * (cmul(conj(a1), conj(c0)) - cmul(cmul(conj(a0), a2), b0));
  // V_21 = conj(a2) conj(b0) - conj(a0) conj(b2);  V_22 = conj(a0) conj(b1) - conj(a1) conj(b0)
  const Cx<R> c1 = cmul(conj(a2), conj(b0)) - cmul(conj(a0), conj(b2));
  const Cx<R> c2 = cmul(conj(a0), conj(b1)) - cmul(conj(a1), conj(b0));
  // U_{r, k+j} = V_{r, j}
  u.e[1][0] = sel(b0, b2, b1);
  u.e[1][1] = sel(b1, b0, b2);
  u.e[1][2] = sel(b2, b1, b0);
  u.e[2][0] = sel(c0, c2, c1);
  u.e[2][1] = sel(c1, c0, c2);
  u.e[2][2] = sel(c2, c1, c0);
}

// ------------------------------------------------------- storage formats --
// Spinor fields: per right-hand side, [parity][NV][Vh] 16-byte vectors,
// followed for scaled formats by a float scale per site [parity][Vh].
// Component c = 3*spin + colour.
//   F64  : NV = 12, double2 = one complex each
//   F32  : NV = 6,  float4  = two complex each
//   F16S : NV = 3,  8 x half = four complex each, times the site scale
//   BF16S: NV = 3,  8 x bfloat16, times the site scale
template <int P> struct SpinFmt;

__device__ __forceinline__ float bf16_to_f(unsigned short b) {
  return __uint_as_float(((unsigned)b) << 16);
}
// float -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ unsigned short f_to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float h_to_f(unsigned short h) {
  return __half2float(__ushort_as_half(h));
}
__device__ __forceinline__ unsigned short f_to_h(float f) {
  return __half_as_ushort(__float2half_rn(f));
}

// Fields are read and written with raw buffer instructions: a 128-bit
// resource (base, size) in scalar registers, a wave-uniform component-plane
// offset in a scalar register and one 32-bit per-lane offset shared by all
// planes.  This keeps address arithmetic out of the vector register budget,
// and the hardware range check turns any access past the field's end into a
// zero load / dropped store instead of a memory fault.  One field (one
// right-hand side) must therefore be smaller than 4 GiB.
typedef __amdgpu_buffer_rsrc_t Rsrc;

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Offset of parity plane p (0 or 1) when one plane is `plane` bytes: a
// select, not an integer multiply (a quarter-rate instruction).
__device__ __forceinline__ uint32_t plane_off(int p, uint32_t plane) { return p ? plane : 0u; }

template <class T>
__device__ __forceinline__ T bld(Rsrc r, uint32_t voff, uint32_t soff) {
  static_assert(sizeof(T) == 16 || sizeof(T) == 8 || sizeof(T) == 4, "buffer load size");
  if constexpr (sizeof(T) == 16) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  } else if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
}
// AUX = 0: ordinary store; AUX = 2: non-temporal (streaming) store that does
// not keep the line in the L2.
//
// A 128-bit store never takes its offset in an SGPR (soffset): a VALU write
// to the store's data registers right after such a store needs a wait state,
// and the compiler only inserts it when soffset is the constant 0.  Without
// it the store can pick up the new register value under load (seen as
// sporadically corrupted first dwords).  The plane offset is therefore added
// to the per-lane offset, which costs one VALU add per store.
template <int AUX = 0, class T>
__device__ __forceinline__ void bst(Rsrc r, uint32_t voff, uint32_t soff, const T& v) {
  static_assert(sizeof(T) == 16 || sizeof(T) == 8 || sizeof(T) == 4, "buffer store size");
  if constexpr (sizeof(T) == 16) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff + soff, 0, AUX);
  } else if constexpr (sizeof(T) == 8) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, AUX);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, AUX);
  }
}

template <> struct SpinFmt<DIRAC_F64> {
  using R = double;
  static constexpr int NV = 12;
  static constexpr bool kScaled = false;
  static constexpr int kSiteBytes = 192;
  __device__ static __forceinline__ void load(Rsrc f, int Vh, int p, int i, Cx<R> (&v)[12]) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 12u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      double2 t = bld<double2>(f, o, (uint32_t)c * (uint32_t)Vh * 16u);
      v[c] = {t.x, t.y};
    }
  }
  __device__ static __forceinline__ void round(Cx<R> (&)[12]) {}
  // store(), returning in q the value left in memory (v itself here).
  template <int AUX = 0>
  __device__ static __forceinline__ void store_q(Rsrc f, int Vh, int p, int i, const Cx<R> (&v)[12],
                                                 Cx<R> (&q)[12]) {
    store<AUX>(f, Vh, p, i, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) q[c] = v[c];
  }
  template <int AUX = 0>
  __device__ static __forceinline__ void store(Rsrc f, int Vh, int p, int i, const Cx<R> (&v)[12]) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 12u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int c = 0; c < 12; ++c)
      bst<AUX>(f, o, (uint32_t)c * (uint32_t)Vh * 16u, make_double2(v[c].re, v[c].im));
  }
  // Store only the storage vectors [v0, v1) (vector k holds component k).
  template <int AUX = 0>
  __device__ static __forceinline__ void store_range(Rsrc f, int Vh, int p, int i, const Cx<R> (&v)[12],
                                                     int v0, int v1) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 12u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int c = 0; c < 12; ++c)
      if (c >= v0 && c < v1)
        bst<AUX>(f, o, (uint32_t)c * (uint32_t)Vh * 16u, make_double2(v[c].re, v[c].im));
  }
  // Load only the storage vectors [v0, v1); other components are zero.
  __device__ static __forceinline__ void load_range(Rsrc f, int Vh, int p, int i, Cx<R> (&v)[12], int v0,
                                                    int v1) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 12u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      v[c] = {0.0, 0.0};
      if (c >= v0 && c < v1) {
        double2 t = bld<double2>(f, o, (uint32_t)c * (uint32_t)Vh * 16u);
        v[c] = {t.x, t.y};
      }
    }
  }
};

template <> struct SpinFmt<DIRAC_F32> {
  using R = float;
  static constexpr int NV = 6;
  static constexpr bool kScaled = false;
  static constexpr int kSiteBytes = 96;
  __device__ static __forceinline__ void load(Rsrc f, int Vh, int p, int i, Cx<R> (&v)[12]) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 6u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 t = bld<float4>(f, o, (uint32_t)k * (uint32_t)Vh * 16u);
      v[2 * k] = {t.x, t.y};
      v[2 * k + 1] = {t.z, t.w};
    }
  }
  __device__ static __forceinline__ void round(Cx<R> (&)[12]) {}
  // store(), returning in q the value left in memory (v itself here).
  template <int AUX = 0>
  __device__ static __forceinline__ void store_q(Rsrc f, int Vh, int p, int i, const Cx<R> (&v)[12],
                                                 Cx<R> (&q)[12]) {
    store<AUX>(f, Vh, p, i, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) q[c] = v[c];
  }
  template <int AUX = 0>
  __device__ static __forceinline__ void store(Rsrc f, int Vh, int p, int i, const Cx<R> (&v)[12]) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 6u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      bst<AUX>(f, o, (uint32_t)k * (uint32_t)Vh * 16u,
               make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im));
  }
  // Load only the storage vectors [v0, v1); other components are zero.
  __device__ static __forceinline__ void load_range(Rsrc f, int Vh, int p, int i, Cx<R> (&v)[12], int v0,
                                                    int v1) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 6u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      v[2 * k] = {0.f, 0.f};
      v[2 * k + 1] = {0.f, 0.f};
      if (k >= v0 && k < v1) {
        float4 t = bld<float4>(f, o, (uint32_t)k * (uint32_t)Vh * 16u);
        v[2 * k] = {t.x, t.y};
        v[2 * k + 1] = {t.z, t.w};
      }
    }
  }
  // Store only the storage vectors [v0, v1) (vector k holds components 2k, 2k+1).
  template <int AUX = 0>
  __device__ static __forceinline__ void store_range(Rsrc f, int Vh, int p, int i, const Cx<R> (&v)[12],
                                                     int v0, int v1) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 6u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k >= v0 && k < v1)
        bst<AUX>(f, o, (uint32_t)k * (uint32_t)Vh * 16u,
                 make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im));
  }
};

template <bool BF> struct SpinScaled {
  using R = float;
  static constexpr int NV = 3;
  static constexpr bool kScaled = true;
  static constexpr int kSiteBytes = 52;
  __device__ static __forceinline__ float dec(unsigned short h) { return BF ? bf16_to_f(h) : h_to_f(h); }
  __device__ static __forceinline__ unsigned short enc(float f) { return BF ? f_to_bf16(f) : f_to_h(f); }
  // the scales follow the 2 * Vh * 48 payload bytes
  __device__ static __forceinline__ uint32_t scale_off(int Vh, int p) {
    return (uint32_t)Vh * 96u + plane_off(p, (uint32_t)Vh * 4u);
  }
  __device__ static __forceinline__ void load(Rsrc f, int Vh, int p, int i, Cx<R> (&v)[12]) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 3u * (uint32_t)Vh * 16u);
    const float s = bld<float>(f, (uint32_t)i * 4u + scale_off(Vh, p), 0u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 t = bld<uint4>(f, o, (uint32_t)k * (uint32_t)Vh * 16u);
      unsigned w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[4 * k + j] = {s * dec((unsigned short)(w[j] & 0xFFFFu)), s * dec((unsigned short)(w[j] >> 16))};
        // the products are final here: the compiler may not fuse them into
        // the additions that follow (which it would do differently in
        // different kernel instances)
        asm("" : "+v"(v[4 * k + j].re), "+v"(v[4 * k + j].im));
      }
    }
  }
  // The 24 stored values unscaled, and the site scale: load() is s * v.
  __device__ static __forceinline__ void load_raw(Rsrc f, int Vh, int p, int i, Cx<R> (&v)[12], float& s) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 3u * (uint32_t)Vh * 16u);
    s = bld<float>(f, (uint32_t)i * 4u + scale_off(Vh, p), 0u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 t = bld<uint4>(f, o, (uint32_t)k * (uint32_t)Vh * 16u);
      unsigned w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v[4 * k + j] = {dec((unsigned short)(w[j] & 0xFFFFu)), dec((unsigned short)(w[j] >> 16))};
    }
  }
  // Site maximum |v|.
  __device__ static __forceinline__ float site_max(const Cx<R> (&v)[12]) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    return m;
  }
  // The payload v / m is formed as (v * pre) * inv: one division per site
  // instead of 24, within one float ulp of v / m, and the site maximum still
  // rounds to exactly +-1 in the 16-bit format.  pre = 1 and inv = 1 / m,
  // except for a denormal m (a site far out on the tail of a point-source
  // solve), whose reciprocal would overflow: there pre = 2^64 and
  // inv = 1 / (m 2^64), both scalings exact.  An all-zero site has inv = 0.
  __device__ static __forceinline__ void site_factors(float m, float& pre, float& inv) {
    pre = (m < 0x1p-126f) ? 0x1p64f : 1.f;
    inv = (m > 0.f) ? 1.f / (m * pre) : 0.f;
  }
  // Replace v by the value the store would leave in memory.
  __device__ static __forceinline__ void round(Cx<R> (&v)[12]) {
    const float m = site_max(v);
    float pre, inv;
    site_factors(m, pre, inv);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      v[c].re = m * dec(enc((v[c].re * pre) * inv));
      v[c].im = m * dec(enc((v[c].im * pre) * inv));
    }
  }
  template <int AUX = 0>
  __device__ static __forceinline__ void store(Rsrc f, int Vh, int p, int i, const Cx<R> (&v)[12]) {
    const float m = site_max(v);
    float pre, inv;
    site_factors(m, pre, inv);
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 3u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      unsigned w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float re = (v[4 * k + j].re * pre) * inv;
        const float im = (v[4 * k + j].im * pre) * inv;
        w[j] = (unsigned)enc(re) | ((unsigned)enc(im) << 16);
      }
      bst<AUX>(f, o, (uint32_t)k * (uint32_t)Vh * 16u, make_uint4(w[0], w[1], w[2], w[3]));
    }
    bst<AUX>(f, (uint32_t)i * 4u + scale_off(Vh, p), 0u, m);
  }
  // store(), returning in q the value left in memory (round() of v), both
  // from the one encoding: q = m * decode(payload).
  template <int AUX = 0>
  __device__ static __forceinline__ void store_q(Rsrc f, int Vh, int p, int i, const Cx<R> (&v)[12],
                                                 Cx<R> (&q)[12]) {
    const float m = site_max(v);
    float pre, inv;
    site_factors(m, pre, inv);
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 3u * (uint32_t)Vh * 16u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      unsigned w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned short re = enc((v[4 * k + j].re * pre) * inv);
        const unsigned short im = enc((v[4 * k + j].im * pre) * inv);
        w[j] = (unsigned)re | ((unsigned)im << 16);
        q[4 * k + j] = {m * dec(re), m * dec(im)};
      }
      bst<AUX>(f, o, (uint32_t)k * (uint32_t)Vh * 16u, make_uint4(w[0], w[1], w[2], w[3]));
    }
    bst<AUX>(f, (uint32_t)i * 4u + scale_off(Vh, p), 0u, m);
  }
};
template <> struct SpinFmt<DIRAC_F16S> : SpinScaled<false> {};
template <> struct SpinFmt<DIRAC_BF16S> : SpinScaled<true> {};

// Bytes of one spinor field (one right-hand side) in format P.
__host__ __device__ inline int64_t spinor_field_bytes(int prec, int64_t V) {
  switch (prec) {
    case DIRAC_F64: return V * 192;
    case DIRAC_F32: return V * 96;
    default: return V * 48 + V * 4;
  }
}

// Gauge links: [parity][mu][NL][Vh] vectors.  Entry k = 3*row + col of the
// row-major colour matrix; LINK12 stores rows 0 and 1 only, LINK10 row 0 and
// the pivot column's rows 1 and 2 (su3_from_row_pivot).
//   F64 18: 9 double2     F64 12: 6 double2
//   F32 18: 9 float2      F32 12: 3 float4 (two entries each)
//   F16S/BF16S 12: 3 x (4 x 16-bit) = two entries each, unscaled
template <int P, int LK> struct LinkFmt;

template <int LK> struct LinkF64 {
  using R = double;
  static constexpr int NL = LK / 2;
  static constexpr int kBytes = LK * 8;
  __device__ static __forceinline__ void load(Rsrc U, int Vh, int p, int mu, int i, M3<R>& u) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 4u * NL * (uint32_t)Vh * 16u);
    const uint32_t base = (uint32_t)(mu * NL) * (uint32_t)Vh * 16u;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      double2 t = bld<double2>(U, o, base + (uint32_t)k * (uint32_t)Vh * 16u);
      u.e[k / 3][k % 3] = {t.x, t.y};
    }
    if constexpr (LK == 12) su3_row2(u);
  }
};
template <> struct LinkFmt<DIRAC_F64, 18> : LinkF64<18> {};
template <> struct LinkFmt<DIRAC_F64, 12> : LinkF64<12> {};

template <> struct LinkFmt<DIRAC_F32, 18> {
  using R = float;
  static constexpr int NL = 9;
  static constexpr int kBytes = 72;
  __device__ static __forceinline__ void load(Rsrc U, int Vh, int p, int mu, int i, M3<R>& u) {
    const uint32_t o = (uint32_t)i * 8u + plane_off(p, 4u * 9u * (uint32_t)Vh * 8u);
    const uint32_t base = (uint32_t)(mu * 9) * (uint32_t)Vh * 8u;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 t = bld<float2>(U, o, base + (uint32_t)k * (uint32_t)Vh * 8u);
      u.e[k / 3][k % 3] = {t.x, t.y};
    }
  }
};
template <> struct LinkFmt<DIRAC_F32, 12> {
  using R = float;
  static constexpr int NL = 3;
  static constexpr int kBytes = 48;
  __device__ static __forceinline__ void load(Rsrc U, int Vh, int p, int mu, int i, M3<R>& u) {
    const uint32_t o = (uint32_t)i * 16u + plane_off(p, 4u * 3u * (uint32_t)Vh * 16u);
    const uint32_t base = (uint32_t)(mu * 3) * (uint32_t)Vh * 16u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float4 t = bld<float4>(U, o, base + (uint32_t)k * (uint32_t)Vh * 16u);
      u.e[(2 * k) / 3][(2 * k) % 3] = {t.x, t.y};
      u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {t.z, t.w};
    }
    su3_row2(u);
  }
};
// 10-real links (su3_from_row_pivot): per (parity, mu) block of 40 Vh bytes,
// plane A = (U_00, U_01), plane B = (U_02, U_1k) as float4, plane C = U_2k
// as float2.
template <> struct LinkFmt<DIRAC_F32, 10> {
  using R = float;
  static constexpr int NL = 3;
  static constexpr int kBytes = 40;
  __device__ static __forceinline__ void load(Rsrc U, int Vh, int p, int mu, int i, M3<R>& u) {
    const uint32_t blk = 40u * (uint32_t)Vh;  // bytes of one (parity, mu) block
    const uint32_t po = plane_off(p, 4u * blk);
    const uint32_t base = (uint32_t)mu * blk;
    const float4 A = bld<float4>(U, (uint32_t)i * 16u + po, base);
    const float4 B = bld<float4>(U, (uint32_t)i * 16u + po, base + 16u * (uint32_t)Vh);
    const float2 C = bld<float2>(U, (uint32_t)i * 8u + po, base + 32u * (uint32_t)Vh);
    u.e[0][0] = {A.x, A.y};
    u.e[0][1] = {A.z, A.w};
    u.e[0][2] = {B.x, B.y};
    su3_from_row_pivot(u, Cx<R>{B.z, B.w}, Cx<R>{C.x, C.y});
  }
};

template <bool BF> struct LinkHalf12 {
  using R = float;
  static constexpr int NL = 3;
  static constexpr int kBytes = 24;
  __device__ static __forceinline__ float dec(unsigned short h) { return BF ? bf16_to_f(h) : h_to_f(h); }
  __device__ static __forceinline__ void load(Rsrc U, int Vh, int p, int mu, int i, M3<R>& u) {
    const uint32_t o = (uint32_t)i * 8u + plane_off(p, 4u * 3u * (uint32_t)Vh * 8u);
    const uint32_t base = (uint32_t)(mu * 3) * (uint32_t)Vh * 8u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint2 t = bld<uint2>(U, o, base + (uint32_t)k * (uint32_t)Vh * 8u);
      u.e[(2 * k) / 3][(2 * k) % 3] = {dec(t.x & 0xFFFFu), dec(t.x >> 16)};
      u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {dec(t.y & 0xFFFFu), dec(t.y >> 16)};
    }
    float zero = 0.f;
    asm("" : "+v"(zero));
    su3_row2_fma(u, zero);
  }
};
template <> struct LinkFmt<DIRAC_F16S, 12> : LinkHalf12<false> {};
template <> struct LinkFmt<DIRAC_BF16S, 12> : LinkHalf12<true> {};

// 10-real 16-bit links: per (parity, mu) block of 20 Vh bytes, plane A =
// (U_00, U_01, U_02, U_1k) as 8 x 16 bits, plane B = U_2k as 2 x 16 bits.
struct LinkHalf10 {
  using R = float;
  static constexpr int NL = 2;
  static constexpr int kBytes = 20;
  __device__ static __forceinline__ float dec(unsigned short h) { return h_to_f(h); }
  __device__ static __forceinline__ void load(Rsrc U, int Vh, int p, int mu, int i, M3<R>& u) {
    const uint32_t blk = 20u * (uint32_t)Vh;
    const uint32_t po = plane_off(p, 4u * blk);
    const uint32_t base = (uint32_t)mu * blk;
    const uint4 A = bld<uint4>(U, (uint32_t)i * 16u + po, base);
    const unsigned C = bld<unsigned>(U, (uint32_t)i * 4u + po, base + 16u * (uint32_t)Vh);
    u.e[0][0] = {dec(A.x & 0xFFFFu), dec(A.x >> 16)};
    u.e[0][1] = {dec(A.y & 0xFFFFu), dec(A.y >> 16)};
    u.e[0][2] = {dec(A.z & 0xFFFFu), dec(A.z >> 16)};
    su3_from_row_pivot(u, Cx<R>{dec(A.w & 0xFFFFu), dec(A.w >> 16)}, Cx<R>{dec(C & 0xFFFFu), dec(C >> 16)});
  }
};
template <> struct LinkFmt<DIRAC_F16S, 10> : LinkHalf10 {};

__host__ __device__ inline int64_t link_bytes(int prec, int link) {
  if (prec == DIRAC_F64) return link * 8;
  if (prec == DIRAC_F32) return link * 4;
  return link * 2;
}

// -------------------------------------------------- spin projection ------
// Chiral basis: gamma_mu = [[0, s_mu], [s_mu^dag, 0]] with s_1 = -i sigma_x,
// s_2 = -i sigma_y, s_3 = -i sigma_z, s_4 = 1.  For psi = (u, d) (upper and
// lower spin pairs) and sign s = +-1:
//   (1 - s gamma) psi = (h, -s s_mu^dag h),  h = u - s s_mu d
//   (1 + s gamma) psi = (h,  s s_mu^dag h),  h = u + s s_mu d
// so each hop needs one half spinor (two colour vectors) and one SU(3)
// product per spin row of the half spinor.

// (s_mu d)_k for spin k = 0, 1 of the half spinor; d0/d1 colour component a.
template <int MU, int K, class R>
__device__ __forceinline__ Cx<R> sig_d(Cx<R> d0, Cx<R> d1) {
  if constexpr (MU == 0) return K == 0 ? mul_mi(d1) : mul_mi(d0);  // (-i d1, -i d0)
  else if constexpr (MU == 1) return K == 0 ? neg(d1) : d0;        // (-d1, d0)
  else if constexpr (MU == 2) return K == 0 ? mul_mi(d0) : mul_i(d1);  // (-i d0, i d1)
  else return K == 0 ? d0 : d1;                                    // (d0, d1)
}

// (s_mu^dag h)_k for spin k = 0, 1 of the lower pair.
template <int MU, int K, class R>
__device__ __forceinline__ Cx<R> sigdag_h(Cx<R> h0, Cx<R> h1) {
  if constexpr (MU == 0) return K == 0 ? mul_i(h1) : mul_i(h0);    // (i h1, i h0)
  else if constexpr (MU == 1) return K == 0 ? h1 : neg(h0);        // (h1, -h0)
  else if constexpr (MU == 2) return K == 0 ? mul_i(h0) : mul_mi(h1);  // (i h0, -i h1)
  else return K == 0 ? h0 : h1;                                    // (h0, h1)
}

// Half spinor h = u + SG * s_mu d of a full spinor v (SG = +1 or -1).
template <int MU, int SG, class R>
__device__ __forceinline__ void project(const Cx<R> (&v)[12], Cx<R> (&h)[2][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Cx<R> d0 = v[6 + a], d1 = v[9 + a];
    Cx<R> e0 = sig_d<MU, 0>(d0, d1), e1 = sig_d<MU, 1>(d0, d1);
    if constexpr (SG > 0) {
      h[0][a] = v[a] + e0;
      h[1][a] = v[3 + a] + e1;
    } else {
      h[0][a] = v[a] - e0;
      h[1][a] = v[3 + a] - e1;
    }
  }
}

// project() for the stored values of a 16-bit site (decoded, unscaled): the
// same sums, each written as fma(e, +-one, u) with one = 1 kept opaque to the
// compiler, so that it is a single mixed-precision fused multiply-add reading
// both 16-bit operands directly instead of two conversions and an addition.
// The product by +-1 is exact, so every h equals project()'s rounded sum.
template <int MU, int SG, class R>
__device__ __forceinline__ void project_fma1(const Cx<R> (&v)[12], Cx<R> (&h)[2][3], R one) {
  const R sg = SG > 0 ? one : -one;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const Cx<R> d0 = v[6 + a], d1 = v[9 + a];
    const Cx<R> e0 = sig_d<MU, 0>(d0, d1), e1 = sig_d<MU, 1>(d0, d1);
    h[0][a] = {fma(e0.re, sg, v[a].re), fma(e0.im, sg, v[a].im)};
    h[1][a] = {fma(e1.re, sg, v[3 + a].re), fma(e1.im, sg, v[3 + a].im)};
  }
}

// acc += (w, SG * s_mu^dag w) for a half spinor w (the hop's contribution).
template <int MU, int SG, class R>
__device__ __forceinline__ void reconstruct_add(Cx<R> (&acc)[12], const Cx<R> (&w)[2][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[a] = acc[a] + w[0][a];
    acc[3 + a] = acc[3 + a] + w[1][a];
    Cx<R> l0 = sigdag_h<MU, 0>(w[0][a], w[1][a]);
    Cx<R> l1 = sigdag_h<MU, 1>(w[0][a], w[1][a]);
    if constexpr (SG > 0) {
      acc[6 + a] = acc[6 + a] + l0;
      acc[9 + a] = acc[9 + a] + l1;
    } else {
      acc[6 + a] = acc[6 + a] - l0;
      acc[9 + a] = acc[9 + a] - l1;
    }
  }
}

// acc += s (w, SG * s_mu^dag w): the same with the half spinor scaled by s on
// the way.  The projection, the colour product and s_mu^dag are linear, so a
// neighbour stored as s * v (a scaled 16-bit site) can be projected and
// multiplied unscaled and take its scale here, in fused multiply-adds that
// replace the additions, instead of in 24 multiplications at the load.
template <int MU, int SG, class R>
__device__ __forceinline__ void reconstruct_fma(Cx<R> (&acc)[12], const Cx<R> (&w)[2][3], R s) {
  const R sl = SG > 0 ? s : -s;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[a].re = fma(s, w[0][a].re, acc[a].re);
    acc[a].im = fma(s, w[0][a].im, acc[a].im);
    acc[3 + a].re = fma(s, w[1][a].re, acc[3 + a].re);
    acc[3 + a].im = fma(s, w[1][a].im, acc[3 + a].im);
    const Cx<R> l0 = sigdag_h<MU, 0>(w[0][a], w[1][a]);
    const Cx<R> l1 = sigdag_h<MU, 1>(w[0][a], w[1][a]);
    acc[6 + a].re = fma(sl, l0.re, acc[6 + a].re);
    acc[6 + a].im = fma(sl, l0.im, acc[6 + a].im);
    acc[9 + a].re = fma(sl, l1.re, acc[9 + a].re);
    acc[9 + a].im = fma(sl, l1.im, acc[9 + a].im);
  }
}

// su3_mul / su3_dag_mul with every product a fused multiply-add from `zero`
// (= 0, kept opaque), for links held as decoded 16-bit values: see
// su3_row2_fma.
template <class R>
__device__ __forceinline__ void su3_mul_fma(const M3<R>& u, const Cx<R> (&h)[2][3], Cx<R> (&w)[2][3], R zero) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cx<R> t = cmadd(Cx<R>{zero, zero}, u.e[a][0], h[s][0]);
      t = cmadd(t, u.e[a][1], h[s][1]);
      t = cmadd(t, u.e[a][2], h[s][2]);
      w[s][a] = t;
    }
}
template <class R>
__device__ __forceinline__ void su3_dag_mul_fma(const M3<R>& u, const Cx<R> (&h)[2][3], Cx<R> (&w)[2][3], R zero) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cx<R> t = cjmadd(Cx<R>{zero, zero}, u.e[0][a], h[s][0]);
      t = cjmadd(t, u.e[1][a], h[s][1]);
      t = cjmadd(t, u.e[2][a], h[s][2]);
      w[s][a] = t;
    }
}

// w = U h, and w = U^dag h, per spin row of the half spinor.
template <class R>
__device__ __forceinline__ void su3_mul(const M3<R>& u, const Cx<R> (&h)[2][3], Cx<R> (&w)[2][3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cx<R> t = cmul(u.e[a][0], h[s][0]);
      t = cmadd(t, u.e[a][1], h[s][1]);
      t = cmadd(t, u.e[a][2], h[s][2]);
      w[s][a] = t;
    }
}
template <class R>
__device__ __forceinline__ void su3_dag_mul(const M3<R>& u, const Cx<R> (&h)[2][3], Cx<R> (&w)[2][3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cx<R> t = cmul(conj(u.e[0][a]), h[s][0]);
      t = cjmadd(t, u.e[1][a], h[s][1]);
      t = cjmadd(t, u.e[2][a], h[s][2]);
      w[s][a] = t;
    }
}

// ------------------------------------------------------ solver scalars ----
// Per right-hand-side scalar state of a CG run, kept in device memory so
// that iterations can be enqueued back to back without host round trips.
struct CgState {
  double rho;     // <r, r> of the current residual
  double alpha;   // step of the current iteration
  double beta;    // direction update coefficient of the current iteration
  double stop2;   // inner loop ends when rho < stop2
  double res[2];  // result of the last plain reduction (re, im)
  double coef[4]; // host-set coefficients for the linear-combination kernels
  int iters;      // iterations completed in this run
  int kmax;       // iteration cap of this run
  int done;       // no more iterations for this right-hand side
  int active;     // the iteration in flight updates this right-hand side
  int status;     // DIRAC_OK / DIRAC_EBREAKDOWN
  int pad[3];
};

enum FinalizeKind : int {
  kFinPlain = 0,   // res = sum
  kFinAlpha = 1,   // alpha = rho / sum (start of an iteration)
  kFinRho = 2,     // rho_new = sum: beta, rho, iters, done
  kFinRhoSet = 3,  // rho = sum (start of a run)
};

__device__ __forceinline__ void cg_finalize(CgState& st, int kind, double s0, double s1) {
  if (kind == kFinPlain) {
    st.res[0] = s0;
    st.res[1] = s1;
  } else if (kind == kFinRhoSet) {
    st.rho = s0;
    st.res[0] = s0;
    st.res[1] = 0.0;
  } else if (kind == kFinAlpha) {
    if (st.done) {
      st.active = 0;
      st.alpha = 0.0;
    } else if (!(s0 > 0.0) || !isfinite(s0) || !isfinite(st.rho)) {
      st.active = 0;
      st.alpha = 0.0;
      st.done = 1;
      st.status = DIRAC_EBREAKDOWN;
    } else {
      st.active = 1;
      st.alpha = st.rho / s0;
    }
  } else if (kind == kFinRho) {
    if (st.active) {
      if (!isfinite(s0)) {
        st.done = 1;
        st.status = DIRAC_EBREAKDOWN;
        st.beta = 0.0;
      } else {
        st.beta = s0 / st.rho;
        st.rho = s0;
      }
      st.iters += 1;
      if (st.rho < st.stop2 || st.iters >= st.kmax) st.done = 1;
    }
  }
}

// ---------------------------------------------- deterministic reduction ----
// Two stages, both in a fixed order: each block reduces NC float64 values per
// right-hand side over its threads and stores them to
// partials[(rhs * nparts + part) * NC + c]; a second kernel (k_finalize, one
// block per right-hand side) sums the partials and applies cg_finalize.  The
// kernel boundary between the stages makes the partials visible; no atomics
// and no device-scope fences are needed (on a multi-XCD device a device-scope
// release fence in every block would write back the L2 each time).

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

struct RedArgs {
  double* partials;    // [nrhs][nparts][NC]
  CgState* state;      // [nrhs]
  int kind;
};

// vals[r][c] are this thread's contributions for right-hand side rhs0 + r
// (r < RPT); blockDim.x is a multiple of 64.  part/nparts: this block's slot
// among the blocks that cover one right-hand side.
template <int RPT, int NC>
__device__ void block_reduce_store(const RedArgs& ra, double (&vals)[RPT][NC], int rhs0, int nrhs, int part,
                                   int nparts) {
  __shared__ double red[16][RPT * NC];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int nwaves = blockDim.x >> 6;
#pragma unroll
  for (int r = 0; r < RPT; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double s = wave_sum(vals[r][c]);
      if (lane == 0) red[wave][r * NC + c] = s;
    }
  __syncthreads();
  if (tid < RPT * NC) {
    const int r = tid / NC, c = tid % NC;
    const int rhs = rhs0 + r;
    if (rhs < nrhs) {
      double s = 0.0;
      for (int w = 0; w < nwaves; ++w) s += red[w][r * NC + c];
      ra.partials[((size_t)rhs * nparts + part) * NC + c] = s;
    }
  }
}

}  // namespace dirac
