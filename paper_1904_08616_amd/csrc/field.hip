// Site-wise field kernels: layout conversion between the canonical
// complex128 arrays and the internal even-odd formats, precision
// conversion, and the BLAS-1 steps of the CG (Algorithm 1: inner products,
// residual norms, vector updates).  One thread per (site, right-hand side),
// except the float64 / float32 CG update, which is element-wise and streams
// each field as one array; component planes are read with coalesced 16-byte
// vectors.  Every
// reduction accumulates in float64 and finishes in a fixed order.
#include <type_traits>

#include "field.h"

namespace dirac {

namespace {

constexpr int kBlock = 256;

struct SiteGrid {
  int nb;      // blocks per parity
  int nparts;  // blocks per right-hand side (reduction partials)
  dim3 grid;
};

// Both parities, or only parity g.vpar (the even-odd solve's half vectors).
SiteGrid site_grid(const Geom& g, int nrhs) {
  SiteGrid s;
  s.nb = (g.Vh + kBlock - 1) / kBlock;
  s.nparts = (g.vpar < 0 ? 2 : 1) * s.nb;
  s.grid = dim3(s.nparts, nrhs);
  return s;
}

struct SiteIdx {
  int p, i, rhs;
  bool valid;
};

__device__ __forceinline__ SiteIdx site_idx(const Geom& g, int nb) {
  SiteIdx s;
  if (g.vpar >= 0) {
    s.p = g.vpar;
    s.i = blockIdx.x * kBlock + threadIdx.x;
  } else {
    s.p = blockIdx.x >= (unsigned)nb ? 1 : 0;
    s.i = (blockIdx.x - s.p * nb) * kBlock + threadIdx.x;
  }
  s.rhs = blockIdx.y;
  s.valid = s.i < g.Vh;
  return s;
}

struct FieldDev {
  const char* ptr;
  int64_t stride;
  uint32_t bytes;
};

__device__ __forceinline__ Rsrc field_rsrc(const FieldDev& f, int rhs) {
  return make_rsrc(f.ptr + (size_t)rhs * f.stride, f.bytes);
}

FieldDev dev(const FieldRef& f) { return FieldDev{f.ptr, f.stride, f.bytes}; }

template <class To, class From>
__device__ __forceinline__ void cvt(const Cx<From> (&a)[12], Cx<To> (&b)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) b[c] = {(To)a[c].re, (To)a[c].im};
}

// Lexicographic site number of checkerboard site (p, i).
__device__ __forceinline__ int64_t lex_site(const Geom& g, int p, int i) {
  Coord c = cb_coords(g, p, i);
  return 2 * (int64_t)i + (c.x & 1);
}

// ------------------------------------------------------------ pack ------
template <int P>
__global__ void __launch_bounds__(kBlock) k_pack_spinor(Geom g, int nb, const double2* src, FieldDev dst) {
  SiteIdx s = site_idx(g, nb);
  if (!s.valid) return;
  const int64_t V = 2 * (int64_t)g.Vh;
  const double2* q = src + ((size_t)s.rhs * V + lex_site(g, s.p, s.i)) * 12;
  Cx<double> v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    double2 t = q[c];
    v[c] = {t.x, t.y};
  }
  using F = SpinFmt<P>;
  Cx<typename F::R> w[12];
  cvt(v, w);
  F::store(field_rsrc(dst, s.rhs), g.Vh, s.p, s.i, w);
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_unpack_spinor(Geom g, int nb, FieldDev src, double2* dst) {
  SiteIdx s = site_idx(g, nb);
  if (!s.valid) return;
  using F = SpinFmt<P>;
  Cx<typename F::R> w[12];
  F::load(field_rsrc(src, s.rhs), g.Vh, s.p, s.i, w);
  const int64_t V = 2 * (int64_t)g.Vh;
  double2* q = dst + ((size_t)s.rhs * V + lex_site(g, s.p, s.i)) * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) q[c] = make_double2((double)w[c].re, (double)w[c].im);
}

// Links: canonical [site][mu][3][3] complex128 -> [parity][mu][NL][Vh].
template <int P, int LK>
__global__ void __launch_bounds__(kBlock) k_pack_gauge(Geom g, int nb, const double2* U, char* out) {
  SiteIdx s = site_idx(g, nb);
  if (!s.valid) return;
  const int64_t n = lex_site(g, s.p, s.i);
  const size_t Vh = (size_t)g.Vh;
  const int nent = LK / 2;  // complex entries stored per link
  for (int mu = 0; mu < 4; ++mu) {
    const double2* m = U + ((size_t)n * 4 + mu) * 9;
    if constexpr (P == DIRAC_F64) {
      double2* b = reinterpret_cast<double2*>(out) + ((size_t)(s.p * 4 + mu) * nent) * Vh + s.i;
      for (int k = 0; k < nent; ++k) b[k * Vh] = m[k];
    } else if constexpr (LK == 10) {
      // row 0 as stored, the pivot chosen on it as the rebuild chooses it
      // (su3_from_row_pivot), then the pivot column's rows 1 and 2
      auto enc = [](double x) -> unsigned { return (unsigned)f_to_h((float)x); };
      Cx<float> r[3];
      unsigned h[3] = {0u, 0u, 0u};
      for (int c = 0; c < 3; ++c) {
        if constexpr (P == DIRAC_F32) {
          r[c] = {(float)m[c].x, (float)m[c].y};
        } else {
          h[c] = enc(m[c].x) | (enc(m[c].y) << 16);
          r[c] = {h_to_f(h[c] & 0xFFFFu), h_to_f(h[c] >> 16)};
        }
      }
      const float m0 = abs2_exact(r[0]), m1 = abs2_exact(r[1]), m2 = abs2_exact(r[2]);
      const int k = (m0 <= m1 && m0 <= m2) ? 0 : (m1 <= m2 ? 1 : 2);
      const double2 bk = m[3 + k], ck = m[6 + k];
      char* blk = out + (size_t)(s.p * 4 + mu) * (size_t)(LinkFmt<P, 10>::kBytes) * Vh;
      if constexpr (P == DIRAC_F32) {
        reinterpret_cast<float4*>(blk)[s.i] = make_float4(r[0].re, r[0].im, r[1].re, r[1].im);
        reinterpret_cast<float4*>(blk + 16 * Vh)[s.i] = make_float4(r[2].re, r[2].im, (float)bk.x, (float)bk.y);
        reinterpret_cast<float2*>(blk + 32 * Vh)[s.i] = make_float2((float)ck.x, (float)ck.y);
      } else {
        reinterpret_cast<uint4*>(blk)[s.i] = make_uint4(h[0], h[1], h[2], enc(bk.x) | (enc(bk.y) << 16));
        reinterpret_cast<unsigned*>(blk + 16 * Vh)[s.i] = enc(ck.x) | (enc(ck.y) << 16);
      }
    } else if constexpr (P == DIRAC_F32 && LK == 18) {
      float2* b = reinterpret_cast<float2*>(out) + ((size_t)(s.p * 4 + mu) * 9) * Vh + s.i;
      for (int k = 0; k < 9; ++k) b[k * Vh] = make_float2((float)m[k].x, (float)m[k].y);
    } else if constexpr (P == DIRAC_F32) {
      float4* b = reinterpret_cast<float4*>(out) + ((size_t)(s.p * 4 + mu) * 3) * Vh + s.i;
      for (int k = 0; k < 3; ++k)
        b[k * Vh] = make_float4((float)m[2 * k].x, (float)m[2 * k].y, (float)m[2 * k + 1].x,
                                (float)m[2 * k + 1].y);
    } else {
      uint2* b = reinterpret_cast<uint2*>(out) + ((size_t)(s.p * 4 + mu) * 3) * Vh + s.i;
      auto enc = [](double x) -> unsigned {
        return P == DIRAC_BF16S ? (unsigned)f_to_bf16((float)x) : (unsigned)f_to_h((float)x);
      };
      for (int k = 0; k < 3; ++k) {
        unsigned lo = enc(m[2 * k].x) | (enc(m[2 * k].y) << 16);
        unsigned hi = enc(m[2 * k + 1].x) | (enc(m[2 * k + 1].y) << 16);
        b[k * Vh] = make_uint2(lo, hi);
      }
    }
  }
}

// --------------------------------------------------------- reductions ----
template <int NC>
__device__ __forceinline__ void site_reduce(const RedArgs& ra, double (&v)[NC], int nrhs, int nb) {
  double vals[1][NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) vals[0][c] = v[c];
  (void)nb;
  block_reduce_store<1, NC>(ra, vals, blockIdx.y, nrhs, blockIdx.x, gridDim.x);
}

RedArgs red_args(const RedTarget& t) { return RedArgs{t.partials, t.state, t.kind}; }

// One block per right-hand side: fixed-order sum of its partials.
constexpr int kFinBlock = 1024;
template <int NC>
__global__ void __launch_bounds__(kFinBlock) k_finalize(RedArgs ra, int nparts) {
  __shared__ double tree[kFinBlock][NC];
  const int rhs = blockIdx.x;
  const int tid = threadIdx.x;
  double s[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = 0.0;
  const double* p = ra.partials + (size_t)rhs * nparts * NC;
  for (int b = tid; b < nparts; b += kFinBlock)
#pragma unroll
    for (int c = 0; c < NC; ++c) s[c] += p[(size_t)b * NC + c];
#pragma unroll
  for (int c = 0; c < NC; ++c) tree[tid][c] = s[c];
  __syncthreads();
  for (int w = kFinBlock / 2; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int c = 0; c < NC; ++c) tree[tid][c] += tree[tid + w][c];
    __syncthreads();
  }
  if (tid == 0) cg_finalize(ra.state[rhs], ra.kind, tree[0][0], NC > 1 ? tree[0][NC - 1] : 0.0);
}

// dst = c * src, optional |dst|^2
template <int PS, int PD, bool NORM>
__global__ void __launch_bounds__(kBlock) k_convert(Geom g, int nb, int nrhs, FieldDev src, FieldDev dst,
                                                    const CgState* cs, int ci, RedArgs ra) {
  SiteIdx s = site_idx(g, nb);
  double n2[1] = {0.0};
  if (s.valid) {
    using FS = SpinFmt<PS>;
    using FD = SpinFmt<PD>;
    Cx<typename FS::R> a[12];
    FS::load(field_rsrc(src, s.rhs), g.Vh, s.p, s.i, a);
    if (cs != nullptr && ci >= 0) {
      const typename FS::R c = (typename FS::R)cs[s.rhs].coef[ci];
#pragma unroll
      for (int k = 0; k < 12; ++k) a[k] = c * a[k];
    }
    Cx<typename FD::R> b[12];
    cvt(a, b);
    FD::store(field_rsrc(dst, s.rhs), g.Vh, s.p, s.i, b);
    if constexpr (NORM) {
      FD::round(b);  // norm of the value as stored
#pragma unroll
      for (int k = 0; k < 12; ++k) n2[0] += (double)b[k].re * b[k].re + (double)b[k].im * b[k].im;
    }
  }
  if constexpr (NORM) site_reduce<1>(ra, n2, nrhs, nb);
}

template <int PA, int PB>
__global__ void __launch_bounds__(kBlock) k_dot(Geom g, int nb, int nrhs, FieldDev a, FieldDev b, RedArgs ra) {
  SiteIdx s = site_idx(g, nb);
  double v[2] = {0.0, 0.0};
  if (s.valid) {
    Cx<typename SpinFmt<PA>::R> x[12];
    Cx<typename SpinFmt<PB>::R> y[12];
    SpinFmt<PA>::load(field_rsrc(a, s.rhs), g.Vh, s.p, s.i, x);
    SpinFmt<PB>::load(field_rsrc(b, s.rhs), g.Vh, s.p, s.i, y);
#pragma unroll
    for (int k = 0; k < 12; ++k) {  // conj(x) y
      v[0] += (double)x[k].re * y[k].re + (double)x[k].im * y[k].im;
      v[1] += (double)x[k].re * y[k].im - (double)x[k].im * y[k].re;
    }
  }
  site_reduce<2>(ra, v, nrhs, nb);
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_norm2(Geom g, int nb, int nrhs, FieldDev a, RedArgs ra) {
  SiteIdx s = site_idx(g, nb);
  double v[1] = {0.0};
  if (s.valid) {
    Cx<typename SpinFmt<P>::R> x[12];
    SpinFmt<P>::load(field_rsrc(a, s.rhs), g.Vh, s.p, s.i, x);
#pragma unroll
    for (int k = 0; k < 12; ++k) v[0] += (double)x[k].re * x[k].re + (double)x[k].im * x[k].im;
  }
  site_reduce<1>(ra, v, nrhs, nb);
}

// y = a x + b y (complex a, b)
template <int PX, int PY>
__global__ void __launch_bounds__(kBlock) k_axpby(Geom g, int nb, FieldDev x, FieldDev y, const CgState* st,
                                                  double are, double aim, double bre, double bim) {
  SiteIdx s = site_idx(g, nb);
  if (!s.valid) return;
  if (st != nullptr) {
    are = st[s.rhs].coef[0];
    aim = st[s.rhs].coef[1];
    bre = st[s.rhs].coef[2];
    bim = st[s.rhs].coef[3];
  }
  using RY = typename SpinFmt<PY>::R;
  Cx<typename SpinFmt<PX>::R> xv[12];
  Cx<RY> yv[12];
  SpinFmt<PX>::load(field_rsrc(x, s.rhs), g.Vh, s.p, s.i, xv);
  SpinFmt<PY>::load(field_rsrc(y, s.rhs), g.Vh, s.p, s.i, yv);
  const Cx<RY> A = {(RY)are, (RY)aim}, B = {(RY)bre, (RY)bim};
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    Cx<RY> xk = {(RY)xv[k].re, (RY)xv[k].im};
    yv[k] = cmadd(cmul(B, yv[k]), A, xk);
  }
  SpinFmt<PY>::store(field_rsrc(y, s.rhs), g.Vh, s.p, s.i, yv);
}

// x += alpha p; p = r + beta p   (where the right-hand side is active).  In
// float64 the three fields' 36 loads take 144 registers: the register budget
// of three waves per SIMD lets every load be in flight before the first wait.
template <int PX, int PP, int PR>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PX == DIRAC_F64 ? 3 : 4)))
k_cg_xp(Geom g, int nb, FieldDev x, FieldDev p, FieldDev r, const CgState* st) {
  SiteIdx s = site_idx(g, nb);
  if (!s.valid) return;
  const CgState& S = st[s.rhs];
  if (!S.active) return;
  using RX = typename SpinFmt<PX>::R;
  using RP = typename SpinFmt<PP>::R;
  Cx<RX> xv[12];
  Cx<RP> pv[12];
  Cx<typename SpinFmt<PR>::R> rv[12];
  const Rsrc xr = field_rsrc(x, s.rhs), pr = field_rsrc(p, s.rhs);
  SpinFmt<PX>::load(xr, g.Vh, s.p, s.i, xv);
  SpinFmt<PP>::load(pr, g.Vh, s.p, s.i, pv);
  SpinFmt<PR>::load(field_rsrc(r, s.rhs), g.Vh, s.p, s.i, rv);
  __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
  const RX alpha = (RX)S.alpha;
  const RP beta = (RP)S.beta;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    xv[k].re = fma(alpha, (RX)pv[k].re, xv[k].re);
    xv[k].im = fma(alpha, (RX)pv[k].im, xv[k].im);
    pv[k].re = fma(beta, pv[k].re, (RP)rv[k].re);
    pv[k].im = fma(beta, pv[k].im, (RP)rv[k].im);
  }
  SpinFmt<PX>::store(xr, g.Vh, s.p, s.i, xv);
  SpinFmt<PP>::store(pr, g.Vh, s.p, s.i, pv);
}

// The same update when x, p and r share one unscaled format (float64 or
// float32): it is element-wise, so it runs over each right-hand side's field
// (or the parity plane of the even-odd vectors) as one array of 16-byte
// elements, one per thread, consecutive threads on consecutive elements.
// The site-wise kernel above holds 36 loads per thread in 12 planes per
// field; this one streams three arrays and computes the same values.  AUX 2
// marks loads and stores non-temporal (fields well beyond the last-level
// cache, where nothing is kept for the next kernel anyway).
template <int P, int AUX>
__global__ void __launch_bounds__(kBlock) k_cg_xp_flat(FieldDev x, FieldDev p, FieldDev r, const CgState* st,
                                                       uint32_t off0, uint32_t n16) {
  const int rhs = blockIdx.y;
  const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n16 || !st[rhs].active) return;
  const uint32_t o = off0 + k * 16u;
  const Rsrc xr = field_rsrc(x, rhs), pr = field_rsrc(p, rhs), rr = field_rsrc(r, rhs);
  using T = typename std::conditional<P == DIRAC_F64, double2, float4>::type;
  using R = typename SpinFmt<P>::R;
  auto ld = [&](Rsrc f) { return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(f, o, 0, AUX)); };
  T xv = ld(xr), pv = ld(pr);
  const T rv = ld(rr);
  const R alpha = (R)st[rhs].alpha, beta = (R)st[rhs].beta;
  if constexpr (P == DIRAC_F64) {
    xv.x = fma(alpha, pv.x, xv.x);
    xv.y = fma(alpha, pv.y, xv.y);
    pv.x = fma(beta, pv.x, rv.x);
    pv.y = fma(beta, pv.y, rv.y);
  } else {
    xv.x = fma(alpha, pv.x, xv.x);
    xv.y = fma(alpha, pv.y, xv.y);
    xv.z = fma(alpha, pv.z, xv.z);
    xv.w = fma(alpha, pv.w, xv.w);
    pv.x = fma(beta, pv.x, rv.x);
    pv.y = fma(beta, pv.y, rv.y);
    pv.z = fma(beta, pv.z, rv.z);
    pv.w = fma(beta, pv.w, rv.w);
  }
  bst<AUX>(xr, o, 0u, xv);
  bst<AUX>(pr, o, 0u, pv);
}

// y = a x + b y (complex a, b; from the CG state when st is given) when x
// and y share one unscaled format: element-wise over the field (or the
// parity plane of the even-odd vectors), the same products as k_axpby.
template <int P>
__global__ void __launch_bounds__(kBlock) k_axpby_flat(FieldDev x, FieldDev y, const CgState* st, double are,
                                                       double aim, double bre, double bim, uint32_t off0,
                                                       uint32_t n16) {
  const int rhs = blockIdx.y;
  const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n16) return;
  if (st != nullptr) {
    are = st[rhs].coef[0];
    aim = st[rhs].coef[1];
    bre = st[rhs].coef[2];
    bim = st[rhs].coef[3];
  }
  using R = typename SpinFmt<P>::R;
  using T = typename std::conditional<P == DIRAC_F64, double2, float4>::type;
  const uint32_t o = off0 + k * 16u;
  const Rsrc xr = field_rsrc(x, rhs), yr = field_rsrc(y, rhs);
  const T xv = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(xr, o, 0, 0));
  T yv = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(yr, o, 0, 0));
  const Cx<R> A = {(R)are, (R)aim}, B = {(R)bre, (R)bim};
  if constexpr (P == DIRAC_F64) {
    const Cx<R> w = cmadd(cmul(B, Cx<R>{yv.x, yv.y}), A, Cx<R>{xv.x, xv.y});
    yv = make_double2(w.re, w.im);
  } else {
    const Cx<R> w0 = cmadd(cmul(B, Cx<R>{yv.x, yv.y}), A, Cx<R>{xv.x, xv.y});
    const Cx<R> w1 = cmadd(cmul(B, Cx<R>{yv.z, yv.w}), A, Cx<R>{xv.z, xv.w});
    yv = make_float4(w0.re, w0.im, w1.re, w1.im);
  }
  bst<0>(yr, o, 0u, yv);
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_zero(Geom g, int nb, FieldDev f) {
  SiteIdx s = site_idx(g, nb);
  if (!s.valid) return;
  using F = SpinFmt<P>;
  Cx<typename F::R> z[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) z[k] = {0, 0};
  F::store(field_rsrc(f, s.rhs), g.Vh, s.p, s.i, z);
}

// ------------------------------------------------------------- force -----
// F_mu(n) = coeff/2 [ sum_a h^{g(n)}_a (x) h^{psi(n+mu)}_a^*        (P = 1 - gamma_mu)
//                   + sum_a h^{psi(n)}_a (x) h^{g(n+mu)}_a^* ]     (P = 1 + gamma_mu)
// where h are the upper projected spin rows: for P = 1 -+ gamma_mu the
// colour-spin outer product summed over all four spins equals the sum over
// the two half-spinor rows (P is twice a Hermitian projector).
template <int MU, class R>
__device__ __forceinline__ void force_dir(const Geom& g, const Rsrc& gr, const Rsrc& pr, int p, int i,
                                          const Coord& c, const Cx<R> (&gn)[12], const Cx<R> (&pn)[12],
                                          double scale, double2* out, int stride) {
  using F = SpinFmt<(sizeof(R) == 8) ? DIRAC_F64 : DIRAC_F32>;
  const int j = nb_fwd<MU>(g, c, i);
  Cx<R> gf[12], pf[12];
  F::load(gr, g.Vh, p ^ 1, j, gf);
  F::load(pr, g.Vh, p ^ 1, j, pf);
  Cx<R> a1[2][3], b1[2][3], a2[2][3], b2[2][3];
  project<MU, -1>(gn, a1);  // (1 - gamma) g(n)
  project<MU, -1>(pf, b1);  // (1 - gamma) psi(n+mu)
  project<MU, 1>(pn, a2);   // (1 + gamma) psi(n)
  project<MU, 1>(gf, b2);   // (1 + gamma) g(n+mu)
#pragma unroll
  for (int ra = 0; ra < 3; ++ra)
#pragma unroll
    for (int cb = 0; cb < 3; ++cb) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        // x (x) y^* : x_ra conj(y_cb)
        re += (double)a1[s][ra].re * b1[s][cb].re + (double)a1[s][ra].im * b1[s][cb].im;
        im += (double)a1[s][ra].im * b1[s][cb].re - (double)a1[s][ra].re * b1[s][cb].im;
        re += (double)a2[s][ra].re * b2[s][cb].re + (double)a2[s][ra].im * b2[s][cb].im;
        im += (double)a2[s][ra].im * b2[s][cb].re - (double)a2[s][ra].re * b2[s][cb].im;
      }
      out[(MU * 9 + ra * 3 + cb) * stride] = make_double2(re * scale, im * scale);
    }
}

// One thread per site over 64 consecutive lexicographic sites (both
// parities).  The output is the canonical [site][mu][3][3] complex128 array,
// 576 contiguous bytes per site: each thread stages its 36 entries in LDS
// (entry-major, so the writes are conflict-free) and the block then writes
// its contiguous 64 x 576 bytes with fully coalesced stores (adding the
// previous contents when accumulating).
constexpr int kForceBlock = 64;
template <int P>
__global__ void __launch_bounds__(kForceBlock) k_force(Geom g, int64_t V, const char* gin, const char* psi,
                                                       uint32_t fbytes, double2* F, double coeff, int acc) {
  __shared__ double2 stage[36 * kForceBlock];
  const int tid = threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.x * kForceBlock;
  const int64_t n = n0 + tid;
  if (n < V) {
    using R = typename SpinFmt<P>::R;
    Coord c;
    int64_t r = n;
    c.x = (int)(r % g.X);
    r /= g.X;
    c.y = (int)(r % g.Y);
    r /= g.Y;
    c.z = (int)(r % g.Z);
    c.t = (int)(r / g.Z);
    const int p = (c.x + c.y + c.z + c.t) & 1;
    const int i = (int)(n >> 1);
    const Rsrc gr = make_rsrc(gin, fbytes), pr = make_rsrc(psi, fbytes);
    Cx<R> gn[12], pn[12];
    SpinFmt<P>::load(gr, g.Vh, p, i, gn);
    SpinFmt<P>::load(pr, g.Vh, p, i, pn);
    const double scale = 0.5 * coeff;
    force_dir<0>(g, gr, pr, p, i, c, gn, pn, scale, stage + tid, kForceBlock);
    force_dir<1>(g, gr, pr, p, i, c, gn, pn, scale, stage + tid, kForceBlock);
    force_dir<2>(g, gr, pr, p, i, c, gn, pn, scale, stage + tid, kForceBlock);
    force_dir<3>(g, gr, pr, p, i, c, gn, pn, scale, stage + tid, kForceBlock);
  }
  __syncthreads();
  const int nvals = (int)min((int64_t)kForceBlock, V - n0) * 36;
  double2* out = F + n0 * 36;
#pragma unroll 4
  for (int k = 0; k < 36; ++k) {
    const int s = k * kForceBlock + tid;  // position in the block's output
    if (s < nvals) {
      double2 v = stage[(s % 36) * kForceBlock + s / 36];
      if (acc) {
        const double2 prev = out[s];
        v.x += prev.x;
        v.y += prev.y;
      }
      out[s] = v;
    }
  }
}

}  // namespace

// ---------------------------------------------------------- dispatch -----
#define PREC_SWITCH(prec, ...)                                               \
  switch (prec) {                                                            \
    case DIRAC_F64: { constexpr int P_ = DIRAC_F64; __VA_ARGS__; } break;     \
    case DIRAC_F32: { constexpr int P_ = DIRAC_F32; __VA_ARGS__; } break;     \
    case DIRAC_F16S: { constexpr int P_ = DIRAC_F16S; __VA_ARGS__; } break;   \
    case DIRAC_BF16S: { constexpr int P_ = DIRAC_BF16S; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                                    \
  }

hipError_t launch_finalize(const RedArgs& ra, int nparts, int nrhs, int nc, hipStream_t st) {
  if (nc == 1)
    hipLaunchKernelGGL(k_finalize<1>, dim3(nrhs), dim3(kFinBlock), 0, st, ra, nparts);
  else
    hipLaunchKernelGGL(k_finalize<2>, dim3(nrhs), dim3(kFinBlock), 0, st, ra, nparts);
  return hipGetLastError();
}

hipError_t pack_spinor(const Geom& g, int nrhs, const void* src, FieldRef dst, hipStream_t st) {
  SiteGrid sg = site_grid(g, nrhs);
  PREC_SWITCH(dst.prec, hipLaunchKernelGGL(k_pack_spinor<P_>, sg.grid, dim3(kBlock), 0, st, g, sg.nb,
                                           (const double2*)src, dev(dst)));
  return hipGetLastError();
}

hipError_t unpack_spinor(const Geom& g, int nrhs, FieldRef src, void* dst, hipStream_t st) {
  SiteGrid sg = site_grid(g, nrhs);
  PREC_SWITCH(src.prec, hipLaunchKernelGGL(k_unpack_spinor<P_>, sg.grid, dim3(kBlock), 0, st, g, sg.nb,
                                           dev(src), (double2*)dst));
  return hipGetLastError();
}

hipError_t pack_gauge(const Geom& g, int prec, int link, const void* U, void* out, hipStream_t st) {
  SiteGrid sg = site_grid(g, 1);
  const double2* u = (const double2*)U;
  char* o = (char*)out;
  if (prec == DIRAC_F64 && link == 18)
    hipLaunchKernelGGL((k_pack_gauge<DIRAC_F64, 18>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, u, o);
  else if (prec == DIRAC_F64 && link == 12)
    hipLaunchKernelGGL((k_pack_gauge<DIRAC_F64, 12>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, u, o);
  else if (prec == DIRAC_F32 && link == 18)
    hipLaunchKernelGGL((k_pack_gauge<DIRAC_F32, 18>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, u, o);
  else if (prec == DIRAC_F32 && link == 12)
    hipLaunchKernelGGL((k_pack_gauge<DIRAC_F32, 12>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, u, o);
  else if (prec == DIRAC_F16S && link == 12)
    hipLaunchKernelGGL((k_pack_gauge<DIRAC_F16S, 12>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, u, o);
  else if (prec == DIRAC_F32 && link == 10)
    hipLaunchKernelGGL((k_pack_gauge<DIRAC_F32, 10>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, u, o);
  else if (prec == DIRAC_F16S && link == 10)
    hipLaunchKernelGGL((k_pack_gauge<DIRAC_F16S, 10>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, u, o);
  else if (prec == DIRAC_BF16S && link == 12)
    hipLaunchKernelGGL((k_pack_gauge<DIRAC_BF16S, 12>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, u, o);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int PS>
static hipError_t convert_from(const Geom& g, int nrhs, FieldRef src, FieldRef dst, const CgState* cs,
                               int ci, const RedTarget* red, hipStream_t st) {
  SiteGrid sg = site_grid(g, nrhs);
  RedArgs ra = red ? red_args(*red) : RedArgs{nullptr, nullptr, 0};
  if (red) {
    PREC_SWITCH(dst.prec, hipLaunchKernelGGL((k_convert<PS, P_, true>), sg.grid, dim3(kBlock), 0, st, g,
                                             sg.nb, nrhs, dev(src), dev(dst), cs, ci, ra));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(ra, sg.nparts, nrhs, 1, st);
  } else {
    PREC_SWITCH(dst.prec, hipLaunchKernelGGL((k_convert<PS, P_, false>), sg.grid, dim3(kBlock), 0, st, g,
                                             sg.nb, nrhs, dev(src), dev(dst), cs, ci, ra));
  }
  return hipGetLastError();
}

hipError_t convert_scale(const Geom& g, int nrhs, FieldRef src, FieldRef dst, const CgState* cs, int ci,
                         const RedTarget* red, hipStream_t st) {
  switch (src.prec) {
    case DIRAC_F64: return convert_from<DIRAC_F64>(g, nrhs, src, dst, cs, ci, red, st);
    case DIRAC_F32: return convert_from<DIRAC_F32>(g, nrhs, src, dst, cs, ci, red, st);
    case DIRAC_F16S: return convert_from<DIRAC_F16S>(g, nrhs, src, dst, cs, ci, red, st);
    case DIRAC_BF16S: return convert_from<DIRAC_BF16S>(g, nrhs, src, dst, cs, ci, red, st);
  }
  return hipErrorInvalidValue;
}

template <int PA>
static hipError_t dot_from(const Geom& g, int nrhs, FieldRef a, FieldRef b, const RedTarget& red,
                           hipStream_t st) {
  SiteGrid sg = site_grid(g, nrhs);
  PREC_SWITCH(b.prec, hipLaunchKernelGGL((k_dot<PA, P_>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, nrhs,
                                         dev(a), dev(b), red_args(red)));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(red_args(red), sg.nparts, nrhs, 2, st);
}

hipError_t dot(const Geom& g, int nrhs, FieldRef a, FieldRef b, const RedTarget& red, hipStream_t st) {
  switch (a.prec) {
    case DIRAC_F64: return dot_from<DIRAC_F64>(g, nrhs, a, b, red, st);
    case DIRAC_F32: return dot_from<DIRAC_F32>(g, nrhs, a, b, red, st);
    case DIRAC_F16S: return dot_from<DIRAC_F16S>(g, nrhs, a, b, red, st);
    case DIRAC_BF16S: return dot_from<DIRAC_BF16S>(g, nrhs, a, b, red, st);
  }
  return hipErrorInvalidValue;
}

hipError_t norm2(const Geom& g, int nrhs, FieldRef a, const RedTarget& red, hipStream_t st) {
  SiteGrid sg = site_grid(g, nrhs);
  PREC_SWITCH(a.prec, hipLaunchKernelGGL((k_norm2<P_>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, nrhs,
                                         dev(a), red_args(red)));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(red_args(red), sg.nparts, nrhs, 1, st);
}

template <int PX>
static hipError_t axpby_from(const Geom& g, int nrhs, FieldRef x, FieldRef y, const CgState* s, double ar,
                             double ai, double br, double bi, hipStream_t st) {
  SiteGrid sg = site_grid(g, nrhs);
  PREC_SWITCH(y.prec, hipLaunchKernelGGL((k_axpby<PX, P_>), sg.grid, dim3(kBlock), 0, st, g, sg.nb,
                                         dev(x), dev(y), s, ar, ai, br, bi));
  return hipGetLastError();
}

hipError_t axpby(const Geom& g, int nrhs, FieldRef x, FieldRef y, const CgState* s, double ar, double ai,
                 double br, double bi, hipStream_t st) {
  if (x.prec == y.prec && (x.prec == DIRAC_F64 || x.prec == DIRAC_F32)) {
    const uint32_t plane = (uint32_t)g.Vh * (x.prec == DIRAC_F64 ? 192u : 96u);
    const uint32_t off0 = g.vpar > 0 ? plane : 0u;
    const uint32_t n16 = (g.vpar >= 0 ? plane : 2u * plane) / 16u;
    const dim3 grid((n16 + kBlock - 1) / kBlock, nrhs);
    if (x.prec == DIRAC_F64)
      hipLaunchKernelGGL(k_axpby_flat<DIRAC_F64>, grid, dim3(kBlock), 0, st, dev(x), dev(y), s, ar, ai, br, bi,
                         off0, n16);
    else
      hipLaunchKernelGGL(k_axpby_flat<DIRAC_F32>, grid, dim3(kBlock), 0, st, dev(x), dev(y), s, ar, ai, br, bi,
                         off0, n16);
    return hipGetLastError();
  }
  switch (x.prec) {
    case DIRAC_F64: return axpby_from<DIRAC_F64>(g, nrhs, x, y, s, ar, ai, br, bi, st);
    case DIRAC_F32: return axpby_from<DIRAC_F32>(g, nrhs, x, y, s, ar, ai, br, bi, st);
    case DIRAC_F16S: return axpby_from<DIRAC_F16S>(g, nrhs, x, y, s, ar, ai, br, bi, st);
    case DIRAC_BF16S: return axpby_from<DIRAC_BF16S>(g, nrhs, x, y, s, ar, ai, br, bi, st);
  }
  return hipErrorInvalidValue;
}

hipError_t cg_xp_update(const Geom& g, int nrhs, FieldRef x, FieldRef p, FieldRef r, const CgState* state,
                        hipStream_t st) {
  if (x.prec == p.prec && p.prec == r.prec && (x.prec == DIRAC_F64 || x.prec == DIRAC_F32)) {
    // one parity plane of Vh sites, or both
    const uint32_t plane = (uint32_t)g.Vh * (x.prec == DIRAC_F64 ? 192u : 96u);
    const uint32_t off0 = g.vpar > 0 ? plane : 0u;
    const uint32_t n16 = (g.vpar >= 0 ? plane : 2u * plane) / 16u;
    const dim3 grid((n16 + kBlock - 1) / kBlock, nrhs);
    // non-temporal when the five vectors of a CG iteration exceed the 256 MiB last-level cache
    const bool nt = 5.0 * (double)n16 * 16.0 * nrhs > 256.0 * (1 << 20);
    if (x.prec == DIRAC_F64) {
      if (nt)
        hipLaunchKernelGGL((k_cg_xp_flat<DIRAC_F64, 2>), grid, dim3(kBlock), 0, st, dev(x), dev(p), dev(r), state,
                           off0, n16);
      else
        hipLaunchKernelGGL((k_cg_xp_flat<DIRAC_F64, 0>), grid, dim3(kBlock), 0, st, dev(x), dev(p), dev(r), state,
                           off0, n16);
    } else {
      if (nt)
        hipLaunchKernelGGL((k_cg_xp_flat<DIRAC_F32, 2>), grid, dim3(kBlock), 0, st, dev(x), dev(p), dev(r), state,
                           off0, n16);
      else
        hipLaunchKernelGGL((k_cg_xp_flat<DIRAC_F32, 0>), grid, dim3(kBlock), 0, st, dev(x), dev(p), dev(r), state,
                           off0, n16);
    }
    return hipGetLastError();
  }
  SiteGrid sg = site_grid(g, nrhs);
#define XP(PX, PP, PR)                                                                              \
  if (x.prec == PX && p.prec == PP && r.prec == PR) {                                              \
    hipLaunchKernelGGL((k_cg_xp<PX, PP, PR>), sg.grid, dim3(kBlock), 0, st, g, sg.nb, dev(x), dev(p), \
                       dev(r), state);                                                             \
    return hipGetLastError();                                                                      \
  }
  XP(DIRAC_F32, DIRAC_F16S, DIRAC_F32)
  XP(DIRAC_F32, DIRAC_BF16S, DIRAC_F32)
#undef XP
  return hipErrorInvalidValue;
}

hipError_t zero(const Geom& g, int nrhs, FieldRef f, hipStream_t st) {
  SiteGrid sg = site_grid(g, nrhs);
  PREC_SWITCH(f.prec, hipLaunchKernelGGL(k_zero<P_>, sg.grid, dim3(kBlock), 0, st, g, sg.nb, dev(f)));
  return hipGetLastError();
}

hipError_t force(const Geom& g, int prec, const void* gin, const void* psi, uint32_t fbytes, void* F,
                 double coeff, int accumulate, hipStream_t st) {
  const int64_t V = 2 * (int64_t)g.Vh;
  const dim3 grid((unsigned)((V + kForceBlock - 1) / kForceBlock));
  if (prec == DIRAC_F64)
    hipLaunchKernelGGL(k_force<DIRAC_F64>, grid, dim3(kForceBlock), 0, st, g, V, (const char*)gin,
                       (const char*)psi, fbytes, (double2*)F, coeff, accumulate);
  else if (prec == DIRAC_F32)
    hipLaunchKernelGGL(k_force<DIRAC_F32>, grid, dim3(kForceBlock), 0, st, g, V, (const char*)gin,
                       (const char*)psi, fbytes, (double2*)F, coeff, accumulate);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dirac
