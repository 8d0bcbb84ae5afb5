/*
 * dirac.h -- C ABI of libdirac: the Wilson-Dirac operator of eq. (1) and the
 * conjugate-gradient solve on D^dagger D (Algorithm 1), on hand-written HIP
 * kernels for AMD gfx950 (MI355X).
 *
 * The operator (eq. (1), Introduction):
 *
 *   (D psi)(n) = (m_q + 4) psi(n)
 *              + 1/2 sum_mu [ U_mu(n) P^{-mu} psi(n+mu) + U_mu(n-mu)^dag P^{+mu} psi(n-mu) ]
 *
 * with P^{-+mu} = 1 -+ gamma_mu (chiral gamma basis, mu = 0..3 <-> x,y,z,t),
 * periodic boundaries, hopping sign as printed.
 *
 * General rules for every entry point:
 *   - Pointers are DEVICE pointers owned by the caller unless marked "host".
 *     The library keeps no reference to them after the call returns (except
 *     a graph plan, see dirac_multi_plan_create), and it never allocates
 *     device memory: scratch comes from caller workspaces sized by the
 *     *_workspace_bytes calls.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued asynchronously on it; only cg_solve, dirac_field_dot,
 *     dirac_autotune and the plan/graph calls synchronise the stream.
 *   - Return value: DIRAC_OK (0) or a negative status.  Arguments are
 *     validated on the host before anything is launched; on error nothing is
 *     launched and dirac_last_error() describes the problem.  Nothing aborts
 *     or throws across the ABI.
 *   - Device buffers must be 256-byte aligned (every hipMalloc / torch CUDA
 *     allocation is); inputs and outputs of one call must not overlap.
 *
 * Canonical (user) layouts, complex128 = two float64 (re, im):
 *   gauge links U : [Lt][Lz][Ly][Lx][4 (mu)][3][3]  (row-major colour matrix)
 *   spinor psi    : [nrhs][Lt][Lz][Ly][Lx][4 (spin)][3 (colour)]
 *   link force F  : same shape as U.
 * Internal layouts are opaque; their sizes come from dirac_*_bytes.  They
 * are structure-of-arrays over checkerboard (even-odd) sites, 16-byte
 * vectors per site component, so neighbouring threads touch neighbouring
 * addresses.
 */
#ifndef DIRAC_H
#define DIRAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage/arithmetic precision of internal fields.
 *   F64   : float64 spinors and links, float64 arithmetic.
 *   F32   : float32 spinors and links, float32 arithmetic.
 *   F16S  : float16 spinor payload with one float32 scale per site
 *           (max |real component| of the site), float16 links (unscaled,
 *           |U_ij| <= 1), float32 arithmetic.
 *   BF16S : as F16S with bfloat16 payloads.
 * Every global reduction accumulates in float64 in all precisions. */
enum { DIRAC_F64 = 0, DIRAC_F32 = 1, DIRAC_F16S = 2, DIRAC_BF16S = 3 };

/* Link storage: the full 3x3 complex matrix (18 reals); its first two rows
 * (12 reals) with row 2 = conj(row0 x row1) rebuilt in registers; or the
 * 10-real form: row 0 and, for the pivot column k (the row-0 entry of
 * smallest modulus, lowest index on ties), U_1k and U_2k, the other four
 * entries rebuilt from the cofactor identity conj(U_ij) = cofactor_ij of a
 * special unitary matrix (a division by 1 - |U_0k|^2 >= 2/3, no
 * trigonometric function).  All are exact for SU(3) up to rounding; the
 * paper streams 10-parameter links and trades link words for arithmetic in
 * the same way (section "Larger Lattice Streamed from the DDR Memory").
 * F16S/BF16S need LINK12, or LINK10 (F16S); LINK10 is built for F32 and
 * F16S and for the Dslash calls (dirac_apply, dirac_dagger_apply,
 * dirac_mdagm_apply, dirac_autotune); the solver, even-odd and
 * multi-lattice calls return DIRAC_EUNSUPPORTED for it. */
enum { DIRAC_LINK18 = 18, DIRAC_LINK12 = 12, DIRAC_LINK10 = 10 };

enum {
  DIRAC_OK = 0,
  DIRAC_EINVAL = -1,       /* bad argument (message in dirac_last_error) */
  DIRAC_EDEVICE = -2,      /* a HIP call failed */
  DIRAC_ENOCONV = -3,      /* solver hit max_iter; x holds the last iterate */
  DIRAC_EBREAKDOWN = -4,   /* NaN/Inf or <p, A p> <= 0 in the solver */
  DIRAC_EUNSUPPORTED = -5, /* valid but not implemented combination */
  DIRAC_EWORKSPACE = -6    /* workspace too small */
};

/* One operator instance: lattice geometry, precision, link storage, number
 * of right-hand sides and quark mass m_q of eq. (1). */
typedef struct dirac_op {
  int32_t L[4];   /* Lx, Ly, Lz, Lt: each even and >= 2, V = product < 2^31 */
  int32_t prec;   /* DIRAC_F64 / F32 / F16S / BF16S */
  int32_t link;   /* DIRAC_LINK18 / DIRAC_LINK12 / DIRAC_LINK10 */
  int32_t nrhs;   /* 1..12 right-hand sides stored one after another */
  int32_t flags;  /* 0 */
  double m_q;     /* quark mass, finite */
} dirac_op;

/* Bytes of one internal spinor buffer holding all nrhs fields, or of one
 * internal gauge buffer.  Negative status on an invalid op. */
int64_t dirac_spinor_bytes(const dirac_op* op);
int64_t dirac_gauge_bytes(const dirac_op* op);

/* Canonical complex128 -> internal (links: round to op->prec and drop row 2
 * for LINK12; spinors: round, and for F16S/BF16S compute the per-site
 * scale) and back.  Unpack of a low-precision field returns its exactly
 * representable complex128 value. */
int dirac_pack_gauge(const dirac_op* op, const void* U_c128, void* U_int, void* stream);
int dirac_pack_spinor(const dirac_op* op, const void* psi_c128, void* psi_int, void* stream);
int dirac_unpack_spinor(const dirac_op* op, const void* psi_int, void* psi_c128, void* stream);

/* Convert an internal spinor buffer between precisions (same geometry and
 * nrhs).  Rounds to nearest even; F16S/BF16S targets recompute the scale. */
int dirac_convert_spinor(const dirac_op* op_src, const void* src,
                         const dirac_op* op_dst, void* dst, void* stream);

/* chi = D psi (eq. (1)), all nrhs fields, each link load shared by the
 * right-hand sides a thread handles.  U_int, psi_int in op's internal
 * layout; chi_int receives the result in the same precision. */
int dirac_apply(const dirac_op* op, const void* U_int, const void* psi_int, void* chi_int,
                void* stream);

/* chi = D^dagger psi = gamma5 D gamma5 psi: eq. (1) with P^{-mu} and P^{+mu}
 * exchanged (the operator applied at Algorithm 1's D^dagger D products). */
int dirac_dagger_apply(const dirac_op* op, const void* U_int, const void* psi_int,
                       void* chi_int, void* stream);

/* chi = D^dagger D psi through tmp (one more internal spinor buffer). */
int dirac_mdagm_apply(const dirac_op* op, const void* U_int, const void* psi_int, void* tmp_int,
                      void* chi_int, void* stream);

/* Bytes of device workspace dirac_field_dot needs for op (reduction
 * partials and per-right-hand-side scalars); negative status on a bad op. */
int64_t dirac_field_dot_workspace_bytes(const dirac_op* op);

/* <a, b> = sum conj(a) b over all sites, per right-hand side, accumulated in
 * float64 with a fixed-order (deterministic) reduction: the inner products of
 * Algorithm 1 (Kernel Description).  a_int, b_int: internal fields of op.
 * work: caller-owned device workspace of work_bytes >=
 * dirac_field_dot_workspace_bytes(op), 256-byte aligned, not overlapping the
 * fields (DIRAC_EWORKSPACE if too small); its contents on entry do not
 * matter.  out_host (host) receives nrhs complex values as (re, im) pairs.
 * Synchronises the stream.  Calls that share one workspace must not overlap
 * in time. */
int dirac_field_dot(const dirac_op* op, const void* a_int, const void* b_int, void* work, int64_t work_bytes,
                    double* out_host, void* stream);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid allocation, callers without a workspace to hand):
 * dirac_field_dot with its workspace in a fixed device array inside the
 * library, 4 MiB per GPU, held from the first call on that GPU until the
 * process ends.  Same kernels and result as dirac_field_dot; ops whose
 * workspace (dirac_field_dot_workspace_bytes) exceeds the array, about
 * 67 million sites x right-hand sides, are rejected with DIRAC_EINVAL.  The
 * array is shared by every call on one GPU and keeps the last call's
 * contents (each call overwrites what it reads); calls of one process are
 * serialised by a lock held until the call's stream has synchronised, so
 * they never overlap.  Allocates nothing and synchronises the stream. */
int dirac_field_dot_noalloc(const dirac_op* op, const void* a_int, const void* b_int, double* out_host,
                            void* stream);

/* y = a x + y on internal fields of one precision, complex scalar a given by
 * (a_re, a_im), same for every right-hand side. */
int dirac_field_axpy(const dirac_op* op, double a_re, double a_im, const void* x_int, void* y_int,
                     void* stream);

/* ---------------------------------------------------------------- CG ---- */

/* Solver parameters (Algorithm 1).
 *   tol         : stop when ||eta - D^dag D x|| / ||eta|| < tol, with the
 *                 residual recomputed in float64 (never the recursive one).
 *   max_iter    : cap on the total number of (inner) CG iterations.
 *   inner_prec  : DIRAC_F64 -> plain float64 CG (inner loop of Algorithm 1
 *                 run entirely in high precision);
 *                 DIRAC_F32 / F16S / BF16S -> Algorithm 1: float64 outer
 *                 loop (true residual, normalisation, solution update),
 *                 inner CG with that storage and float32 arithmetic.
 *   inner_delta : inner stop when ||r_inner|| < inner_delta (the inner
 *                 residual starts at norm 1); <= 0 picks 1e-3 (F32) or
 *                 0.1 (F16S/BF16S).
 *   inner_kmax  : cap on one inner solve (<= 0: 10000).  Every cycle after
 *                 the first is further capped at twice the first cycle's
 *                 iteration count (at least 50).  A cycle that does not
 *                 lower the best true residual so far counts as stalled;
 *                 from the third stalled cycle on no search direction is
 *                 carried into the next cycle, and two capped cycles in a
 *                 row, or six stalled cycles, finish the solve with float64
 *                 CG from the current iterate (stats.fallback).
 *   check_every : iterations launched between host convergence checks
 *                 (<= 0: automatic).
 *   single_launch : run the CG iterations in a single launch, one workgroup
 *                 per right-hand side with the scalars in registers and no
 *                 host polling (cg_solve only; small lattices, where the
 *                 five dependent launches of an iteration are all latency):
 *                 0 automatic (lattices of at most 1024 sites), 1 always,
 *                 -1 never.  Same recurrence and stopping rules; results
 *                 agree with the multi-kernel iteration up to rounding order.
 *                 A launch runs a bounded number of iterations, and the host
 *                 launches again until every right-hand side is done.
 *   reserved    : must be 0.
 */
typedef struct cg_params {
  double tol;
  int32_t max_iter;
  int32_t inner_prec;
  double inner_delta;
  int32_t inner_kmax;
  int32_t check_every;
  int32_t single_launch;
  int32_t reserved;
} cg_params;

/* Per right-hand-side results (host). */
typedef struct cg_stats {
  int32_t status;      /* DIRAC_OK, DIRAC_ENOCONV or DIRAC_EBREAKDOWN */
  int32_t iters;       /* CG iterations (inner iterations for Algorithm 1) */
  int32_t outer;       /* outer cycles (true-residual recomputations) */
  int32_t dslash_hi;   /* high-precision D or D^dag applications */
  int32_t dslash_lo;   /* low-precision D or D^dag applications */
  int32_t fallback;    /* 0, or the number of Algorithm 1 cycles after which
                          the safeguards handed the solve to float64 CG */
  double true_rel_res; /* final ||eta - A x|| / ||eta||, float64 */
  double seconds;      /* wall time of the whole solve */
} cg_stats;

/* Bytes of scratch the solve needs for op_hi (which must be DIRAC_F64) and
 * params.  The caller allocates it (any device allocation). */
int64_t cg_workspace_bytes(const dirac_op* op_hi, const cg_params* params);

/* Solve D^dagger D x = eta for each of op_hi->nrhs right-hand sides.
 *   op_hi : DIRAC_F64 operator (LINK18 or LINK12).
 *   U_hi  : links packed for op_hi.
 *   U_lo  : links packed for the inner precision (op_hi with prec =
 *           params->inner_prec and link = DIRAC_LINK12, or op_hi's link for
 *           F32); NULL when inner_prec == DIRAC_F64.
 *   eta   : F64 internal source(s); x: F64 internal initial guess on entry
 *           (a restart / resume point; zero it for x0 = 0), solution on exit.
 *   stats : host array of nrhs entries.
 * Returns DIRAC_OK when every right-hand side converged, else the first
 * non-OK per-RHS status (x still holds each RHS's last iterate).
 * Synchronises the stream. */
int cg_solve(const dirac_op* op_hi, const void* U_hi, const void* U_lo, const void* eta, void* x,
             void* work, int64_t work_bytes, const cg_params* params, cg_stats* stats,
             void* stream);

/* ----------------------------------------------------- even-odd form ---- */

/* Not a method of the paper: the even-odd (Schur complement) form of D.
 * Every hop of eq. (1) joins sites of opposite parity ((x+y+z+t) mod 2) and
 * the mass term stays on its site, so in (even, odd) blocks
 *   D = [[A, K_eo], [K_oe, A]],   A = m_q + 4,
 * with K the hopping sum of eq. (1) (its factor 1/2 included), and the
 * even-site Schur complement is
 *   D_hat = A - K_eo K_oe / A.
 * D^dagger has the same form with the adjoint hop (the projector swap of
 * dirac_dagger_apply), and its Schur complement is D_hat^dagger.
 *
 * Even vectors live in the even-parity plane of an ordinary internal field of
 * op (the layout of dirac_pack_spinor); the odd plane is ignored or used as
 * scratch as stated.
 *
 * The hops run one thread per output site, or, when op's launch
 * configuration is the t-streaming one (float64 and float32), in a
 * t-streaming form with the input half-slice in LDS: its tile is op's,
 * doubled in z (else y) until its (X / 2) * tile_y * tile_z column pairs
 * fill 3/4 of a block of 128 or 256 threads (float32 also 512), at least 32
 * pairs, walking at most 8 slices, in XCD-contiguous order, with the face
 * spinors of the next slice requested a step ahead when the tile is at least
 * 2 deep in y and z.  Both forms compute the same sums (to rounding). */

/* out_e = D_hat in_e (dagger = 0) or D_hat^dagger in_e (dagger = 1), for
 * each of op->nrhs fields, in op's format (the 16-bit formats round the
 * odd intermediate and the result to their storage, as dirac_apply rounds
 * its output).  Only the even plane of `in` is read.  The even plane of `out`
 * receives the result; its odd plane is overwritten with the intermediate
 * K_oe in_e.  in and out must not overlap (DIRAC_EINVAL).  Asynchronous. */
int dirac_schur_apply(const dirac_op* op, const void* U_int, const void* in_int, void* out_int, int32_t dagger,
                      void* stream);

/* Bytes of scratch cg_solve_eo needs. */
int64_t cg_workspace_bytes_eo(const dirac_op* op_hi, const cg_params* params);

/* Solve D x = b (eq. (1)), or D^dagger x = b when dagger != 0, for each of
 * op_hi->nrhs sources through the Schur complement (written for D; for
 * D^dagger every K below is the adjoint hop and the CG runs on
 * D_hat D_hat^dagger):
 *   b_hat = b_e - K_eo b_o / A,
 *   D_hat^dagger D_hat x_e = D_hat^dagger b_hat   (cg_solve's CG: plain
 *       float64 for inner_prec = DIRAC_F64, Algorithm 1 with an inner solve
 *       in F32, F16S or BF16S otherwise; U_lo as for cg_solve),
 *   x_o = (b_o - K_oe x_e) / A.
 * A source has converged when ||b - D x|| / ||b|| < params->tol, recomputed
 * in float64 on the full lattice after the reconstruction; until then the
 * CG tolerance on the normal equations (first 0.25 tol) is tightened and the
 * solve resumed from the current x (at most 6 passes, max_iter CG
 * iterations in all).
 * inner_delta <= 0 picks 1e-3 (F32), 0.02 (F16S) or 0.1 (BF16S): the Schur
 * system lets an F16S inner solve reach a smaller residual than D^dagger D.
 * Arguments as for cg_solve, with b in place of eta; x: the even plane holds
 * the initial guess on entry, x the full solution on exit.  stats: iters
 * and outer summed over the passes, dslash_hi / dslash_lo count applications
 * of D_hat or D_hat^dagger, true_rel_res = ||b - D x|| / ||b|| (D^dagger in
 * place of D for the adjoint solve).
 * Synchronises the stream.  (D^dagger D x = eta itself is cg_solve's.) */
int cg_solve_eo(const dirac_op* op_hi, const void* U_hi, const void* U_lo, const void* b, void* x, void* work,
                int64_t work_bytes, const cg_params* params, int32_t dagger, cg_stats* stats, void* stream);

/* --------------------------------------------------------- measurement ---- */

/* Memory-bandwidth reference kernels for measurements (not used by any
 * solve): kind 0 copies `bytes` from src to dst, kind 1 reads src (dst is a
 * 16-byte sink that is never written in practice), kind 2 writes dst (src is
 * ignored).  16-byte vectors with non-temporal accesses, four 256-thread
 * blocks per CU.  bytes: a positive multiple of 16; device buffers, 16-byte
 * aligned, not overlapping for a copy (DIRAC_EINVAL otherwise).
 * Asynchronous. */
int dirac_bandwidth_probe(int32_t kind, const void* src, void* dst, int64_t bytes, void* stream);

/* ------------------------------------------------------------ gradient ---- */

/* Link gradient of a real loss L through chi = D(U) psi (the backward of
 * eq. (1) with respect to U), given g = dL/dRe chi + i dL/dIm chi:
 *
 *   F_mu(n) = coeff/2 [ sum_alpha g(n)_alpha (P^{-mu} psi(n+mu))_alpha^dag
 *                     + sum_alpha (P^{+mu} psi(n))_alpha g(n+mu)_alpha^dag ],
 *
 * evaluated with half spinors (two colour outer products per term).
 * g_int, psi_int: internal spinors of op (F64 or F32, nrhs = 1).
 * F_c128: canonical complex128 [Lt][Lz][Ly][Lx][4][3][3]; written, or added
 * to when accumulate != 0.  One gather per link, no atomics. */
int dirac_force(const dirac_op* op, const void* g_int, const void* psi_int, void* F_c128,
                double coeff, int32_t accumulate, void* stream);

/* --------------------------------------------- batching and autotuning ---- */

/* Apply D (dagger = 0) or D^dagger (dagger = 1) on up to 8 independent
 * lattices (own geometry, links and m_q; one shared precision and link
 * storage; nrhs = 1) in ONE kernel launch that walks a work list of
 * (lattice, tile) pairs.  ops, U, psi, chi are host arrays of n entries.
 * The launch form is either t-streaming tiles (each lattice its largest tile
 * of at most 256 columns, one t_chunk for all) or per-site blocks: the form
 * timed fastest by dirac_multi_plan_create for the same set of lattices,
 * else streaming with t_chunk 4 when every lattice has a tile. */
int dirac_multi_apply(int32_t n, const dirac_op* ops, const void* const* U,
                      const void* const* psi, void* const* chi, int32_t dagger, void* stream);

/* Time the launch forms of dirac_multi_apply on these buffers and stream
 * (chi is overwritten; the stream is synchronised), keep the fastest for
 * this set of lattices, capture it into a hipGraph once and return an opaque
 * plan (host) that replays it with dirac_plan_launch.  The plan keeps the
 * pointers: the buffers must outlive it. */
int dirac_multi_plan_create(int32_t n, const dirac_op* ops, const void* const* U,
                            const void* const* psi, void* const* chi, int32_t dagger,
                            void* stream, void** plan_out);
int dirac_plan_launch(void* plan, void* stream);
int dirac_plan_destroy(void* plan);

/* Launch configuration of the Dslash kernels for one op.  Three kernel
 * families compute the same per-site arithmetic (eq. (1)):
 *   - one thread per site (lds = 0, rhs_per_thread 1..4): block_sites
 *     threads per block, each thread doing rhs_per_thread right-hand sides
 *     with one load of each link;
 *   - direction split (lds = 0, rhs_per_thread -2 or -4): 2 or 4 waves share
 *     each block of 64 sites, one direction pair per wave, partial spinors
 *     combined in LDS (nrhs = 1; for lattices too small to fill the device);
 *   - t-streaming (lds = 1): a block owns all of x times tile_y rows times
 *     tile_z planes (32 to 512 columns, float64 up to 256, in a block of
 *     128, 192, 256, 384 or 512 threads, float64 128 or 256) and walks
 *     t_chunk time slices; the current
 *     slice is staged in LDS and the t neighbours stay in registers
 *     (tile_y | Ly and tile_z | Lz; one block per tile and right-hand side,
 *     the blocks of a tile adjacent so that they share its links in the L2).
 * xcd_remap orders tiles so that each XCD sweeps one contiguous region
 * (0 or 1).  For the t-streaming kernel it is a mask: bit 0 that XCD order,
 * bit 1 t-chunks fastest in the block order, bit 2 odd t-chunks walk down in
 * t, so that neighbouring chunks read their shared halo slice at the same
 * time; bit 3 (float64 only) requests each direction's links and spinors one
 * direction ahead of its hops, so that two directions' loads are in flight;
 * bit 4 (float64 only; tile_y and tile_z at least 2, else DIRAC_EINVAL)
 * loads the spinors beyond the tile's y and z faces one time slice ahead,
 * in the step in which the neighbouring tile reads them, so that the L2
 * serves the second read.
 * nt_store writes the output with non-temporal stores. */
typedef struct dirac_launch {
  int32_t block_sites;
  int32_t rhs_per_thread;
  int32_t xcd_remap;
  int32_t nt_store;
  int32_t lds;
  int32_t tile_y, tile_z, t_chunk;
  int32_t tuned; /* out only: 1 when chosen by the autotuner or set explicitly */
} dirac_launch;

/* Time every launch candidate above that fits this op on the given buffers
 * with HIP events (each on two launches, then the 16 fastest again on
 * enough launches for about 2 ms) and remember the fastest for every later
 * call with the same (device, geometry, precision, links, nrhs).  chi_int
 * is overwritten.  Synchronises the stream.  If the environment variable
 * DIRAC_TUNE_CACHE names a file, results are appended there and read back
 * by later processes.  With DIRAC_TUNE_VERBOSE set (not "0") the final
 * timings are printed to stderr. */
int dirac_autotune(const dirac_op* op, const void* U_int, const void* psi_int, void* chi_int,
                   void* stream);

/* The launch configuration the next call with this op will use (host out). */
int dirac_launch_config(const dirac_op* op, dirac_launch* out);

/* Force the launch configuration for this op (tests, expert tuning).
 * EINVAL when it does not fit the op (see dirac_launch). */
int dirac_set_launch_config(const dirac_op* op, const dirac_launch* cfg);

/* Description of the last error on the calling host thread ("" if none). */
const char* dirac_last_error(void);

/* Library version string, e.g. "dirac 0.1 gfx950". */
const char* dirac_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DIRAC_H */
