/*
 * qdwf -- domain-wall fermion Dirac operator and Krylov solver for MI355X (gfx950).
 *
 * C ABI of libqdwf.so. Plain pointers and sizes only; every device buffer is
 * owned by the caller unless stated otherwise. All calls return a status code
 * (QDWF_OK = 0); on failure qdwf_last_error() gives a thread-local message.
 * Argument checks happen before any device work, so a call that returns
 * QDWF_EINVAL has launched nothing. No exception or abort crosses the ABI.
 *
 * What is computed (the paper, arXiv 2112.01852, Sections 4.1-4.3, measures
 * the Domain Wall kernel -- the 4D Wilson hopping term with SU(3) link
 * multiplies applied on every slice of the fifth dimension -- and counts 1320
 * real flops per 5D site for it in Table 3; the operator itself is not written
 * out in the paper, so the standard conventions below are the definitions
 * used):
 *
 *   lattice     L = (Lx, Ly, Lz, Lt), all even; lex = ((t*Lz+z)*Ly+y)*Lx+x;
 *               parity = (x+y+z+t) mod 2.
 *   gamma       DeGrand-Rossi chiral basis, gamma5 = diag(1,1,-1,-1);
 *               P+ keeps spins 0,1 and P- keeps spins 2,3.
 *   hop         (D_h psi)(x,s) = sum_mu [ (1-g_mu) U_mu(x) psi(x+mu,s)
 *                                       + (1+g_mu) U_mu(x-mu)^dag psi(x-mu,s) ],
 *               each hop across the mu boundary multiplied by bc[mu].
 *   Wilson      D_W = (4 - M5) - D_h / 2 inside D; the standalone Wilson
 *               operator of qdwf_apply_Dw is (4 + m) - D_h / 2 for a mass m.
 *   5th dim     (S_u psi)_s = psi_{s+1}, row Ls-1 takes -mf psi_0;
 *               (S_d psi)_s = psi_{s-1}, row 0 takes -mf psi_{Ls-1};
 *               C = P- S_u + P+ S_d; A = b + c C; B = 1 - C.
 *   operator    D = D_W A + B (Shamir: b = 1, c = 0); D^dag = A^dag D_W^dag + B^dag.
 *   even-odd    M_ee = M_oo = alpha + beta C, alpha = b(4-M5)+1, beta = c(4-M5)-1;
 *               M_pq = -1/2 D_h^{pq} A (p != q);
 *               M_pc = M_oo - M_oe M_ee^-1 M_eo on odd sites.
 *   flops       1320 per 5D output site per hop application (Table 3),
 *               times the number of right-hand sides; 5D-local work is not counted.
 *
 * Canonical (caller-facing) layouts, row-major, interleaved complex:
 *   gauge   U[mu][t][z][y][x][a][b]                 (mu = x, y, z, t)
 *   spinor  psi[rhs][s][t][z][y][x][spin][colour]
 * Internal spinor fields (what the operators take) are produced by
 * qdwf_pack_spinor. A half field holds one parity: (V/2)*Ls 5D sites (i, s),
 * 24 reals per site, where i numbers the 4D sites of that parity in the
 * library's traversal order (8 slabs along z, one per XCD, (x,y,z) tiles
 * swept along t; qdwf_geometry_tables exports it). A full field is the even
 * half followed by the odd half. nrhs fields of the same kind are stored
 * back to back. Two layouts of the 24 reals c = (spin*3 + colour)*2 + re/im
 * exist (Section 4.3 compares the same two choices for SVE registers):
 *   QDWF_RIRI  interleaved complex, blocked over the slices of a 4D site in
 *              chunks of 4 reals: offset i*Ls*24 + (c/4)*Ls*4 + s*4 + c%4;
 *              for Ls = 1 over 16 consecutive sites (i/16 and i%16 in place
 *              of i and s), which needs V/2 to be a multiple of 16
 *   QDWF_RRII  split planes: offset ((c%2)*12 + c/2)*(V/2)*Ls + i*Ls + s
 * Precisions give the storage type of a real; arithmetic is FP64 for QDWF_F64
 * and FP32 for the others (FP16/BF16 are storage only, rounded to nearest even).
 */
#ifndef QDWF_H
#define QDWF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------- */
#define QDWF_OK        0
#define QDWF_EINVAL    1   /* bad argument; nothing was launched */
#define QDWF_ENOMEM    2   /* a library-owned allocation failed (create / set_gauge only) */
#define QDWF_EDEVICE   3   /* a HIP call failed; message carries hipGetErrorString */
#define QDWF_ENOTCONV  4   /* solver hit max_iter before reaching tol (stats are filled) */
#define QDWF_ENAN      5   /* solver met a NaN or Inf */
#define QDWF_EBUSY     6   /* pool request not finished yet */

/* ---- enums ------------------------------------------------------------ */
#define QDWF_F64   0
#define QDWF_F32   1
#define QDWF_F16   2
#define QDWF_BF16  3

#define QDWF_RRII  0
#define QDWF_RIRI  1

#define QDWF_EVEN  0
#define QDWF_ODD   1
#define QDWF_FULL  2

/* 5D-local operator selectors for qdwf_apply_Mee */
#define QDWF_MEE_FWD   0   /* M_ee                 */
#define QDWF_MEE_INV   1   /* M_ee^-1              */

/* solver systems */
#define QDWF_SYS_NORMAL_PC 0   /* M_pc^dag M_pc x = b on odd half fields      */
#define QDWF_SYS_FULL      1   /* D x = b on full fields (Schur + normal eq.) */

/* workspace selectors for qdwf_workspace_bytes */
#define QDWF_OP_MPC     0
#define QDWF_OP_MDAGM   1
#define QDWF_OP_SOLVE   2
#define QDWF_OP_REDUCE  3
#define QDWF_OP_TUNE    4

/* ---- types ------------------------------------------------------------ */
typedef struct {
  int32_t L[4];     /* extents x, y, z, t; each even and >= 2                 */
  int32_t Ls;       /* fifth-dimension extent, 1 <= Ls <= 64 (1: 4D fields,    */
                    /* V/2 a multiple of 16)                                    */
  int32_t bc[4];    /* +1 periodic, -1 antiperiodic per direction            */
  double M5;        /* domain-wall height                                    */
  double mf;        /* quark mass (wall coupling -mf)                        */
  double b, c;      /* Mobius coefficients (b != 0); Shamir is b = 1, c = 0   */
} qdwf_action;

typedef struct qdwf_ctx qdwf_ctx;

typedef struct {
  int32_t system;       /* QDWF_SYS_NORMAL_PC or QDWF_SYS_FULL                      */
  int32_t inner_prec;   /* precision of the inner Dslash: QDWF_F64 = plain FP64 CG; */
                        /* F32/F16/BF16 = reliable-update mixed-precision CG        */
  int32_t layout;       /* layout of x, b and every internal vector                 */
  int32_t max_iter;     /* total inner iterations allowed (default 20000 if <= 0)   */
  double tol;           /* target relative FP64 true residual |b-Ax|/|b|            */
  double delta;         /* reliable-update threshold (default 0.1 if <= 0)          */
  int32_t x0_is_guess;  /* nonzero: x holds an initial guess; else x0 = 0          */
  int32_t check_every;  /* iterations between host convergence checks (>= 1)        */
  int32_t use_graph;    /* nonzero: replay the inner iterations as a HIP graph      */
} qdwf_solve_params;

typedef struct {
  int32_t iterations;        /* inner CG iterations (max over right-hand sides)   */
  int32_t reliable_updates;  /* FP64 true-residual recomputations                 */
  int32_t converged;         /* number of right-hand sides that reached tol      */
  int32_t restarts;          /* reserved                                          */
  double true_residual;      /* max over rhs of |b - A x| / |b| in FP64 (system solved) */
  double full_residual;      /* QDWF_SYS_FULL: max over rhs of |b - D x| / |b|    */
  double seconds;            /* wall time of the call                              */
  int64_t flops;             /* hop flops executed (1320 convention)               */
} qdwf_solve_stats;

/* ---- errors ----------------------------------------------------------- */
/* Thread-local message of the last failing call on this thread ("" if none). */
const char* qdwf_last_error(void);

/* ---- lifecycle -------------------------------------------------------- */
/* Validates the action and, on `device`, allocates the library-owned
 * neighbour tables (int32 [2][8][V/2]), the site index (int32 [V]), the
 * 5D-local matrices and the link arrays (filled by qdwf_set_gauge). With
 * Ls = 16 and Lx in {8, 16, 24, 32} it also allocates doubled links (the 8
 * links of each site, 2 x 144 x V/2 reals) in FP32, FP16 and BF16 for the
 * t-sweep form of qdwf_apply_D: 1.2 GB at 32^4. With Ls = 1 it allocates
 * lane-major forward links for the Wilson kernel instead (2 x 4 x 18 x V/2
 * reals in FP64 and in FP32). Distinct contexts are independent; one context must not
 * be used from two threads at once. */
int qdwf_create(const qdwf_action* act, int device, qdwf_ctx** out);
int qdwf_destroy(qdwf_ctx* ctx);

/* Packs the canonical gauge field U (device pointer; complex128 when
 * canon_prec = QDWF_F64, complex64 when QDWF_F32) into library-owned link
 * arrays in every precision, per parity, with the boundary factors bc folded
 * into the links (and rebuilds the doubled links where the context has them). Stream-ordered on `stream` (a hipStream_t, NULL = default). */
int qdwf_set_gauge(qdwf_ctx* ctx, const void* U, int canon_prec, void* stream);

/* Number of reals in one right-hand side of an internal field of `subset`
 * (QDWF_EVEN / QDWF_ODD half field, QDWF_FULL full field). */
size_t qdwf_field_reals(const qdwf_ctx* ctx, int subset);

/* ---- layout conversion ------------------------------------------------ */
/* Canonical spinor (device, complex128 if src_prec = QDWF_F64, complex64 if
 * QDWF_F32; nrhs fields back to back) -> internal field of `subset` in
 * (prec, layout). Down-conversion rounds to nearest even. */
int qdwf_pack_spinor(qdwf_ctx* ctx, void* dst, int prec, int layout, const void* src,
                     int src_prec, int subset, int nrhs, void* stream);
/* Internal -> canonical. For a half field only the sites of that parity are
 * written; the others are left untouched. */
int qdwf_unpack_spinor(qdwf_ctx* ctx, void* dst, int dst_prec, const void* src, int prec,
                       int layout, int subset, int nrhs, void* stream);

/* ---- operators (all asynchronous on `stream`; out must not alias in) --- */
/* Full 5D domain-wall operator: out = D in (dagger = 0) or D^dag in
 * (dagger = 1). in, out: full fields, nrhs right-hand sides. With Ls = 16,
 * the interleaved layout and FP32 storage with 16- or 32-wide x rows, it
 * runs as a sweep of whole x-rows along t (same result up to FP32 rounding
 * order); the environment variable QDWF_SWEEP=1 / 0 forces that form on
 * (also for FP16 and BF16 storage and other row widths in {8, 16, 24, 32})
 * or off. */
int qdwf_apply_D(qdwf_ctx* ctx, void* out, const void* in, int dagger, int prec, int layout,
                 int nrhs, void* stream);

/* Wilson Dslash kernel (Section 4.1, Table 1): out = D_h in, or D_h^dag in
 * (dagger = 1, the projectors (1 -+ g_mu) swapped), on every slice s. With
 * subset = QDWF_FULL, in and out are full fields; with subset = QDWF_EVEN or
 * QDWF_ODD, out is the half field of that parity and in the half field of
 * the other parity. For Ls = 1 these are 4D Wilson fields. Links and the
 * boundary factors bc are those of the context; M5, mf, b, c are not used.
 * 1320 flops per output site. */
int qdwf_apply_Dh(qdwf_ctx* ctx, void* out, const void* in, int subset, int dagger, int prec,
                  int layout, int nrhs, void* stream);

/* Wilson operator: out = (4 + mass) in - 1/2 D_h in (dagger = 1: with
 * D_h^dag) on full fields, every slice s. mass must be finite. */
int qdwf_apply_Dw(qdwf_ctx* ctx, void* out, const void* in, double mass, int dagger, int prec,
                  int layout, int nrhs, void* stream);

/* 4D-local block on `subset` fields: which = QDWF_MEE_FWD gives M_ee,
 * QDWF_MEE_INV gives M_ee^-1; dagger = 1 gives the adjoint. M_ee = M_oo, so
 * the same call serves either parity. out may equal in. */
int qdwf_apply_Mee(qdwf_ctx* ctx, void* out, const void* in, int subset, int dagger, int which,
                   int prec, int layout, int nrhs, void* stream);

/* Off-diagonal block into parity out_parity from half field of parity
 * q = 1 - out_parity: dagger = 0 gives M_{p,q} in = -1/2 D_h A in;
 * dagger = 1 gives (M_{q,p})^dag in = -1/2 A^dag D_h^dag in. */
int qdwf_apply_Deo(qdwf_ctx* ctx, void* out, const void* in, int out_parity, int dagger,
                   int prec, int layout, int nrhs, void* stream);

/* Schur complement on odd half fields: M_pc in (dagger = 0) or M_pc^dag in.
 * ws: qdwf_workspace_bytes(ctx, QDWF_OP_MPC, prec, nrhs) bytes of device memory. */
int qdwf_apply_Mpc(qdwf_ctx* ctx, void* out, const void* in, int dagger, int prec, int layout,
                   int nrhs, void* ws, void* stream);

/* Normal operator on odd half fields: out = M_pc^dag M_pc in.
 * ws: qdwf_workspace_bytes(ctx, QDWF_OP_MDAGM, prec, nrhs) bytes. */
int qdwf_apply_MdagM(qdwf_ctx* ctx, void* out, const void* in, int prec, int layout, int nrhs,
                     void* ws, void* stream);

/* Device workspace size in bytes for an operation (see QDWF_OP_*). */
size_t qdwf_workspace_bytes(const qdwf_ctx* ctx, int op, int prec, int nrhs);

/* ---- domain decomposition emulated on one GPU --------------------------- */
/* D applied as a run split into `ranks` slabs along t would apply it (the
 * paper's 4-rank runs, Section 4.2): each slab packs its two t-faces into
 * spin-projected half spinors (12 reals per face site and slice), the half
 * spinors are exchanged (device copies), the hop runs on the slabs with the
 * cross-slab links zeroed, and the face sites add the received hops.
 * ranks must divide Lt into slabs of at least 2 slices; ranks = 1 exercises
 * the same path across the periodic boundary. Full fields, one right-hand
 * side, D only (no dagger); the result equals qdwf_apply_D up to the order
 * of summation on face sites.
 * ws: qdwf_split_workspace_bytes(ctx, ranks, prec) bytes, filled once by
 * qdwf_split_prepare for this ranks and prec (and again after each
 * qdwf_set_gauge); it holds the cut links, a site table and the face
 * buffers. qdwf_split_prepare synchronises `stream`. */
size_t qdwf_split_workspace_bytes(const qdwf_ctx* ctx, int ranks, int prec);
int qdwf_split_prepare(qdwf_ctx* ctx, int ranks, int prec, void* ws, void* stream);
int qdwf_apply_D_split(qdwf_ctx* ctx, void* out, const void* in, int ranks, int prec, int layout,
                       void* ws, void* stream);

/* ---- streaming probes (no context) ------------------------------------- */
/* Per-site SU(3) product of the Benchmark_su3 study (Section 4.2):
 * C[i] = A[i] B[i] for i < n, each a 3x3 complex matrix stored row-major with
 * interleaved complex (18 reals), FP64 or FP32 (prec). Device arrays on
 * `device`, C must not alias A or B; n = 0 launches nothing. 198 real flops
 * and 54 reals of traffic per matrix. Asynchronous on `stream`. */
int qdwf_su3_mul(void* C, const void* A, const void* B, int64_t n, int prec, int device,
                 void* stream);

/* STREAM triad (Section 3): a[i] = b[i] + s c[i] for i < n reals, FP64 or
 * FP32. a may equal b or c element for element; s must be finite. */
int qdwf_triad(void* a, const void* b, const void* c, double s, int64_t n, int prec, int device,
               void* stream);

/* ---- reductions ------------------------------------------------------- */
/* Per right-hand side r: out[2r] = Re <x_r, y_r>, out[2r+1] = Im <x_r, y_r>,
 * accumulated in FP64 with a fixed reduction order (bitwise reproducible for
 * a given field size). x, y: fields of `subset`, same (prec, layout). out is a
 * host array of 2*nrhs doubles; the call synchronises `stream`.
 * ws: qdwf_workspace_bytes(ctx, QDWF_OP_REDUCE, prec, nrhs) bytes. */
int qdwf_dot(qdwf_ctx* ctx, double* out, const void* x, const void* y, int subset, int prec,
             int layout, int nrhs, void* ws, void* stream);

/* qdwf_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same results, bit for bit, with the partial sums in a
 * static device array of QDWF_NOALLOC_SCRATCH_BYTES per GPU (held until the
 * process ends) instead of a workspace. The call allocates nothing. It
 * returns QDWF_EINVAL, launching nothing, when the reduction needs more
 * scratch than that (qdwf_workspace_bytes(ctx, QDWF_OP_REDUCE, prec, nrhs)
 * bytes; up to 32 right-hand sides fit for any field size). Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other threads,
 * other streams) race and must be serialised by the caller. The first call
 * on a device looks up the array's device address. Synchronises `stream`. */
#define QDWF_NOALLOC_SCRATCH_BYTES 540672
int qdwf_dot_noalloc(qdwf_ctx* ctx, double* out, const void* x, const void* y, int subset,
                     int prec, int layout, int nrhs, void* stream);

/* ---- solver ----------------------------------------------------------- */
/* Solves for nrhs right-hand sides at once: every launch of the solve covers
 * all of them (the hop takes one right-hand side per block unless the tuner
 * chose blocks that share their staged links between several), and a
 * right-hand side that has converged or waits for its reliable update skips
 * its hops. x, b are FP64 fields in params->layout: odd half fields for
 * QDWF_SYS_NORMAL_PC, full fields for QDWF_SYS_FULL. inner_prec = QDWF_F64
 * runs plain FP64 CG; any other value runs CG with that inner precision and
 * FP64 reliable updates (true residual recomputed in FP64; x accumulated in
 * FP64). Convergence is decided only on the FP64 true residual <= tol.
 * ws: qdwf_workspace_bytes(ctx, QDWF_OP_SOLVE, inner_prec, nrhs) bytes.
 * Synchronises `stream` before returning; stats may be NULL.
 * Returns QDWF_ENOTCONV if max_iter is reached, QDWF_ENAN on NaN/Inf. */
int qdwf_solve(qdwf_ctx* ctx, void* x, const void* b, int nrhs, const qdwf_solve_params* params,
               qdwf_solve_stats* stats, void* ws, void* stream);

/* ---- autotuner -------------------------------------------------------- */
/* Times every launch shape of the hop kernel (threads per block, right-hand
 * sides per block, XCD-aware block order, LDS reservation capping resident
 * blocks per CU) on D and D^dag for (prec, layout, nrhs) and keeps the fastest
 * for this context; later calls of every operator with that precision,
 * layout and nrhs use it. If the environment variable QDWF_TUNE_CACHE names a
 * file, results are appended to it and contexts of the same shape created
 * later pick them up. ws: qdwf_workspace_bytes(ctx, QDWF_OP_TUNE, prec, nrhs)
 * bytes (overwritten). best_ms (may be NULL) receives 2 doubles: the best
 * D and D^dag times. Synchronous. */
int qdwf_tune(qdwf_ctx* ctx, int prec, int layout, int nrhs, void* ws, void* stream,
              double* best_ms);
/* The shape the operators will use: {threads, nrhs per block, xcd order, lds reservation}. */
int qdwf_tuned_shape(qdwf_ctx* ctx, int prec, int layout, int dagger, int nrhs, int32_t* shape4);

/* Traversal and layout search for the lattice of `act` (Section 4.3 compares
 * the two complex layouts; the site order is this library's own choice).
 * The site traversal order -- the split dimension cut into 8 slabs (one per
 * XCD), the sweep dimension, and the tile over the other dimensions -- is
 * fixed when a context is created, and the spinor layout when a field is
 * packed, so the search runs on throwaway contexts on `device` (unit links,
 * zero fields): for each candidate traversal (split z / sweep t with x tiles
 * of 32 or 16 and y tiles of 2, 4 or 8; split y / sweep t; split t / sweep z,
 * each capped by the extents) and each layout (RIRI, RRII) it times
 * qdwf_apply_D (dagger 0, precision prec, nrhs right-hand sides, the launch
 * shape each context would use). choice7 receives {split, sweep, tile x,
 * tile y, tile z, tile t, layout} of the fastest, best_ms (may be NULL) its
 * time per application. If QDWF_TUNE_CACHE names a file the choice is
 * appended to it, keyed by lattice, Ls and device architecture, and every
 * later qdwf_create of that lattice and Ls takes that traversal (unless
 * QDWF_ORDER or QDWF_TILE is set); the caller packs in the returned layout.
 * Allocates device memory (the contexts, canonical unit links and two
 * fields) on `device`; `stream` must belong to `device`; synchronous.
 * Returns QDWF_EINVAL for an invalid action, device or precision. */
int qdwf_tune_traversal(const qdwf_action* act, int device, int prec, int nrhs, void* stream,
                        int32_t* choice7, double* best_ms);
/* The traversal of a context: {split, sweep, tile x, tile y, tile z, tile t}
 * (host buffer of 6 int32). */
int qdwf_traversal(qdwf_ctx* ctx, int32_t* order6);

/* ---- serving pool ----------------------------------------------------- */
/* Continuous batching of independent solves of M_pc^dag M_pc x_o = b_o, each
 * with its own lattice, action, gauge field and source. Requests wait in FIFO
 * order until their device memory (qdwf_request_bytes) fits the caller's
 * arena and one of max_slots slots is free. All admitted requests advance
 * together: each qdwf_pool_step replays one round -- check_every repetitions
 * of [the reliable updates that are due; one CG iteration] -- in which every
 * step of the iteration is a single launch covering all of them (kernels walk
 * a device table of the requests' arguments), captured as a HIP graph when
 * the pool is created. A request's result does not depend on what else is
 * in the pool: its arithmetic is that of qdwf_solve on one right-hand side
 * with the same parameters.
 *
 * Memory: the caller owns the arena (device memory, 256-byte aligned, kept
 * valid until qdwf_pool_destroy); the pool sub-allocates it for its own table
 * and states (qdwf_pool_overhead_bytes), for each admitted request's links,
 * matrices, vectors and workspace, and for the site tables of each lattice
 * shape (shared by the requests of that shape, kept while room allows). After
 * qdwf_pool_create the pool allocates no device memory; it holds pinned host
 * staging allocated at creation. Not thread-safe per pool. */
typedef struct qdwf_pool qdwf_pool;

typedef struct {
  qdwf_action act;            /* lattice and action; 8 <= Ls <= 32                  */
  const void* U;              /* canonical gauge field, complex128, device          */
  const void* b;              /* canonical source, complex128, device; odd sites used */
  void* x_out;                /* canonical complex128 device buffer; odd sites are  */
                              /* written when the request finishes                   */
  qdwf_solve_params params;   /* tol, delta, max_iter per request; inner_prec and    */
                              /* layout must be the pool's; system NORMAL_PC, x0 = 0 */
} qdwf_request;               /* U, b, x_out must stay valid until the request ends */

/* Arena bytes a request occupies while admitted, counting its lattice shape's
 * site tables (shared with other admitted requests of that shape). */
size_t qdwf_request_bytes(const qdwf_action* act, const qdwf_solve_params* params);
/* Arena bytes the pool keeps for itself (0 for max_slots out of range). */
size_t qdwf_pool_overhead_bytes(int max_slots);
/* params: inner_prec and layout of every request, check_every = iterations
 * per round (1..64; default 8 if <= 0). max_slots in [1, 64]. The arena's
 * size is the pool's budget; creation fails with QDWF_EINVAL if it is smaller
 * than qdwf_pool_overhead_bytes(max_slots). */
int qdwf_pool_create(int device, void* arena, size_t arena_bytes, int max_slots,
                     const qdwf_solve_params* params, qdwf_pool** out);
/* Waits for the round in flight, then frees the pool (not the arena). */
int qdwf_pool_destroy(qdwf_pool* pool);
/* Queues a request (never blocks); QDWF_EINVAL if it can never fit the arena
 * or its parameters do not match the pool. */
int qdwf_pool_submit(qdwf_pool* pool, const qdwf_request* req, uint64_t* id);
/* One scheduling step on `stream` (a hipStream_t, NULL = default): waits for
 * the previous round, retires the requests it finished (their x_out written
 * by work queued on `stream`), admits queued requests that fit, and queues
 * the next round for all admitted requests. *n_active (may be NULL) receives
 * the number of requests admitted after the step. */
int qdwf_pool_step(qdwf_pool* pool, void* stream, int* n_active);
/* QDWF_EBUSY while the request is queued or running; otherwise its solve
 * status (QDWF_OK, QDWF_ENOTCONV, QDWF_ENAN, ...) with stats filled, after
 * which the id is forgotten. A finished request's x_out is complete once the
 * work queued on the step's stream has run. */
int qdwf_pool_poll(qdwf_pool* pool, uint64_t id, qdwf_solve_stats* stats);
/* Arena bytes in use now and at peak (including the pool's own), and the
 * numbers of admitted and queued requests. */
int qdwf_pool_info(qdwf_pool* pool, size_t* in_use, size_t* peak, int* n_active, int* n_queued);

/* ---- geometry (tests) ------------------------------------------------- */
/* Copies the tables the kernels use into host buffers: cb_of_lex[V] (int32:
 * the internal index i of each lex site within its parity), nbr[2][V/2][8]
 * (int32: internal index of the neighbour, in the opposite parity, in
 * directions +x,+y,+z,+t,-x,-y,-z,-t) and sign[2][V/2][8] (int8 boundary
 * factor of the hop). Any pointer may be NULL. Synchronous. */
int qdwf_geometry_tables(qdwf_ctx* ctx, int32_t* cb_of_lex, int32_t* nbr, int8_t* sign);

#ifdef __cplusplus
}
#endif

#endif /* QDWF_H */
