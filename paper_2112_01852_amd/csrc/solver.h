// Solver-side declarations shared by the API layer and the serving pool.
#pragma once

#include "common.h"

namespace qdwf {

enum { ST_RUN = 0, ST_UPDATE = 1, ST_DONE = 2, ST_NAN = 3, ST_BREAKDOWN = 4, ST_NOTCONV = 5 };

// Per right-hand-side CG state, resident on the device.
struct RhsState {
  double rr;           // inner |r|^2 in scaled units
  double rr_prev;      // inner |r|^2 of the previous iteration
  double pAp, alpha, beta;
  double alpha_hist[8];   // alpha of each iteration of the current group (grouped x updates)
  double rr_ru;        // inner |r|^2 right after the last reliable update
  double sigma;        // scale of the inner vectors (physical = inner / sigma)
  double sigma_ratio;  // new sigma / old sigma at a reliable update
  double w_r;          // weight of r in the p restart at a reliable update
  double bb;           // |b|^2
  double thresh;       // inner |r|^2 at which the target is reached
  double rr_true;      // last FP64 true |b - A x|^2
  int status, iters, ru;
  int fresh;           // set by a reliable update, cleared by the next iteration
  int first;           // the next reliable update is the initial one
  int final;           // out of iterations: the next reliable update ends the solve
  int max_iter;        // iteration limit kept on the device (0: the host enforces it)
  int xstep;           // the iteration's x step is due (running when |r|^2 was taken)
  int xmask;           // bit j: iteration j of the current group took its step
};

// The CG step a solver iteration fuses into the epilogue hop of M_pc or
// M_pc^dag (HopArgs::cg and the fields after it; x and p only for cg = 3).
struct CgFuse {
  int mode;
  void* r;
  const double* alpha;
  int alpha_stride;
  double* site;
  void* x;
  const void* p;
};

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace of a solve of nrhs right-hand sides of n reals: byte offsets of
// its vectors, each on a 256-byte boundary.
struct Layout {
  // FP64 vectors: r_hi, Ax, v_hi, te1_hi, te2_hi
  size_t off_rh, off_ax, off_vh, off_t1h, off_t2h;
  // inner: x_lo, r_lo (R type); p, Ap, v, te1, te2 (S type)
  size_t off_xl, off_rl, off_p, off_ap, off_v, off_t1, off_t2;
  size_t off_part, off_state, off_stage;
  size_t total;
};
// Search-direction slots of qdwf_solve's grouped iterations (the serving
// pool's members have one).
constexpr int kGroupSlots = 8;
// grouped: off_p is the first of kGroupSlots consecutive slots, each
// al256(p bytes) apart
Layout solver_layout(long n, int nrhs, int inner, bool grouped = false);

int reduce_blocks(long n);
int site_blocks(long nsite);
// skip, skip_stride: per right-hand-side flags of the hops (HopArgs::skip)
int apply_hop_parity(qdwf_ctx* ctx, int prec, int layout, int dagger, int out_par, void* out,
                     const void* in, const void* z, double scale, int nrhs, long rs,
                     hipStream_t st, const int* skip = nullptr, int skip_stride = 0);
int apply_mpc(qdwf_ctx* ctx, int prec, int layout, int dagger, void* out, const void* in,
              void* te1, void* te2, int nrhs, long rs, hipStream_t st,
              const int* skip = nullptr, int skip_stride = 0, const CgFuse* cg = nullptr);
int apply_mdagm(qdwf_ctx* ctx, int prec, int layout, void* out, const void* in, void* v,
                void* te1, void* te2, int nrhs, long rs, hipStream_t st,
                const int* skip = nullptr, int skip_stride = 0);
int dot_re_im(qdwf_ctx* ctx, double* out_host, const void* x, const void* y, long n, int prec,
              int layout, int nrhs, void* ws, hipStream_t st);
size_t dot_ws_bytes(long n, int nrhs);
size_t solve_ws_bytes(const qdwf_ctx* ctx, int inner, int nrhs, int system);
int solve(qdwf_ctx* ctx, double* x, const double* b, int nrhs, const qdwf_solve_params& prm,
          qdwf_solve_stats* stats, void* ws, hipStream_t st);

}  // namespace qdwf
