// Solver-side declarations shared by the API layer and the serving pool.
#pragma once

#include "common.h"

namespace qdwf {

enum { ST_RUN = 0, ST_UPDATE = 1, ST_DONE = 2, ST_NAN = 3, ST_BREAKDOWN = 4 };

// Per right-hand-side CG state, resident on the device.
struct RhsState {
  double rr;           // inner |r|^2 in scaled units
  double rr_prev;      // inner |r|^2 of the previous iteration
  double pAp, alpha, beta;
  double rr_ru;        // inner |r|^2 right after the last reliable update
  double sigma;        // scale of the inner vectors (physical = inner / sigma)
  double sigma_ratio;  // new sigma / old sigma at a reliable update
  double w_r;          // weight of r in the p restart at a reliable update
  double bb;           // |b|^2
  double thresh;       // inner |r|^2 at which the target is reached
  double rr_true;      // last FP64 true |b - A x|^2
  int status, iters, ru;
  int fresh;           // set by a reliable update, cleared by the next iteration
};

int reduce_blocks(long n);
int apply_hop_parity(qdwf_ctx* ctx, int prec, int layout, int dagger, int out_par, void* out,
                     const void* in, const void* z, double scale, int nrhs, long rs,
                     hipStream_t st);
int apply_mpc(qdwf_ctx* ctx, int prec, int layout, int dagger, void* out, const void* in,
              void* te1, void* te2, int nrhs, long rs, hipStream_t st);
int apply_mdagm(qdwf_ctx* ctx, int prec, int layout, void* out, const void* in, void* v,
                void* te1, void* te2, int nrhs, long rs, hipStream_t st);
int dot_re_im(qdwf_ctx* ctx, double* out_host, const void* x, const void* y, long n, int prec,
              int layout, int nrhs, void* ws, hipStream_t st);
size_t dot_ws_bytes(long n, int nrhs);
size_t solve_ws_bytes(const qdwf_ctx* ctx, int inner, int nrhs, int system);
int solve(qdwf_ctx* ctx, double* x, const double* b, int nrhs, const qdwf_solve_params& prm,
          qdwf_solve_stats* stats, void* ws, hipStream_t st);

// Resumable normal-equation CG on odd half fields (stride = one half field):
// begin() launches the set-up, then complete() waits for the last round and
// launch() starts the next one, until complete() reports finished.
struct Solver {
  virtual ~Solver() {}
  virtual int begin() = 0;
  virtual int launch() = 0;
  virtual int complete(bool* finished) = 0;
  virtual void fill_stats(qdwf_solve_stats* stats) const = 0;
  virtual int result() const = 0;
};
Solver* make_solver(qdwf_ctx* ctx, const qdwf_solve_params& prm, int nrhs, double* x,
                    const double* b, void* ws, hipStream_t st);

// Geometry-only sizes used for admission control.
size_t ctx_bytes(const qdwf_action& a);
size_t solve_ws_bytes_for(const qdwf_action& a, int inner, int nrhs);

}  // namespace qdwf
