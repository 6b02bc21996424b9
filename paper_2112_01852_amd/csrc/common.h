// Internal declarations of libqdwf: storage types, the context, launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "qdwf.h"

namespace qdwf {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

#define QDWF_HIP(call)                                                               \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::qdwf::fail(QDWF_EDEVICE, "%s failed: %s (%s:%d)", #call,             \
                          hipGetErrorString(e_), __FILE__, __LINE__);                \
  } while (0)

// ---------------------------------------------------------- storage types
// bf16 is kept as raw bits; conversions round to nearest even.
struct bf16 {
  uint16_t u;
};

template <class S> struct Store;

// from64() converts an FP64 value with a single rounding (used by the packers).
template <> struct Store<double> {
  typedef double compute;
  __device__ __host__ static inline double to(double v) { return v; }
  __device__ __host__ static inline double from(double v) { return v; }
  __device__ static inline double from64(double v) { return v; }
};
template <> struct Store<float> {
  typedef float compute;
  __device__ __host__ static inline float to(float v) { return v; }
  __device__ __host__ static inline float from(float v) { return v; }
  __device__ static inline float from64(double v) { return (float)v; }
};
// FP32 value of v rounded to odd: correct final rounding to any format with
// at least two fewer significand bits (round-to-odd, Boldo and Melquiond).
__device__ inline float round_to_odd_f32(double v) {
  float f = (float)v;
  if ((double)f != v) {
    uint32_t u = __float_as_uint(f);
    if (!(u & 1u)) u = (fabs((double)f) < fabs(v)) ? u + 1u : u - 1u;
    f = __uint_as_float(u);
  }
  return f;
}
template <> struct Store<_Float16> {
  typedef float compute;
  __device__ static inline float to(_Float16 v) { return (float)v; }
  __device__ static inline _Float16 from(float v) { return (_Float16)v; }
  __device__ static inline _Float16 from64(double v) { return (_Float16)round_to_odd_f32(v); }
};
template <> struct Store<bf16> {
  typedef float compute;
  __device__ static inline float to(bf16 v) { return __uint_as_float(((uint32_t)v.u) << 16); }
  __device__ static inline bf16 from(float v) {
    uint32_t x = __float_as_uint(v);
    bf16 r;
    if ((x & 0x7f800000u) == 0x7f800000u && (x & 0x007fffffu)) {
      r.u = (uint16_t)((x >> 16) | 0x40);  // quiet NaN
    } else {
      x += 0x7fffu + ((x >> 16) & 1u);
      r.u = (uint16_t)(x >> 16);
    }
    return r;
  }
  __device__ static inline bf16 from64(double v) { return from(round_to_odd_f32(v)); }
};

inline size_t prec_bytes(int prec) {
  switch (prec) {
    case QDWF_F64: return 8;
    case QDWF_F32: return 4;
    default: return 2;
  }
}

// -------------------------------------------------------------- geometry
struct Geom {
  int L[4];
  int Ls;
  int V;      // 4D volume
  int Vh;     // V/2
  long n5h;   // Vh*Ls: 5D sites of one parity
};

// 5D-local chiral matrices (Ls x Ls per chirality) kept on device.
// MAT_AMEEINV = (A/b) M_ee^-1 = (1 + (c/b) C) M_ee^-1: the first stage of M_pc
// hands the second its input with A already applied.
enum MatKind { MAT_MEE = 0, MAT_MEE_DAG, MAT_MEEINV, MAT_MEEINV_DAG, MAT_AMEEINV, MAT_COUNT };

// Launch shape of the hop kernel, chosen per (precision, layout, nrhs) by
// the tuner or by the default rule.
struct HopShape {
  int threads;   // threads per block (multiple of 64)
  int nrb;       // right-hand sides per block
  int xcd;       // 1: XCD-aware block order
  int lds_pad;   // extra LDS bytes per block: caps the blocks resident per CU
  int sweep;     // 1: the t-sweep traversal of the full operator where it applies
};

}  // namespace qdwf

namespace qdwf {

// Site tables of a lattice shape and boundary: the traversal order of each
// parity and the neighbour table in that order, built on the host; shared by
// every context of that shape (a serving pool keeps one per shape).
struct GeomTables {
  int L[4], bc[4];
  int tile[4];                     // tile of the traversal order (1 on the sweep dimension)
  int order[2];                    // split and sweep dimension of the traversal order
  std::vector<int32_t> site_lex;   // [2][Vh] lex index of each internal site
  std::vector<int32_t> idx;        // [V] internal index of each lex site
  std::vector<int32_t> nbr;        // [2][8][Vh] internal index of each neighbour
  std::vector<int8_t> sign;        // [2][8][Vh] boundary factor of each hop
};
// qdwf_solve's captured inner iterations and what they were captured for.
struct SolveGraph {
  hipGraphExec_t exec = nullptr;
  const void* ws = nullptr;
  int nrhs = 0, inner = -1, layout = -1, k = 0;
  double delta2 = -1.0;
};

// Site traversal order of a lattice: the split dimension (cut into 8 slabs,
// one per XCD), the sweep dimension, and the tile over the other dimensions
// (tile[sweep] is 1).
struct Traversal {
  int split, sweep;
  int tile[4];
};
// The default tile for a split and sweep dimension: (x, y, z) tile
// 32 x 4 x Lz/8 for split z, sweep t; otherwise 4 on every dimension and
// L/8 on the split one (each capped by the extent).
Traversal default_traversal(const int L[4], int split, int sweep);
// The traversal a new context of this lattice takes: QDWF_ORDER /
// QDWF_TILE if either is set; else the last one qdwf_tune_traversal stored
// in the QDWF_TUNE_CACHE file for this lattice, Ls and device architecture
// (not looked up when Ls <= 0); else default_traversal(L, 2, 3).
Traversal pick_traversal(const int L[4], int Ls, int device);
// qdwf_create with the traversal tr (nullptr: pick_traversal's).
int create_context(const qdwf_action* act, int device, const Traversal* tr, qdwf_ctx** out);
// Builds the tables (throws std::bad_alloc on host memory exhaustion).
std::shared_ptr<const GeomTables> build_geometry(const int L[4], const int bc[4],
                                                 const Traversal& tr);

// Device arrays of a context, each on a 256-byte boundary of one block:
// byte offsets, SIZE_MAX where absent. geom_bytes: the site tables, which come
// first (nbr, site_lex, idx); the rest depends on the action.
struct CtxLayout {
  size_t nbr, site_lex, idx, mat64, mat32;
  size_t links[4], dlinks[4], wlinks[4];
  size_t geom_bytes, total;
};
// with_geom: the block holds the site tables; link_mask: bit p set for the
// packed links of precision p; derived: the doubled links of the t-sweep and
// the lane-major links of 4D contexts, where the geometry has them.
CtxLayout ctx_layout(const qdwf_action& a, bool with_geom, unsigned link_mask, bool derived);

}  // namespace qdwf
struct qdwf_ctx;
namespace qdwf {
// Points the context's array members at the block `base` laid out by lay.
void place_arrays(qdwf_ctx* c, char* base, const CtxLayout& lay);
// Copies the site tables (with_geom) and the 5D-local matrices of c to the
// device (synchronous copies; contexts of qdwf_create).
hipError_t upload_tables(qdwf_ctx* c, bool with_geom);
// Releases qdwf_solve's per-context state (pinned copy, event, graph), or
// only its cached graph (after anything that changes the launches it holds).
void forget_solver_state(qdwf_ctx* c);
void forget_graph(qdwf_ctx* c);

}  // namespace qdwf

struct qdwf_ctx {
  qdwf_action act;
  int device;
  qdwf::Geom g;
  std::shared_ptr<const qdwf::GeomTables> geo;   // host copy of the site tables
  void* d_block;           // the context's device block (nullptr when the arrays live
                           // in memory the context does not own, e.g. a pool arena)
  int32_t* d_nbr;          // [2][8][Vh] neighbour internal index
  int32_t* d_site_lex;     // [2][Vh] lex index of each internal site
  int tile[4];             // tile of the traversal order (1 on the sweep dimension)
  int order[2];            // split and sweep dimension of the traversal order
  void* d_links[4];        // per precision: [2][4][Vh][18] reals, bc folded in
                           // (nullptr for a precision the context does not keep)
  void* d_dlinks[4];       // per precision (32- and 16-bit, t-sweep geometries only):
                           // [2][Vh][8][18], the 8 links of each site (U_mu(x), then
                           // U_mu(x - mu) taken from the other parity), bc folded in
  int32_t* d_idx;          // [V] internal index of each lex site
  void* d_wlinks[4];       // FP64 and FP32, Ls = 1 only: lane-major forward links of the
                           // Wilson kernel, per [parity][mu]: [4][Vh][4] then [Vh][2] reals
  bool gauge_set;
  double* d_mat64;         // [MAT_COUNT][2][Ls][Ls]
  float* d_mat32;
  std::vector<double> h_mat;  // host copy
  // qdwf_solve's reusable host state: pinned copy of the per-rhs CG states
  // and the round event (created on first use, freed with the context), and
  // the graph of its inner iterations for the last workspace it was given
  void* h_pin;
  size_t h_pin_bytes;
  hipEvent_t ev;
  qdwf::SolveGraph graph;
};

namespace qdwf {

// ------------------------------------------------------ kernel launchers
// Hop family. One launch computes, for every output parity p in
// [par0, par0 + npar) and every right-hand side r,
//   h      = D_h   chi          (dagger = 0, chi = A in)  or
//   h      = A^dag D_h^dag in   (dagger = 1)
//   out    = hop_scale * h + [epi] (alpha z + beta C z)   (C^dag when dagger)
//   out    = hop_scale * M_ee^-1 h  (M_ee^-dag when dagger)  with minv = 1
// in[p] is the half field of parity 1-p feeding output parity p; z[p] is at
// parity p. rhs strides are in reals.
struct HopArgs {
  const void* in[2];
  void* out[2];
  const void* z[2];
  long rs_in, rs_out, rs_z;
  int par0, npar;
  int nrhs;
  int epi;
  int minv;   // 1: apply M_ee^-1 (M_ee^-dag when dagger) to the result; Ls = 16, epi = 0
  int chi;    // D_h only (dagger = 0): without minv, in holds (A/b) in, which the hop
              // takes as it is; with minv, the result is multiplied by A/b
  double hop_scale, alpha, beta;
  const void* links;   // links to use instead of the context's (nullptr: the context's)
  // nullptr, or one int per right-hand side (at skip[r * skip_stride]): a
  // block whose right-hand sides all hold a nonzero value there does no work
  // and leaves its outputs as they were (the solver passes its per-rhs
  // status, so the hops of a right-hand side that waits for its reliable
  // update cost a launch, not a pass over memory)
  const int* skip;
  int skip_stride;
  // CG step fused into a one-parity hop with epilogue (no minv), for the
  // solver's M_pc p and M_pc^dag (M_pc p); cg_site[r * Vh + i] receives a
  // sum of squares over the Ls slices of checkerboard site i of rhs r:
  //   cg = 1: of the output as stored;
  //   cg = 2: the output is not stored; cg_r -= alpha_r * output instead
  //     (alpha_r = cg_alpha[r * cg_alpha_stride]; cg_r in FP16 for FP16
  //     storage, else in the compute type: double for FP64 storage and
  //     float otherwise; in the output's layout and rhs stride), and the
  //     sums are of the updated cg_r as stored;
  //   cg = 3: as cg = 2, and cg_x += alpha_r * cg_p at the same sites (the
  //     iteration's step: cg_p the search direction in the storage type,
  //     cg_x the inner solution in the compute type; both in the output's
  //     layout and rhs stride).
  // Rhs whose skip flag is set are left alone.
  int cg;
  void* cg_r;
  const double* cg_alpha;
  int cg_alpha_stride;
  double* cg_site;
  void* cg_x;
  const void* cg_p;
};
int launch_hop(qdwf_ctx* ctx, int prec, int layout, int dagger, const HopArgs& a,
               hipStream_t st, const HopShape* shape = nullptr);

// t-sweep traversal of the full operator (both parities, epi, z = the input
// itself, no fused M_ee^-1, the context's links): Ls = 16, interleaved
// layout, 32- or 16-bit storage, Lx in {8, 16, 24, 32}. sweep_eligible says
// whether launch_sweep accepts the call; launch_hop routes there when the
// launch shape asks for it (HopShape::sweep) or QDWF_SWEEP=1 forces it.
bool sweep_eligible(const qdwf_ctx* ctx, int prec, int layout, const HopArgs& a);
int launch_sweep(qdwf_ctx* ctx, int prec, int dagger, const HopArgs& a, hipStream_t st);
// Whether the context keeps doubled links for the t-sweep, and their build
// from the packed links (after every gauge update).
bool sweep_geometry(const qdwf::Geom& g);
int launch_doubled_links(qdwf_ctx* ctx, hipStream_t st);
// Lane-major links of the Wilson kernel (Ls = 1 contexts), after every gauge update.
int launch_wilson_links(qdwf_ctx* ctx, hipStream_t st);

// Wilson family (no fifth-dimension terms, links read from global memory):
// out = hop_scale * D_h in  (+ alpha z when epi), D_h^dag when dagger, with
// the same argument conventions as launch_hop (beta is unused).
int launch_wilson(qdwf_ctx* ctx, int prec, int layout, int dagger, const HopArgs& a,
                  hipStream_t st);

// Streaming probes: C[i] = A[i] B[i] for n 3x3 complex matrices, and
// a = b + s c for n reals (FP64 or FP32).
int launch_su3_mul(void* C, const void* A, const void* B, long n, int prec, hipStream_t st);
int launch_triad(void* a, const void* b, const void* c, double s, long n, int prec,
                 hipStream_t st);

// out = K in with K the chiral Ls x Ls matrices of `kind`, on `nhalf` half
// fields of nrhs right-hand sides each (half fields are consecutive with
// stride rs_half reals inside one rhs block of stride rs reals).
int launch_local(qdwf_ctx* ctx, int prec, int layout, MatKind kind, void* out, const void* in,
                 int nhalf, long rs_half, long rs, int nrhs, hipStream_t st);

int launch_pack(qdwf_ctx* ctx, void* dst, int prec, int layout, const void* src, int src_prec,
                int subset, int nrhs, hipStream_t st, bool unpack);
int launch_pack_links(qdwf_ctx* ctx, const void* U, int canon_prec, hipStream_t st);

// Default hop launch shape and tuner cache lookup.
HopShape default_shape(const qdwf_ctx* ctx, int prec, int nrhs);
bool tuned_shape(const qdwf_ctx* ctx, int prec, int layout, int dagger, int nrhs, HopShape* out);
void forget_tuning(const qdwf_ctx* ctx);

}  // namespace qdwf
