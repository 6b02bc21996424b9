// Grouped CG: the even-odd normal-equation solves of many independent
// requests (each its own lattice, Ls, mass, gauge field and source) advanced
// together, one launch per step of the iteration for all of them. The serving
// pool's engine.
//
// A group keeps, in device memory the caller provides, a descriptor table:
// per request its hop arguments for the four stages of M_pc^dag M_pc (inner
// precision and FP64), its local-operator arguments, its vectors and its CG
// state. Every grouped kernel walks the units of all requests listed in the
// table (blocks of a request's field, grid-stride over a fixed grid), so one
// captured round of iterations serves any membership: changing the members
// rewrites the table, never the graph.
//
// Each request's arithmetic is that of qdwf_solve on one right-hand side
// with the same parameters: the same kernel bodies (hopbody.h, localbody.h,
// cgbody.h), its own reduction tree, and the same sequence of iterations and
// reliable updates. A round is `k` repetitions of [reliable update for the
// requests that asked for one; one iteration for the running ones], each
// step skipping the requests it does not apply to. Results are therefore
// independent of what else is in the group.
#pragma once

#include "common.h"
#include "solver.h"

namespace qdwf {

constexpr int kGroupMax = 64;   // requests in one group

// One request of a group. Device pointers; the context's links, site tables
// and 5D-local matrices must be in place (context made by the caller).
struct GroupMember {
  qdwf_ctx* ctx;
  double* xo;           // FP64 solution, odd half field (written at the end)
  const double* bo;     // FP64 source, odd half field
  char* ws;             // solver_layout(n, 1, inner).total bytes
  RhsState* st;         // its CG state
  double tol;           // target relative FP64 true residual
  double delta;         // reliable-update threshold (<= 0: 0.1)
  int max_iter;         // iteration limit (<= 0: 20000)
};

class GroupEngine {
 public:
  // inner / layout: precision and layout every member uses; k: iterations
  // per round. table_mem: group_table_bytes() bytes of device memory (kept
  // for the engine's life); capture: a stream with no work in flight used to
  // capture the round (not the null stream). Host staging for the table is
  // allocated here (pinned).
  static int create(int device, int inner, int layout, int k, void* table_mem,
                    hipStream_t capture, GroupEngine** out);
  ~GroupEngine();
  // Replaces the member list (n <= kGroupMax) and uploads the table on st.
  // The previous round must have completed (its table is still being read
  // otherwise).
  int set_members(const GroupMember* m, int n, hipStream_t st);
  // Starts a new member's solve on st: |b|^2, state, x = 0; its first round
  // then opens with the initial reliable update.
  int start_member(const GroupMember& m, hipStream_t st);
  // One round (k repetitions) for every member, on st.
  int launch_round(hipStream_t st);
  int inner() const { return inner_; }
  int layout() const { return layout_; }

 private:
  GroupEngine() = default;
  int capture(hipStream_t cs);
  int device_ = 0, inner_ = 0, layout_ = 0, k_ = 1;
  void* table_ = nullptr;     // device
  void* staging_ = nullptr;   // pinned host copy of the table
  hipGraphExec_t exec_ = nullptr;
};

size_t group_table_bytes();

}  // namespace qdwf
