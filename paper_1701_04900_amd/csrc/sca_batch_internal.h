// Internal declarations of the batched engine, shared with the adjoint.
#pragma once
#include <vector>

#include "sca_internal.h"

struct sca_batch;

namespace sca {

constexpr int kBC = 8;           // columns per gradient work item
constexpr int kBMaxGroups = 32;  // fold: max column groups per instance and round

struct BInst {
  const void* A;
  long long lda;
  int m, n;
  int row_off, col_off, blk_off, nblk;
  double lam, c, beta, tau, F_star;
  unsigned int inst_id;
  int pad;
};

struct BItem {
  int pos;   // first position in the drawn list
  int cnt;   // columns (<= kBC), all of one block
  int inst;  // instance
};

struct BState {
  RoundState rs;   // round counter, step, totals, compaction results
  int items;       // work items of the round in flight
  int tiles;       // fold tiles of the fold in flight
  long long cost;  // fused round: total cost of the round's items (the shares' split)
};


// FP64 residual A_k x_k - b_k of every instance into the batch's r64 (stream-ordered).
void batch_fresh_residual(sca_batch* B, const void* x, hipStream_t s);

}  // namespace sca

// Host object of a batch.
struct sca_batch {
  using BInst = sca::BInst;
  using BItem = sca::BItem;
  using BState = sca::BState;
  int dtype = SCA_F32;
  size_t esize = 4;
  int K = 0;
  long long Mtot = 0, Ntot = 0;
  int Btot = 0;
  int ncu = 256;
  int reg = 0;
  double theta = 0, eta = 1;
  std::vector<BInst> hinst;
  std::vector<long long> xoff, roff;
  // device
  BInst* d_inst = nullptr;
  int *d_blk_inst = nullptr, *d_blk_col0 = nullptr, *d_blk_len = nullptr, *d_blk_cols = nullptr;
  int *d_row_inst = nullptr, *d_col_inst = nullptr;
  int *d_chunk_a = nullptr, *d_chunk_b = nullptr, *d_chunk_cnt = nullptr;
  double* d_cn2 = nullptr;
  void* d_b = nullptr;
  double* d_r64 = nullptr;
  void* d_rrun = nullptr;  // running residual of batch_solve
  int* d_sel_cols = nullptr;
  BItem* d_items = nullptr;
  void* d_dx_sel = nullptr;
  int* d_J_idx = nullptr;
  void* d_J_val = nullptr;
  int *d_J_lo = nullptr, *d_Jn = nullptr, *d_G = nullptr, *d_ng = nullptr, *d_nrt = nullptr,
      *d_tile_off = nullptr;
  double* d_part = nullptr;
  BState* d_state = nullptr;
  int* d_active = nullptr;
  long long* d_done = nullptr;
  long long* d_upd = nullptr;
  double* d_F = nullptr;
  double *d_cm = nullptr, *d_cs = nullptr;
  int* d_cz = nullptr;
  double* d_pr = nullptr;
  // fused round (bf_q > 0): one pass over the drawn columns with the fold from registers;
  // item cost prefix, first item of every workgroup's share, first/last item of every
  // instance, chunk cost sums, one partial m-vector per (workgroup, instance) slot
  int bf_wg_per_cu = 2;  // 256-thread workgroups per CU
  int bf_kind = 1;       // 1: fused round, 0: two-pass round
  int bf_q = 0;          // row groups per thread (template), 0 when the fused round cannot run
  long long bf_pst = 0;  // partial slot stride (elements)
  int bf_gmax = 0;       // largest grid the partial slots were allocated for
  long long* d_item_pref = nullptr;
  long long* d_chunk_cost = nullptr;
  int* d_wg_first = nullptr;
  int* d_inst_lo = nullptr;
  int* d_inst_hi = nullptr;
  int* d_tile_base = nullptr;
  int* d_tile_inst = nullptr;  // instance of every fused-reduction tile
  int bf_tiles = 0;
  void* d_bpart = nullptr;
  // checks of sca_batch_solve from the running residual (candidates confirmed fresh)
  int* d_cand = nullptr;
  sca_adj_cache* adj = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_rounds = 0;
  const void* graph_x = nullptr;
  double graph_tol = 0;
  double graph_tol_merit = 0;
  double graph_p = 0;
  uint64_t graph_seed = 0;
};

