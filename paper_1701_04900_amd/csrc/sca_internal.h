// Internal declarations shared by the host translation units of libsca.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "../../include/sca.h"
#include "sca_kernels.h"

struct sca_adj_cache;  // adjoint workspace (created on first use)

struct sca_problem {
  // problem data
  int dtype = SCA_F32;
  size_t esize = 4;
  int64_t m = 0, n = 0, lda = 0;
  const void* A = nullptr;  // dense: borrowed column-major A
  const void* b = nullptr;  // borrowed
  double lam = 0, c = 0, beta = INFINITY;
  int reg = 0;
  double theta = 0, eta = 1;
  int64_t nblocks = 0;
  std::vector<int64_t> block_ptr_host;
  double cn2_min = 0;
  int ncu = 256;
  int grad_wg_per_cu = 2;  // gradient kernel: 256-thread workgroups per CU
  int grad_unroll = 2;     // gradient kernel: 16-byte loads (wave) / row steps (wg) in flight
  int grad_kind = 1;       // 0: one wave per column, 1: one workgroup per group of columns
  int grad_cols = 8;       // workgroup variant: columns per group

  // sparse A (library-owned CSC: colptr n+1, rowidx nnz, vals nnz)
  bool sparse = false;
  int64_t nnz = 0;
  long long* csc_colptr = nullptr;
  int* csc_rowidx = nullptr;
  void* csc_vals = nullptr;
  // binned fold: rows in bins of 2^bin_log; counts per (workgroup, bin) of the gradient
  // grid, bin totals, moved columns per workgroup, and up to nnz (row, value) entries
  int bin_log = 0, bin_nb = 0, bin_grid = 0, bin_unroll = 8;
  bool bin_panel = true;  // gradient with r staged in LDS panels
  // panel-split gradient (sp_np > 0): rows in sp_np panels of sp_pe rows; pofs[j][P] is the
  // first entry of column j in panel P (n x (sp_np + 1) ints); sp_part holds one partial
  // dot product per (panel, drawn coordinate) (sp_np x n, dtype)
  int sp_np = 0, sp_pe = 0;
  int* d_pofs = nullptr;
  void* d_sp_part = nullptr;
  int* d_bin_cnt = nullptr;
  int* d_bin_tot = nullptr;
  int* d_bin_moved = nullptr;
  void* d_ent = nullptr;  // fold entries (row within bin, product): 8 (FP32) or 16 (FP64) bytes

  // device workspace
  int* d_bp = nullptr;
  int blk_uniform = 0;  // > 0: every block but the last has this many columns
  double* d_cn2 = nullptr;
  sca::RoundState* d_state = nullptr;
  int* d_sel_cols = nullptr;
  void* d_blk_list = nullptr;  // drawn blocks and list positions (kSelList + 1 int2)
  void* d_dx_sel = nullptr;
  int* d_chunk_cnt = nullptr;
  int* d_J_idx = nullptr;
  void* d_J_val = nullptr;
  void* d_part = nullptr;  // kMaxGroups x ldp partial sums (room for doubles)
  int64_t ldp = 0;
  double* d_r64 = nullptr;  // FP64 residual of the last fresh evaluation
  void* d_rtmp = nullptr;   // running residual of sca_solve (dtype)
  double* d_scal = nullptr; // small results
  int* d_int = nullptr;
  int obj_blocks = 256;
  double* d_obj_part = nullptr;
  int probe_waves = 0;
  double* d_wmax = nullptr;
  double* d_wsum = nullptr;
  int* d_wcnt = nullptr;

  sca_adj_cache* adj = nullptr;

  // graph of check_every rounds + objective used by sca_solve (built on first use)
  hipStream_t cap = nullptr;
  hipGraphExec_t sgraph = nullptr;
  double skey[14] = {0};

  // bounded-delay rounds: state and list of the group in flight, residual versions
  sca::RoundState* d_mbstate = nullptr;
  int* d_mbcols = nullptr;
  void* d_ring = nullptr;
  int ring_slots = 0;

  // profiling
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::vector<int> ev_kind;
  std::vector<double> ev_bytes;
  size_t ev_used = 0;
  double prof_ms[SCA_K_NKINDS] = {0, 0, 0, 0};
  int64_t prof_n[SCA_K_NKINDS] = {0, 0, 0, 0};
  double prof_bytes[SCA_K_NKINDS] = {0, 0, 0, 0};
};

namespace sca {

// lock-free rounds: most workgroups sca_opts.async_workgroups may ask for
constexpr int kAsyncMaxWorkgroups = 65536;
sca_status set_error(sca_status st, const char* fmt, ...);
sca_status validate_opts(const sca_opts* o);
sca_status dev_alloc(void** p, size_t bytes);
int device_cu_count();
sca_status validate_problem_args(sca_dtype dtype, int64_t m, int64_t n, const void* b,
                                 double lambda, double c, double beta, const int64_t* block_ptr,
                                 int64_t nblocks);
sca_status alloc_workspace(sca_problem* p, const int64_t* block_ptr);
void free_workspace(sca_problem* p);
sca_status finish_create(sca_problem* p, hipStream_t s);
sca_status report(sca_problem* p, const sca_opts* o, const void* x, double* F, double* merit,
                  double* MF, int64_t* nnz, hipStream_t s);
BRParams make_brparams(const sca_problem* p, double tau);
double gamma_at_round(double g0, double mu, long long k);
uint64_t selection_threshold(double p);
void prof_begin(sca_problem* p, hipStream_t s, int kind);
void prof_end(sca_problem* p, hipStream_t s, double bytes);
void apply_tuning(sca_problem* p);
bool batch_tuning(int dtype, int64_t mmax, sca_launch* out);  // the batch row of the table
void launch_select(sca_problem* p, const sca_opts* o, uint64_t Tthr, hipStream_t s);
void init_round_state(sca_problem* p, const sca_opts* o, int64_t round_begin, hipStream_t s);
void residual_any(sca_problem* p, const void* x, void* r_out, hipStream_t s);

void adjoint_release(sca_adj_cache* c);

// sparse (CSC) path
void launch_colnorm2_csc(sca_problem* p, hipStream_t s);
void launch_round_csc(sca_problem* p, const sca_opts* o, void* x, void* r, hipStream_t s,
                      uint64_t Tthr, const BRParams& bp);
void launch_residual_csc(sca_problem* p, const void* x, void* r_out, hipStream_t s);
void launch_probe_csc(sca_problem* p, const void* x, const BRParams& bp, hipStream_t s);
}  // namespace sca
