// Host side of libsca: argument validation, problem objects, workspace, launch
// sequences of the round, checks and the solve loop.  See include/sca.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sca.h"
#include "sca_internal.h"
#include "sca_kernels.h"

using namespace sca;

// ------------------------------------------------------------------ errors
static thread_local char g_err[512] = "";

sca_status sca::set_error(sca_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

extern "C" const char* sca_last_error(void) { return g_err; }
extern "C" const char* sca_version(void) { return "libsca 0.1 (gfx950)"; }

// ------------------------------------------------------------------ helpers
double sca::gamma_at_round(double g0, double mu, long long k) {
  double g = g0;
  for (long long i = 0; i < k; ++i) g = g * (1.0 - mu * g);
  return g;
}

uint64_t sca::selection_threshold(double p) {
  // floor(p * 2^32); p = 1 gives 2^32, i.e. every block.
  return (uint64_t)std::floor(p * 4294967296.0);
}

sca_status sca::validate_opts(const sca_opts* o) {
  if (!o) return set_error(SCA_EINVAL, "opts is NULL");
  if (o->struct_size != sizeof(sca_opts))
    return set_error(SCA_EINVAL, "opts.struct_size %zu != %zu", o->struct_size, sizeof(sca_opts));
  if (!(o->gamma > 0.0 && o->gamma <= 1.0))
    return set_error(SCA_EINVAL, "gamma must lie in (0, 1]");
  if (!(o->gamma_mu >= 0.0) || !std::isfinite(o->gamma_mu))
    return set_error(SCA_EINVAL, "gamma_mu must be finite and >= 0");
  if (!(o->tau >= 0.0) || !std::isfinite(o->tau))
    return set_error(SCA_EINVAL, "tau must be finite and >= 0");
  if (!(o->select_p > 0.0 && o->select_p <= 1.0))
    return set_error(SCA_EINVAL, "select_p must lie in (0, 1]");
  if (o->delay_chunks < 0 || o->delay_chunks > (1 << 20) || o->delay_stale < 0)
    return set_error(SCA_EINVAL, "delay_chunks must lie in [0, 2^20] and delay_stale be >= 0");
  if (o->async_workgroups < 0 || o->async_workgroups > kAsyncMaxWorkgroups)
    return set_error(SCA_EINVAL, "async_workgroups must lie in [0, %d]", kAsyncMaxWorkgroups);
  if (o->async_workgroups > 0 && o->delay_chunks > 1)
    return set_error(SCA_EINVAL, "lock-free rounds and bounded-delay rounds exclude each other");
  return SCA_OK;
}

int sca::device_cu_count() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu <= 0)
    return 256;
  return ncu;
}

sca_status sca::dev_alloc(void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return set_error(SCA_ENOMEM, "hipMalloc(%zu) failed", bytes);
  }
  return SCA_OK;
}

BRParams sca::make_brparams(const sca_problem* p, double tau) {
  BRParams bp;
  bp.tau = tau;
  bp.lam = p->lam;
  bp.lam_eta = p->lam * p->eta;
  bp.c2 = 2.0 * p->c;
  bp.beta = p->beta;
  bp.theta = p->theta;
  bp.eta = p->eta;
  bp.reg = p->reg;
  return bp;
}

// ------------------------------------------------------------------ launch shapes
static bool launch_valid(const sca_launch* l) {
  if (!l || l->struct_size != sizeof(sca_launch)) return false;
  if (l->grad_wg_per_cu < 1 || l->grad_wg_per_cu > 16) return false;
  const int c = l->grad_cols, u = l->grad_unroll;
  switch (l->grad_kind) {
    case 0:
      return u == 4 || u == 8 || u == 16;
    case 1:
      return (c == 2 && u == 4) || (c == 4 && (u == 1 || u == 2 || u == 4)) ||
             (c == 8 && (u == 1 || u == 2)) || (c == 16 && (u == 1 || u == 2));
    case 2:
      return (c == 8 && u == 2) || (c == 16 && u == 1);
    case 3:
      return (c == 4 && (u == 2 || u == 4)) || (c == 8 && u == 1);
    case 4:
      return (c == 1 || c == 2 || c == 4 || c == 8) && u == 1 && l->grad_wg_per_cu == 1;
    default:
      return false;
  }
}

// Fused round (k_grad_br_fold): q row groups of 16 bytes per thread of a 1024-thread
// workgroup hold a whole column, in registers up to the register limit (FP32: 5, m <= 20480;
// FP64: 3, m <= 6144) and beyond it in thread-private LDS slots (FP32: 4 in registers and 2
// or 3 in LDS, m <= 28672 -- 5 + 3 would spill registers; FP64: 3 + 1..3, m <= 12288); 0
// when the problem is sparse or its columns are longer.
static int fused_qmax_regs(const sca_problem* p) {
  return p->esize == 4 ? kFusedMaxQ32 : kFusedMaxQ64;
}
static int fused_q(const sca_problem* p) {
  if (p->sparse) return 0;
  const int64_t vn = 16 / (int64_t)p->esize;
  const int64_t q = ((p->m + vn - 1) / vn + 1023) / 1024;
  const int64_t qmax = p->esize == 4 ? 7 : kFusedMaxQ64 + kFusedMaxL;
  return q <= qmax ? (int)q : 0;
}

// Workgroups (= fold partials) of the fused round: one per compute unit, at most 256
// (k_part_reduce adds at most 16 partials per wave).
static int fused_groups(const sca_problem* p) { return std::max(1, std::min(p->ncu, 256)); }

// Largest column group whose registers fit (without spills) next to Q row groups of r and
// of the partial (two buffers of C columns).
static int fused_cmax(const sca_problem* p, int q) {
  if (q > fused_qmax_regs(p)) return 1;
  if (p->esize == 4) return q == 1 ? 8 : q == 2 ? 4 : q == 3 ? 2 : 1;
  return q == 1 ? 4 : q == 2 ? 2 : 1;
}

// Takes launch shape l for problem p; false when p cannot run it.
static bool take_launch(sca_problem* p, const sca_launch* l) {
  int cols = l->grad_cols;
  if (l->grad_kind == 4) {
    const int q = fused_q(p);
    if (q == 0) return false;
    cols = std::min(cols, fused_cmax(p, q));
  }
  p->grad_kind = l->grad_kind;
  p->grad_cols = cols;
  p->grad_unroll = l->grad_unroll;
  p->grad_wg_per_cu = l->grad_wg_per_cu;
  return true;
}

static std::vector<sca_tune_entry> g_tuning;

extern "C" sca_status sca_tuning_set(const sca_tune_entry* e, int64_t count) {
  if (count < 0 || (count > 0 && !e)) return set_error(SCA_EINVAL, "bad tuning table");
  for (int64_t i = 0; i < count; ++i) {
    const sca_launch& l = e[i].launch;
    const bool batch_ok = l.struct_size == sizeof(sca_launch) &&
                          (l.grad_kind == 0 ||
                           (l.grad_kind == 1 && l.grad_cols == 4 &&
                            l.grad_wg_per_cu >= 1 && l.grad_wg_per_cu <= 4));
    const bool ok_launch = e[i].target == 0 ? launch_valid(&l) : e[i].target == 1 && batch_ok;
    if (!ok_launch || e[i].m_lo > e[i].m_hi || (e[i].dtype != SCA_F32 && e[i].dtype != SCA_F64))
      return set_error(SCA_EINVAL, "tuning row %lld is invalid", (long long)i);
  }
  g_tuning.assign(e, e + count);
  return SCA_OK;
}

void sca::apply_tuning(sca_problem* p) {
  for (const sca_tune_entry& e : g_tuning) {
    if (e.target == 0 && e.dtype == p->dtype && p->m >= e.m_lo && p->m <= e.m_hi &&
        take_launch(p, &e.launch))
      return;
  }
}

bool sca::batch_tuning(int dtype, int64_t mmax, sca_launch* out) {
  for (const sca_tune_entry& e : g_tuning) {
    if (e.target == 1 && e.dtype == dtype && mmax >= e.m_lo && mmax <= e.m_hi) {
      *out = e.launch;
      return true;
    }
  }
  return false;
}

extern "C" sca_status sca_problem_get_launch(sca_problem* p, sca_launch* out) {
  if (!p || !out) return set_error(SCA_EINVAL, "NULL argument");
  out->struct_size = sizeof(sca_launch);
  out->grad_kind = p->grad_kind;
  out->grad_cols = p->grad_cols;
  out->grad_unroll = p->grad_unroll;
  out->grad_wg_per_cu = p->grad_wg_per_cu;
  return SCA_OK;
}

extern "C" sca_status sca_problem_set_launch(sca_problem* p, const sca_launch* l) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  if (!launch_valid(l) || !take_launch(p, l))
    return set_error(SCA_EINVAL, "launch shape not available for this problem");
  if (p->sgraph) {  // the solve graph bakes the launch shape in
    (void)hipGraphExecDestroy(p->sgraph);
    p->sgraph = nullptr;
  }
  return SCA_OK;
}

// ------------------------------------------------------------------ problem lifetime
sca_status sca::validate_problem_args(sca_dtype dtype, int64_t m, int64_t n, const void* b,
                                      double lambda, double c, double beta,
                                      const int64_t* block_ptr, int64_t nblocks) {
  if (dtype != SCA_F32 && dtype != SCA_F64) return set_error(SCA_EINVAL, "unknown dtype");
  if (m <= 0 || n <= 0 || m > INT32_MAX / 2 || n > INT32_MAX / 2)
    return set_error(SCA_EINVAL, "m, n must lie in [1, 2^30)");
  if (!b) return set_error(SCA_EINVAL, "b is NULL");
  if (((uintptr_t)b) % (dtype == SCA_F32 ? 4 : 8))
    return set_error(SCA_EINVAL, "b is not aligned to its element size");
  if (!(lambda >= 0.0) || !std::isfinite(lambda))
    return set_error(SCA_EINVAL, "lambda must be finite and >= 0");
  if (!(c >= 0.0) || !std::isfinite(c)) return set_error(SCA_EINVAL, "c must be finite and >= 0");
  if (!(beta > 0.0)) return set_error(SCA_EINVAL, "beta must be > 0 (INFINITY for no box)");
  if (!block_ptr || nblocks <= 0 || nblocks > n)
    return set_error(SCA_EINVAL, "block_ptr must hold nblocks+1 offsets, 1 <= nblocks <= n");
  if (block_ptr[0] != 0 || block_ptr[nblocks] != n)
    return set_error(SCA_EINVAL, "block_ptr must start at 0 and end at n");
  for (int64_t i = 0; i < nblocks; ++i)
    if (block_ptr[i + 1] <= block_ptr[i])
      return set_error(SCA_EINVAL, "block %lld is empty or block_ptr is not ascending",
                       (long long)i);
  if (c > 0.0 && !std::isfinite(beta))
    return set_error(SCA_EINVAL, "c > 0 needs a finite box bound (else F is unbounded below)");
  return SCA_OK;
}

sca_status sca::alloc_workspace(sca_problem* p, const int64_t* block_ptr) {
  const int n = (int)p->n;
  const size_t es = p->esize;
  const int nch = (n + kChunk - 1) / kChunk + 1;
  sca_status st;
#define ALLOC(ptr, bytes)                                       \
  do {                                                          \
    if ((st = dev_alloc((void**)&(ptr), (bytes))) != SCA_OK) return st; \
  } while (0)
  ALLOC(p->d_bp, sizeof(int) * (p->nblocks + 1));
  ALLOC(p->d_cn2, sizeof(double) * n);
  ALLOC(p->d_state, sizeof(RoundState));
  ALLOC(p->d_sel_cols, sizeof(int) * n);
  ALLOC(p->d_blk_list, sizeof(int2) * (kSelList + 1));
  ALLOC(p->d_dx_sel, es * n);
  ALLOC(p->d_mbstate, sizeof(RoundState));
  ALLOC(p->d_mbcols, sizeof(int) * n);
  if (hipMemset(p->d_mbstate, 0, sizeof(RoundState)) != hipSuccess)
    return set_error(SCA_EHIP, "memset of the group state failed");
  ALLOC(p->d_chunk_cnt, sizeof(int) * nch);
  ALLOC(p->d_J_idx, sizeof(int) * n);
  ALLOC(p->d_J_val, es * n);
  p->ldp = (p->m + 63) / 64 * 64;
  // fold partials: kMaxGroups column groups (FP64 room) or one per workgroup of the fused round
  ALLOC(p->d_part, p->sparse ? 64
                             : std::max(sizeof(double) * kMaxGroups, es * fused_groups(p)) *
                                   p->ldp);
  ALLOC(p->d_r64, sizeof(double) * p->ldp);
  ALLOC(p->d_rtmp, es * p->ldp);
  ALLOC(p->d_scal, sizeof(double) * 64);
  ALLOC(p->d_int, sizeof(int) * 64);
  p->obj_blocks = 256;
  ALLOC(p->d_obj_part, sizeof(double) * 3 * p->obj_blocks);
  p->probe_waves = 4 * 4 * p->ncu;
  ALLOC(p->d_wmax, sizeof(double) * p->probe_waves);
  ALLOC(p->d_wsum, sizeof(double) * p->probe_waves);
  ALLOC(p->d_wcnt, sizeof(int) * p->probe_waves);
#undef ALLOC
  std::vector<int> bp32(p->nblocks + 1);
  for (int64_t i = 0; i <= p->nblocks; ++i) bp32[i] = (int)block_ptr[i];
  if (hipMemcpy(p->d_bp, bp32.data(), sizeof(int) * bp32.size(), hipMemcpyHostToDevice) !=
      hipSuccess)
    return set_error(SCA_EHIP, "copy of block_ptr failed");
  p->block_ptr_host.assign(block_ptr, block_ptr + p->nblocks + 1);
  // equal blocks (the last one possibly shorter): the in-kernel draws compute the block
  // bounds instead of loading them
  {
    const int64_t B = p->nblocks > 0 ? block_ptr[1] - block_ptr[0] : 0;
    bool uni = B > 0 && block_ptr[0] == 0;
    for (int64_t i = 0; uni && i < p->nblocks; ++i)
      uni = block_ptr[i] == i * B && (i + 1 < p->nblocks ? block_ptr[i + 1] == (i + 1) * B
                                                          : block_ptr[i + 1] - block_ptr[i] <= B);
    p->blk_uniform = uni && B <= INT32_MAX ? (int)B : 0;
  }
  return SCA_OK;
}

void sca::free_workspace(sca_problem* p) {
  void* ptrs[] = {p->d_bp, p->d_cn2, p->d_state, p->d_mbstate, p->d_mbcols, p->d_ring,
                  p->d_blk_list,
                  p->d_sel_cols, p->d_dx_sel, p->d_chunk_cnt,
                  p->d_J_idx, p->d_J_val, p->d_part, p->d_r64, p->d_rtmp, p->d_scal,
                  p->d_int, p->d_obj_part, p->d_wmax, p->d_wsum, p->d_wcnt,
                  p->csc_colptr, p->csc_rowidx, p->csc_vals, p->d_bin_cnt, p->d_bin_tot,
                  p->d_bin_moved, p->d_ent, p->d_pofs, p->d_sp_part};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  adjoint_release(p->adj);
  p->adj = nullptr;
  if (p->sgraph) (void)hipGraphExecDestroy(p->sgraph);
  p->sgraph = nullptr;
  if (p->cap) (void)hipStreamDestroy(p->cap);
  p->cap = nullptr;
  for (auto& e : p->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p->events.clear();
}

// Column norms, minimum column norm and a finite check of b; synchronises once.
sca_status sca::finish_create(sca_problem* p, hipStream_t s) {
  init_round_state(p, nullptr, 0, s);
  if (p->sparse) {
    launch_colnorm2_csc(p, s);
  } else if (p->dtype == SCA_F32) {
    hipLaunchKernelGGL(k_colnorm2<float>, dim3(4 * p->ncu), dim3(256), 0, s,
                       (const float*)p->A, (long long)p->lda, (int)p->m, (int)p->n, p->d_cn2);
  } else {
    hipLaunchKernelGGL(k_colnorm2<double>, dim3(4 * p->ncu), dim3(256), 0, s,
                       (const double*)p->A, (long long)p->lda, (int)p->m, (int)p->n, p->d_cn2);
  }
  if (hipMemsetAsync(p->d_int, 0, sizeof(int), s) != hipSuccess)
    return set_error(SCA_EHIP, "memset failed");
  if (p->dtype == SCA_F32)
    hipLaunchKernelGGL(k_count_nonfinite<float>, dim3(64), dim3(256), 0, s, (const float*)p->b,
                       (long long)p->m, p->d_int);
  else
    hipLaunchKernelGGL(k_count_nonfinite<double>, dim3(64), dim3(256), 0, s, (const double*)p->b,
                       (long long)p->m, p->d_int);
  std::vector<double> cn2(p->n);
  int bad = 0;
  if (hipMemcpyAsync(cn2.data(), p->d_cn2, sizeof(double) * p->n, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(&bad, p->d_int, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "set-up kernels failed: %s", hipGetErrorString(hipGetLastError()));
  if (bad) return set_error(SCA_EINVAL, "b holds NaN or Inf");
  double mn = INFINITY;
  for (double v : cn2) {
    if (!std::isfinite(v)) return set_error(SCA_EINVAL, "A holds NaN or Inf");
    mn = std::min(mn, v);
  }
  p->cn2_min = mn;
  return SCA_OK;
}

extern "C" sca_status sca_problem_create_dense(sca_problem** out, sca_dtype dtype, int64_t m,
                                               int64_t n, const void* A, int64_t lda,
                                               const void* b, double lambda, double c,
                                               double beta, const int64_t* block_ptr,
                                               int64_t nblocks, void* stream) {
  if (!out) return set_error(SCA_EINVAL, "out is NULL");
  *out = nullptr;
  sca_status st = validate_problem_args(dtype, m, n, b, lambda, c, beta, block_ptr, nblocks);
  if (st != SCA_OK) return st;
  const size_t es = dtype == SCA_F32 ? 4 : 8;
  if (!A) return set_error(SCA_EINVAL, "A is NULL");
  if (((uintptr_t)A) % 16) return set_error(SCA_EINVAL, "A must be 16-byte aligned");
  if (lda < m || (lda * (int64_t)es) % 16)
    return set_error(SCA_EINVAL, "lda must be >= m and lda*sizeof(element) a multiple of 16");
  sca_problem* p = new (std::nothrow) sca_problem();
  if (!p) return set_error(SCA_ENOMEM, "host allocation failed");
  p->dtype = dtype;
  p->esize = es;
  p->m = m;
  p->n = n;
  p->lda = lda;
  p->A = A;
  p->b = b;
  p->lam = lambda;
  p->c = c;
  p->beta = beta;
  p->nblocks = nblocks;
  p->ncu = device_cu_count();
  apply_tuning(p);
  if ((st = alloc_workspace(p, block_ptr)) != SCA_OK ||
      (st = finish_create(p, (hipStream_t)stream)) != SCA_OK) {
    free_workspace(p);
    delete p;
    return st;
  }
  *out = p;
  return SCA_OK;
}

extern "C" sca_status sca_problem_set_regularizer(sca_problem* p, sca_reg reg, double theta) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  if (reg == SCA_REG_L1) {
    p->reg = 0;
    p->theta = 0.0;
    p->eta = 1.0;
    return SCA_OK;
  }
  if (reg != SCA_REG_EXP && reg != SCA_REG_LOG) return set_error(SCA_EINVAL, "unknown regulariser");
  if (!(theta > 0.0) || !std::isfinite(theta)) return set_error(SCA_EINVAL, "theta must be > 0");
  p->reg = (int)reg;
  p->theta = theta;  // (the solve graph compares its baked-in parameters before reuse)
  p->eta = reg == SCA_REG_EXP ? theta : theta / std::log1p(theta);
  return SCA_OK;
}

extern "C" sca_status sca_problem_update_rhs(sca_problem* p, const void* b, double lambda,
                                             void* stream) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  if (!b || ((uintptr_t)b) % p->esize) return set_error(SCA_EINVAL, "b is NULL or misaligned");
  if (!(lambda >= 0.0) || !std::isfinite(lambda))
    return set_error(SCA_EINVAL, "lambda must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  if (hipMemsetAsync(p->d_int, 0, sizeof(int), s) != hipSuccess)
    return set_error(SCA_EHIP, "memset failed");
  if (p->dtype == SCA_F32)
    hipLaunchKernelGGL(k_count_nonfinite<float>, dim3(64), dim3(256), 0, s, (const float*)b,
                       (long long)p->m, p->d_int);
  else
    hipLaunchKernelGGL(k_count_nonfinite<double>, dim3(64), dim3(256), 0, s, (const double*)b,
                       (long long)p->m, p->d_int);
  int bad = 0;
  if (hipMemcpyAsync(&bad, p->d_int, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "finite check failed");
  if (bad) return set_error(SCA_EINVAL, "b holds NaN or Inf");
  p->b = b;
  p->lam = lambda;
  return SCA_OK;
}

extern "C" void sca_problem_destroy(sca_problem* p) {
  if (!p) return;
  free_workspace(p);
  delete p;
}

// ------------------------------------------------------------------ profiling
void sca::prof_begin(sca_problem* p, hipStream_t s, int kind) {
  if (!p->profiling) return;
  if (p->ev_used >= p->events.size()) {
    std::pair<hipEvent_t, hipEvent_t> e;
    (void)hipEventCreate(&e.first);
    (void)hipEventCreate(&e.second);
    p->events.push_back(e);
  }
  p->ev_kind.resize(p->events.size());
  p->ev_kind[p->ev_used] = kind;
  (void)hipEventRecord(p->events[p->ev_used].first, s);
}

void sca::prof_end(sca_problem* p, hipStream_t s, double bytes) {
  if (!p->profiling) return;
  p->ev_bytes.resize(p->events.size());
  p->ev_bytes[p->ev_used] = bytes;
  (void)hipEventRecord(p->events[p->ev_used].second, s);
  ++p->ev_used;
}

static void prof_collect(sca_problem* p) {
  if (!p->profiling || p->ev_used == 0) return;
  (void)hipEventSynchronize(p->events[p->ev_used - 1].second);
  for (size_t i = 0; i < p->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->events[i].first, p->events[i].second) == hipSuccess) {
      p->prof_ms[p->ev_kind[i]] += ms;
      p->prof_n[p->ev_kind[i]] += 1;
      p->prof_bytes[p->ev_kind[i]] += p->ev_bytes[i];
    }
  }
  p->ev_used = 0;
}

extern "C" sca_status sca_profile_get(sca_problem* p, double* ms, int64_t* launches,
                                      double* bytes, int reset) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  for (int k = 0; k < SCA_K_NKINDS; ++k) {
    if (ms) ms[k] = p->prof_ms[k];
    if (launches) launches[k] = p->prof_n[k];
    if (bytes) bytes[k] = p->prof_bytes[k];
    if (reset) {
      p->prof_ms[k] = 0;
      p->prof_n[k] = 0;
      p->prof_bytes[k] = 0;
    }
  }
  return SCA_OK;
}

// ------------------------------------------------------------------ launch sequences
// S.1: the block draw of the round in flight (see k_select).
// When many columns are expected per round the single-workgroup draw only lists the drawn
// blocks and k_select_expand writes their columns with the whole grid.
void sca::launch_select(sca_problem* p, const sca_opts* o, uint64_t Tthr, hipStream_t s) {
  const double expect = std::min(1.0, o->select_p) * (double)p->n;
  int2* blk = expect >= (double)kSelExpandCols ? (int2*)p->d_blk_list : nullptr;
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, (int)p->nblocks, p->d_bp, o->seed,
                     o->instance, Tthr, p->d_state, p->d_sel_cols, blk);
  if (blk) {
    const int g = std::max(1, std::min(p->ncu, (int)((p->nblocks + 3) / 4)));
    hipLaunchKernelGGL(k_select_expand, dim3(g), dim3(256), 0, s, (const int2*)blk, p->d_bp,
                       p->d_sel_cols);
  }
}

// S.2-S.4 on the coordinates listed in 'list' (count and step in *st), reading r.
template <typename T>
static void grad_dense(sca_problem* p, T* x, const T* r, RoundState* st, const int* list,
                       const BRParams& bp, hipStream_t s) {
  const int m = (int)p->m;
  const dim3 ggrid(p->ncu * p->grad_wg_per_cu);
#define GRAD_LAUNCH(UU)                                                                     \
  hipLaunchKernelGGL((k_grad_br<T, UU>), ggrid, dim3(256), 0, s, (const T*)p->A,           \
                     (long long)p->lda, m, r, x, p->d_cn2, list, st, (T*)p->d_dx_sel, bp)
#define GRAD_WG_LAUNCH_NT(CC, UU, NTT)                                                      \
  hipLaunchKernelGGL((k_grad_br_wg<T, CC, UU, NTT>), ggrid, dim3(256), 0, s, (const T*)p->A, \
                     (long long)p->lda, m, r, x, p->d_cn2, list, st, (T*)p->d_dx_sel, bp)
#define GRAD_WG_LAUNCH(CC, UU)                                                              \
  hipLaunchKernelGGL((k_grad_br_wg<T, CC, UU>), ggrid, dim3(256), 0, s, (const T*)p->A,      \
                     (long long)p->lda, m, r, x, p->d_cn2, list, st, (T*)p->d_dx_sel, bp)
#define GRAD_WW_LAUNCH(CC, UU)                                                              \
  hipLaunchKernelGGL((k_grad_br_wwalk<T, CC, UU>), ggrid, dim3(256), 0, s, (const T*)p->A,   \
                     (long long)p->lda, m, r, x, p->d_cn2, list, st, (T*)p->d_dx_sel, bp)
  if (p->grad_kind == 4) {  // (fused problems run k_grad_br_fold; kept as a safe default)
    GRAD_WG_LAUNCH(4, 4);
  } else if (p->grad_kind == 3) {  // one wave per group of columns
    if (p->grad_cols == 4 && p->grad_unroll == 2)
      GRAD_WW_LAUNCH(4, 2);
    else if (p->grad_cols == 8 && p->grad_unroll == 1)
      GRAD_WW_LAUNCH(8, 1);
    else
      GRAD_WW_LAUNCH(4, 4);
  } else if (p->grad_kind == 2) {  // ordinary (temporal) loads
    if (p->grad_cols == 16)
      GRAD_WG_LAUNCH_NT(16, 1, false);
    else
      GRAD_WG_LAUNCH_NT(8, 2, false);
  } else if (p->grad_kind == 1 && p->grad_cols == 16) {
    if (p->grad_unroll == 2)
      GRAD_WG_LAUNCH_NT(16, 2, true);
    else
      GRAD_WG_LAUNCH_NT(16, 1, true);
  } else if (p->grad_kind == 1) {
    if (p->grad_cols == 2 && p->grad_unroll == 4)
      GRAD_WG_LAUNCH(2, 4);
    else if (p->grad_cols == 4 && p->grad_unroll == 4)
      GRAD_WG_LAUNCH(4, 4);
    else if (p->grad_cols == 8 && p->grad_unroll == 2)
      GRAD_WG_LAUNCH(8, 2);
    else if (p->grad_cols == 8 && p->grad_unroll == 1)
      GRAD_WG_LAUNCH(8, 1);
    else if (p->grad_cols == 4 && p->grad_unroll == 1)
      GRAD_WG_LAUNCH(4, 1);
    else
      GRAD_WG_LAUNCH(4, 2);
  } else if (p->grad_unroll == 4) {
    GRAD_LAUNCH(4);
  } else if (p->grad_unroll == 16) {
    GRAD_LAUNCH(16);
  } else {
    GRAD_LAUNCH(8);
  }
#undef GRAD_LAUNCH
#undef GRAD_WG_LAUNCH
#undef GRAD_WG_LAUNCH_NT
#undef GRAD_WW_LAUNCH
}

// S.5: ordered list of the moved coordinates of 'list' (count in *st), then
// out = base + sum of their columns times their moves (out may alias base).
template <typename T>
static void fold_dense(sca_problem* p, RoundState* st, const int* list, const T* base, T* out,
                       hipStream_t s) {
  const int m = (int)p->m, n = (int)p->n;
  prof_begin(p, s, SCA_K_COMPACT);
  const int nch = (n + kChunk - 1) / kChunk;
  const int cgrid = std::max(1, std::min(nch, 2 * p->ncu));
  int* S_ptr = (int*)((char*)st + offsetof(RoundState, S_cnt));
  hipLaunchKernelGGL(k_compact_count<T>, dim3(cgrid), dim3(1024), 0, s, (const T*)p->d_dx_sel,
                     (const int*)S_ptr, p->d_chunk_cnt);
  hipLaunchKernelGGL(k_compact_scatter<T>, dim3(cgrid), dim3(1024), 0, s,
                     (const T*)p->d_dx_sel, list, (const int*)S_ptr, (const int*)p->d_chunk_cnt,
                     p->d_J_idx, (T*)p->d_J_val, st, 1);
  prof_end(p, s, 0.0);
  prof_begin(p, s, SCA_K_FOLD);
  constexpr int VN = V16<T>::N;
  const int nrt = (m + 256 * VN - 1) / (256 * VN);
  const int fgrid = std::max(1, std::min(nrt * kMaxGroups, 8 * p->ncu));
  hipLaunchKernelGGL((k_fold_partial<T, T>), dim3(fgrid), dim3(256), 0, s, (const T*)p->A,
                     (long long)p->lda, m, (const int*)p->d_J_idx, (const T*)p->d_J_val,
                     (const RoundState*)st, (T*)p->d_part, (long long)p->ldp);
  hipLaunchKernelGGL((k_fold_reduce<T, T, T>), dim3((m + 255) / 256), dim3(256), 0, s, base, 1.0,
                     (const T*)p->d_part, (long long)p->ldp, (const RoundState*)st, m, out,
                     (double*)nullptr);
  prof_end(p, s, 0.0);
}

// The fused round draws the blocks itself when every thread of a workgroup handles at most
// 32 blocks and a workgroup's share of the drawn list fits its LDS list.
static bool fused_draws(const sca_problem* p) {
  const int64_t G = fused_groups(p);
  const int64_t cap = fused_q(p) > fused_qmax_regs(p) ? kFusedSelColsL : kFusedSelCols;
  return p->nblocks <= kFusedSelBlocks && (p->n + G - 1) / G <= cap;
}

// S.1-S.5 fused (k_grad_br_fold, one workgroup per compute unit, S.1 inside when
// fs.on) on the coordinates listed in 'list' (count and step in *st) with the gradient from
// r_read, then out = base + the partials (and the round state advanced when S.1 ran inside).
template <typename T>
static void grad_fold_dense(sca_problem* p, T* x, const T* r_read, const T* base, T* out,
                            RoundState* st, const int* list, const BRParams& bp,
                            const FusedSel& fs, hipStream_t s) {
  const int m = (int)p->m, G = fused_groups(p);
  const int q = fused_q(p), c = p->grad_cols;
  prof_begin(p, s, SCA_K_GRAD);
#define FUSED(QQ, CC)                                                                       \
  hipLaunchKernelGGL((k_grad_br_fold<T, QQ, CC>), dim3(G), dim3(1024), 0, s, (const T*)p->A, \
                     (long long)p->lda, m, r_read, x, p->d_cn2, list, st, (T*)p->d_part,      \
                     (long long)p->ldp, bp, fs)
#define FUSED_L(QQ, LL)                                                                     \
  hipLaunchKernelGGL((k_grad_br_fold<T, QQ, 1, LL>), dim3(G), dim3(1024), 0, s,             \
                     (const T*)p->A, (long long)p->lda, m, r_read, x, p->d_cn2, list, st,     \
                     (T*)p->d_part, (long long)p->ldp, bp, fs)
  if constexpr (sizeof(T) == 4) {
    if (q > kFusedMaxQ32) {  // 4 row groups in registers, the rest in LDS
      if (q == 6)
        FUSED_L(4, 2);
      else
        FUSED_L(4, 3);
    } else {
    switch (q * 16 + c) {
      case 16 + 8: FUSED(1, 8); break;
      case 16 + 4: FUSED(1, 4); break;
      case 16 + 2: FUSED(1, 2); break;
      case 16 + 1: FUSED(1, 1); break;
      case 32 + 4: FUSED(2, 4); break;
      case 32 + 2: FUSED(2, 2); break;
      case 32 + 1: FUSED(2, 1); break;
      case 48 + 2: FUSED(3, 2); break;
      case 48 + 1: FUSED(3, 1); break;
      case 64 + 1: FUSED(4, 1); break;
      default: FUSED(5, 1); break;
    }
    }
  } else {
    if (q > kFusedMaxQ64) {
      if (q == kFusedMaxQ64 + 1)
        FUSED_L(kFusedMaxQ64, 1);
      else if (q == kFusedMaxQ64 + 2)
        FUSED_L(kFusedMaxQ64, 2);
      else
        FUSED_L(kFusedMaxQ64, 3);
    } else {
    switch (q * 16 + c) {
      case 16 + 4: FUSED(1, 4); break;
      case 16 + 2: FUSED(1, 2); break;
      case 16 + 1: FUSED(1, 1); break;
      case 32 + 2: FUSED(2, 2); break;
      case 32 + 1: FUSED(2, 1); break;
      default: FUSED(3, 1); break;
    }
    }
  }
#undef FUSED
#undef FUSED_L
  prof_end(p, s, 0.0);
  prof_begin(p, s, SCA_K_FOLD);
  constexpr int VN = V16<T>::N;
  const int nq = (m + VN - 1) / VN;
  hipLaunchKernelGGL(k_part_reduce<T>, dim3((nq + kPartRows - 1) / kPartRows), dim3(256), 0, s,
                     (const T*)p->d_part, (long long)p->ldp, G, m, base, out, st, fs.on);
  prof_end(p, s, 0.0);
}

template <typename T>
static void launch_round_dense(sca_problem* p, const sca_opts* o, T* x, T* r, hipStream_t s,
                               uint64_t Tthr, const BRParams& bp) {
  FusedSel fs{p->d_bp,   (int)p->nblocks, 0, o->seed, Tthr, o->instance, p->blk_uniform,
              (int)p->n};
  if (p->grad_kind == 4 && fused_draws(p)) {
    fs.on = 1;
    grad_fold_dense<T>(p, x, r, r, r, p->d_state, p->d_sel_cols, bp, fs, s);
    return;
  }
  prof_begin(p, s, SCA_K_SELECT);
  launch_select(p, o, Tthr, s);
  prof_end(p, s, 0.0);
  if (p->grad_kind == 4) {
    grad_fold_dense<T>(p, x, r, r, r, p->d_state, p->d_sel_cols, bp, fs, s);
    return;
  }
  prof_begin(p, s, SCA_K_GRAD);
  grad_dense<T>(p, x, r, p->d_state, p->d_sel_cols, bp, s);
  prof_end(p, s, 0.0);
  fold_dense<T>(p, p->d_state, p->d_sel_cols, r, r, s);
}

// ------------------------------------------------------------------ bounded-delay rounds
// Group t of q: the drawn coordinates [t*per, min(S, (t+1)*per)), per = ceil(S/q), listed
// in mb_cols with their count and the round's step in *mb.
static __global__ void __launch_bounds__(1024)
k_mb_window(const RoundState* __restrict__ st, int t, int q, const int* __restrict__ sel,
            RoundState* __restrict__ mb, int* __restrict__ mb_cols) {
  const int S = st->S_cnt;
  const int per = (int)(((long long)S + q - 1) / q);
  const int lo = (int)min((long long)S, (long long)t * per);
  const int hi = min(S, lo + per);
  for (int i = lo + (int)threadIdx.x; i < hi; i += 1024) mb_cols[i - lo] = sel[i];
  if (threadIdx.x == 0) {
    mb->S_cnt = hi - lo;
    mb->work_ctr = 0;
    mb->gamma_cur = st->gamma_cur;
    mb->k = st->k;
    mb->J_cnt = 0;
    mb->G = 1;
    mb->ngroups = 0;
  }
}

static __global__ void k_mb_finish(RoundState* __restrict__ st, RoundState* __restrict__ mb) {
  st->moved_updates += mb->moved_updates;
  mb->moved_updates = 0;
}

template <typename T>
static __global__ void k_copy_vec(const T* __restrict__ src, T* __restrict__ dst, int m) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    dst[i] = src[i];
}

static sca_status ensure_ring(sca_problem* p, int slots) {
  if (p->ring_slots >= slots) return SCA_OK;
  if (p->d_ring) (void)hipFree(p->d_ring);
  p->d_ring = nullptr;
  p->ring_slots = 0;
  sca_status st = dev_alloc(&p->d_ring, p->esize * (size_t)p->ldp * slots);
  if (st != SCA_OK) return st;
  p->ring_slots = slots;
  return SCA_OK;
}

static int ring_slots_for(const sca_opts* o) {
  const int64_t q = o->delay_chunks;
  return (int)std::min<int64_t>(o->delay_stale, q) + 2;
}

template <typename T>
static void launch_round_delayed(sca_problem* p, const sca_opts* o, T* x, T* r, hipStream_t s,
                                 uint64_t Tthr, const BRParams& bp) {
  const int m = (int)p->m;
  const int q = (int)o->delay_chunks;
  const int R = ring_slots_for(o);
  const int64_t stale = o->delay_stale;
  T* ring = (T*)p->d_ring;
  auto slot = [&](int64_t v) { return ring + (size_t)(v % R) * p->ldp; };
  const dim3 vgrid((unsigned)std::max(1, std::min((m + 255) / 256, 4 * p->ncu)));
  prof_begin(p, s, SCA_K_SELECT);
  launch_select(p, o, Tthr, s);
  prof_end(p, s, 0.0);
  hipLaunchKernelGGL(k_copy_vec<T>, vgrid, dim3(256), 0, s, (const T*)r, slot(0), m);
  for (int t = 0; t < q; ++t) {
    hipLaunchKernelGGL(k_mb_window, dim3(1), dim3(1024), 0, s, (const RoundState*)p->d_state, t,
                       q, (const int*)p->d_sel_cols, p->d_mbstate, p->d_mbcols);
    const T* stale_r = slot(std::max<int64_t>(0, t - stale));
    if (p->grad_kind == 4) {  // the group's S.2-S.5 fused, read from the stale version
      const FusedSel off{p->d_bp, (int)p->nblocks, 0, o->seed, Tthr, o->instance, 0, 0};
      grad_fold_dense<T>(p, x, stale_r, slot(t), slot(t + 1), p->d_mbstate, p->d_mbcols, bp,
                         off, s);
      continue;
    }
    prof_begin(p, s, SCA_K_GRAD);
    grad_dense<T>(p, x, stale_r, p->d_mbstate, p->d_mbcols, bp, s);
    prof_end(p, s, 0.0);
    fold_dense<T>(p, p->d_mbstate, p->d_mbcols, slot(t), slot(t + 1), s);
  }
  hipLaunchKernelGGL(k_copy_vec<T>, vgrid, dim3(256), 0, s, (const T*)slot(q), r, m);
  hipLaunchKernelGGL(k_mb_finish, dim3(1), dim3(1), 0, s, p->d_state, p->d_mbstate);
}

// ------------------------------------------------------------------ lock-free rounds
// Asynchronous rounds with real races (Algorithm 1 with the delays of Assumption D1 left to
// the hardware): after the draw, W workgroups take the round's drawn coordinates one at a
// time from the round's work counter.  For coordinate j a workgroup reads a_j and the
// residual r as it stands in memory (relaxed agent-scope loads, so every read sees the
// folds that have reached the L2 by then, and misses those of the at most W - 1 coordinates
// in flight on other workgroups), forms the partial gradient, the best response and the
// step (S.2-S.4; x_j is its own: D4) and folds d * a_j into r with one atomic add per row
// (S.5).  Nondeterministic for W > 1 (the order of the atomic adds and of the reads); W = 1
// is a sequential sweep over the drawn coordinates in ascending order.
template <typename T>
__global__ void __launch_bounds__(256)
k_async_round(const T* __restrict__ A, long long lda, int m, T* r, T* __restrict__ x,
              const double* __restrict__ cn2, const int* __restrict__ sel_cols,
              RoundState* __restrict__ st, BRParams bp) {
  __shared__ int s_t;
  __shared__ T s_red[4];
  __shared__ T s_d;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int S = st->S_cnt;
  const T gamma = (T)st->gamma_cur;
  long long moved = 0;
  for (;;) {
    if (threadIdx.x == 0) s_t = atomicAdd(&st->work_ctr, 1);
    __syncthreads();
    const int t = s_t;
    if (t >= S) break;
    const int j = sel_cols[t];
    const T* a = A + (size_t)j * lda;
    T acc = (T)0;
    for (int i = threadIdx.x; i < m; i += 256)
      acc += a[i] * __hip_atomic_load(&r[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    acc = wave_sum(acc);
    if (lane == 0) s_red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      const T dot = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
      const T xj = x[j];
      T g = dot - (T)bp.c2 * xj;
      if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
      const T q = (T)(cn2[j] + bp.tau);
      const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
      const T d = gamma * (xh - xj);
      x[j] = xj + d;
      s_d = d;
      moved += d != (T)0;
    }
    __syncthreads();
    const T d = s_d;
    if (d != (T)0)
      for (int i = threadIdx.x; i < m; i += 256) unsafeAtomicAdd(&r[i], a[i] * d);
    __threadfence();  // this coordinate's folds are in memory before the next one's reads
    __syncthreads();  // s_t, s_red and s_d are written again by the next coordinate
  }
  if (threadIdx.x == 0 && moved)
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->moved_updates),
              (unsigned long long)moved);
}

template <typename T>
static void launch_round_async(sca_problem* p, const sca_opts* o, T* x, T* r, hipStream_t s,
                               uint64_t Tthr, const BRParams& bp) {
  prof_begin(p, s, SCA_K_SELECT);
  launch_select(p, o, Tthr, s);  // also resets the work counter
  prof_end(p, s, 0.0);
  prof_begin(p, s, SCA_K_GRAD);
  hipLaunchKernelGGL(k_async_round<T>, dim3((unsigned)o->async_workgroups), dim3(256), 0, s,
                     (const T*)p->A, (long long)p->lda, (int)p->m, r, x,
                     (const double*)p->d_cn2, (const int*)p->d_sel_cols, p->d_state, bp);
  prof_end(p, s, 0.0);
}

// Fresh residual with FP64 accumulation: r64 = A x - b (and r_out in the dtype if given).
template <typename T>
static void launch_residual_dense(sca_problem* p, const T* x, T* r_out, hipStream_t s) {
  const int m = (int)p->m, n = (int)p->n;
  int* N_ptr = (int*)((char*)p->d_state + offsetof(RoundState, n_all));
  const int nch = (n + kChunk - 1) / kChunk;
  const int cgrid = std::max(1, std::min(nch, 2 * p->ncu));
  hipLaunchKernelGGL(k_compact_count<T>, dim3(cgrid), dim3(1024), 0, s, x, (const int*)N_ptr,
                     p->d_chunk_cnt);
  hipLaunchKernelGGL(k_compact_scatter<T>, dim3(cgrid), dim3(1024), 0, s, x, (const int*)nullptr,
                     (const int*)N_ptr, (const int*)p->d_chunk_cnt, p->d_J_idx, (T*)p->d_J_val,
                     p->d_state, 0);
  constexpr int VN = V16<T>::N;
  const int nrt = (m + 256 * VN - 1) / (256 * VN);
  const int fgrid = std::max(1, std::min(nrt * kMaxGroups, 8 * p->ncu));
  hipLaunchKernelGGL((k_fold_partial<T, double>), dim3(fgrid), dim3(256), 0, s, (const T*)p->A,
                     (long long)p->lda, m, (const int*)p->d_J_idx, (const T*)p->d_J_val,
                     (const RoundState*)p->d_state, (double*)p->d_part, (long long)p->ldp);
  hipLaunchKernelGGL((k_fold_reduce<T, double, T>), dim3((m + 255) / 256), dim3(256), 0, s,
                     (const T*)p->b, -1.0, (const double*)p->d_part, (long long)p->ldp,
                     (const RoundState*)p->d_state, m, r_out, p->d_r64);
}

template <typename T>
static void launch_objective(sca_problem* p, const T* x, const void* r, bool r_is64,
                             const BRParams& bp, double* out_dev, hipStream_t s) {
  if (r_is64)
    hipLaunchKernelGGL((k_obj_partial<T, double>), dim3(p->obj_blocks), dim3(256), 0, s,
                       (const double*)r, (int)p->m, x, (int)p->n, bp, p->d_obj_part);
  else
    hipLaunchKernelGGL((k_obj_partial<T, T>), dim3(p->obj_blocks), dim3(256), 0, s,
                       (const T*)r, (int)p->m, x, (int)p->n, bp, p->d_obj_part);
  hipLaunchKernelGGL(k_obj_final, dim3(1), dim3(256), 0, s, (const double*)p->d_obj_part,
                     p->obj_blocks, p->c, p->lam, out_dev);
}

template <typename T>
static void launch_probe(sca_problem* p, const T* x, const BRParams& bp, double* out_dev,
                         hipStream_t s) {
  if (p->sparse) {
    launch_probe_csc(p, (const void*)x, bp, s);
  } else {
    hipLaunchKernelGGL((k_probe<T>), dim3(p->probe_waves / 4), dim3(256), 0, s, (const T*)p->A,
                       (long long)p->lda, (int)p->m, (const double*)p->d_r64, x, (int)p->n,
                       (const double*)p->d_cn2, bp, p->d_wmax, p->d_wsum, p->d_wcnt);
  }
  hipLaunchKernelGGL(k_probe_final, dim3(1), dim3(256), 0, s, (const double*)p->d_wmax,
                     (const double*)p->d_wsum, (const int*)p->d_wcnt, p->probe_waves, out_dev);
}

// ------------------------------------------------------------------ dispatch helpers
template <typename T>
static void run_rounds_t(sca_problem* p, const sca_opts* o, int64_t nrounds, T* x, T* r,
                         hipStream_t s) {
  const uint64_t Tthr = selection_threshold(o->select_p);
  const BRParams bp = make_brparams(p, o->tau);
  const bool delayed = o->delay_chunks > 1 && o->delay_stale < o->delay_chunks - 1;
  for (int64_t i = 0; i < nrounds; ++i) {
    if (p->sparse)
      launch_round_csc(p, o, (void*)x, (void*)r, s, Tthr, bp);
    else if (o->async_workgroups > 0)
      launch_round_async<T>(p, o, x, r, s, Tthr, bp);
    else if (delayed)
      launch_round_delayed<T>(p, o, x, r, s, Tthr, bp);
    else
      launch_round_dense<T>(p, o, x, r, s, Tthr, bp);
  }
}

void sca::residual_any(sca_problem* p, const void* x, void* r_out, hipStream_t s) {
  if (p->sparse) {
    launch_residual_csc(p, x, r_out, s);
  } else if (p->dtype == SCA_F32) {
    launch_residual_dense<float>(p, (const float*)x, (float*)r_out, s);
  } else {
    launch_residual_dense<double>(p, (const double*)x, (double*)r_out, s);
  }
}

static void objective_any(sca_problem* p, const void* x, const void* r, bool r_is64,
                          const BRParams& bp, double* out_dev, hipStream_t s) {
  if (p->dtype == SCA_F32)
    launch_objective<float>(p, (const float*)x, r, r_is64, bp, out_dev, s);
  else
    launch_objective<double>(p, (const double*)x, r, r_is64, bp, out_dev, s);
}

static void probe_any(sca_problem* p, const void* x, const BRParams& bp, double* out_dev,
                      hipStream_t s) {
  if (p->dtype == SCA_F32)
    launch_probe<float>(p, (const float*)x, bp, out_dev, s);
  else
    launch_probe<double>(p, (const double*)x, bp, out_dev, s);
}

static sca_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(SCA_EHIP, "%s: %s", what, hipGetErrorString(e));
  return SCA_OK;
}

static sca_status check_tau(const sca_problem* p, double tau) {
  if (!(p->cn2_min + tau > 0.0))
    return set_error(SCA_EINVAL, "a column of A is zero and tau = 0: q_j = 0");
  return SCA_OK;
}

// Round counter and step of round_begin; clears the coordinate-update counter.
void sca::init_round_state(sca_problem* p, const sca_opts* o, int64_t round_begin, hipStream_t s) {
  const double g = o ? gamma_at_round(o->gamma, o->gamma_mu, round_begin) : 1.0;
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, p->d_state, (long long)round_begin,
                     g, o ? o->gamma_mu : 0.0, (int)p->n, 1);
}

// ------------------------------------------------------------------ public entry points
// Bounded-delay rounds: dense problems only; their residual versions are allocated here
// (outside any graph capture).
static sca_status prepare_delay(sca_problem* p, const sca_opts* o) {
  if (o->async_workgroups > 0 && p->sparse)
    return set_error(SCA_EINVAL, "lock-free rounds need a dense problem");
  if (o->delay_chunks <= 1) return SCA_OK;
  if (p->sparse) return set_error(SCA_EINVAL, "bounded-delay rounds need a dense problem");
  return ensure_ring(p, ring_slots_for(o));
}

extern "C" sca_status sca_step(sca_problem* p, const sca_opts* o, int64_t round_begin,
                               int64_t nrounds, void* x, void* r, void* stream) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if ((st = check_tau(p, o->tau)) != SCA_OK) return st;
  if ((st = prepare_delay(p, o)) != SCA_OK) return st;
  if (round_begin < 0 || nrounds < 0) return set_error(SCA_EINVAL, "negative round range");
  if (!x || !r) return set_error(SCA_EINVAL, "x or r is NULL");
  if (((uintptr_t)r) % 16) return set_error(SCA_EINVAL, "r must be 16-byte aligned");
  if (((uintptr_t)x) % p->esize) return set_error(SCA_EINVAL, "x is misaligned");
  hipStream_t s = (hipStream_t)stream;
  p->profiling = (o->flags & SCA_FLAG_PROFILE) != 0;
  init_round_state(p, o, round_begin, s);
  if (p->dtype == SCA_F32)
    run_rounds_t<float>(p, o, nrounds, (float*)x, (float*)r, s);
  else
    run_rounds_t<double>(p, o, nrounds, (double*)x, (double*)r, s);
  st = check_launch("sca_step");
  prof_collect(p);
  p->profiling = false;
  return st;
}

extern "C" sca_status sca_residual(sca_problem* p, const void* x, void* r, void* stream) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  if (!x || !r) return set_error(SCA_EINVAL, "x or r is NULL");
  hipStream_t s = (hipStream_t)stream;
  residual_any(p, x, r, s);
  return check_launch("sca_residual");
}

extern "C" sca_status sca_select_blocks(sca_problem* p, const sca_opts* o, int64_t k,
                                        uint8_t* mask, void* stream) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (!mask || k < 0) return set_error(SCA_EINVAL, "mask is NULL or k < 0");
  hipLaunchKernelGGL(k_select_mask, dim3(std::max<int64_t>(1, std::min<int64_t>(
                                        1024, (p->nblocks + 255) / 256))),
                     dim3(256), 0, (hipStream_t)stream, (int)p->nblocks, o->seed, o->instance,
                     selection_threshold(o->select_p), (long long)k, mask);
  return check_launch("sca_select_blocks");
}

extern "C" sca_status sca_philox4x32_10(const uint32_t* in, uint32_t* out, int64_t count,
                                        void* stream) {
  if (count < 0 || (count > 0 && (!in || !out)))
    return set_error(SCA_EINVAL, "bad philox arguments");
  if (count == 0) return SCA_OK;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)std::min<int64_t>(1024, (count + 255) / 256)),
                     dim3(256), 0, (hipStream_t)stream, in, out, (long long)count);
  return check_launch("sca_philox4x32_10");
}

// F (fresh residual), merit, M_F, nnz into host scalars.  Synchronises.
sca_status sca::report(sca_problem* p, const sca_opts* o, const void* x, double* F,
                       double* merit, double* MF, int64_t* nnz, hipStream_t s) {
  const BRParams bp = make_brparams(p, o->tau);
  residual_any(p, x, nullptr, s);
  objective_any(p, x, p->d_r64, true, bp, p->d_scal, s);
  const bool want_probe = merit || MF || nnz;
  if (want_probe) probe_any(p, x, bp, p->d_scal + 8, s);
  double h[16];
  if (hipMemcpyAsync(h, p->d_scal, sizeof(double) * 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "objective: %s", hipGetErrorString(hipGetLastError()));
  if (F) *F = h[0];
  if (merit) *merit = h[8];
  if (MF) *MF = h[9];
  if (nnz) *nnz = (int64_t)h[10];
  return SCA_OK;
}

extern "C" sca_status sca_objective(sca_problem* p, const sca_opts* o, const void* x, double* F,
                                    double* merit, double* MF, int64_t* nnz, void* stream) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if ((st = check_tau(p, o->tau)) != SCA_OK) return st;
  if (!x) return set_error(SCA_EINVAL, "x is NULL");
  return report(p, o, x, F, merit, MF, nnz, (hipStream_t)stream);
}

// One graph = check_every rounds followed by the FP64 objective of the running residual
// (into d_scal[0]); rebuilt when any baked-in argument changes.
static sca_status solve_graph(sca_problem* p, const sca_opts* o, void* x, void* r,
                              const BRParams& bp) {
  const double key[14] = {(double)(uintptr_t)x, (double)(uintptr_t)r, (double)o->check_every,
                          o->select_p, (double)o->seed, (double)o->instance, o->tau, p->lam,
                          p->c, p->beta, (double)p->reg, p->theta, (double)o->delay_chunks,
                          (double)o->delay_stale};
  bool same = p->sgraph != nullptr;
  for (int i = 0; same && i < 14; ++i)
    same = key[i] == p->skey[i] || (key[i] != key[i] && p->skey[i] != p->skey[i]);
  if (same) return SCA_OK;
  if (p->sgraph) {
    (void)hipGraphExecDestroy(p->sgraph);
    p->sgraph = nullptr;
  }
  if (!p->cap && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
    return set_error(SCA_EHIP, "stream creation failed");
  hipGraph_t g;
  if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return set_error(SCA_EHIP, "graph capture failed to start");
  if (p->dtype == SCA_F32)
    run_rounds_t<float>(p, o, o->check_every, (float*)x, (float*)r, p->cap);
  else
    run_rounds_t<double>(p, o, o->check_every, (double*)x, (double*)r, p->cap);
  objective_any(p, x, r, false, bp, p->d_scal, p->cap);
  if (hipStreamEndCapture(p->cap, &g) != hipSuccess)
    return set_error(SCA_EHIP, "graph capture failed");
  const hipError_t e = hipGraphInstantiate(&p->sgraph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    p->sgraph = nullptr;
    return set_error(SCA_EHIP, "graph instantiation failed");
  }
  for (int i = 0; i < 14; ++i) p->skey[i] = key[i];
  return SCA_OK;
}

extern "C" sca_status sca_solve(sca_problem* p, const sca_opts* o, void* x, sca_stats* stats,
                                void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if ((st = check_tau(p, o->tau)) != SCA_OK) return st;
  if ((st = prepare_delay(p, o)) != SCA_OK) return st;
  if (!x) return set_error(SCA_EINVAL, "x is NULL");
  if (stats && stats->struct_size != sizeof(sca_stats))
    return set_error(SCA_EINVAL, "stats.struct_size mismatch");
  if (o->max_rounds < 0 || o->check_every < 1 || o->refresh_every < 0)
    return set_error(SCA_EINVAL, "max_rounds >= 0, check_every >= 1, refresh_every >= 0");
  if (o->tol_rel_obj > 0.0 && !(std::isfinite(o->F_star) && o->F_star != 0.0))
    return set_error(SCA_EINVAL, "tol_rel_obj needs a finite nonzero F_star");
  hipStream_t s = (hipStream_t)stream;
  const BRParams bp = make_brparams(p, o->tau);
  p->profiling = (o->flags & SCA_FLAG_PROFILE) != 0;
  void* r = p->d_rtmp;  // running residual in the dtype (library-owned)
  // r^0 = A x^0 - b (FP64 accumulation); round counter and step from round 0
  init_round_state(p, o, 0, s);
  residual_any(p, x, r, s);
  int64_t k = 0;
  int32_t checks = 0;
  sca_status result = SCA_ENOTCONV;
  double F = NAN;
  // without profiling, whole checks run as one graph launch (rounds + objective)
  const bool use_graph = !p->profiling;
  if (use_graph && (st = solve_graph(p, o, x, r, bp)) != SCA_OK) return st;
  while (k < o->max_rounds) {
    const int64_t nr = std::min<int64_t>(o->check_every, o->max_rounds - k);
    const bool refresh = o->refresh_every > 0 && (checks + 1) % o->refresh_every == 0;
    if (use_graph && nr == o->check_every && !refresh) {
      if (hipGraphLaunch(p->sgraph, s) != hipSuccess)
        return set_error(SCA_EHIP, "graph launch failed");
    } else {
      if (p->dtype == SCA_F32)
        run_rounds_t<float>(p, o, nr, (float*)x, (float*)r, s);
      else
        run_rounds_t<double>(p, o, nr, (double*)x, (double*)r, s);
      if (refresh) residual_any(p, x, r, s);
      objective_any(p, x, r, false, bp, p->d_scal, s);
    }
    k += nr;
    ++checks;
    if (hipMemcpyAsync(&F, p->d_scal, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_error(SCA_EHIP, "solve: %s", hipGetErrorString(hipGetLastError()));
    prof_collect(p);
    if (!std::isfinite(F)) {
      result = SCA_ENONFINITE;
      break;
    }
    bool done = false;
    if (o->tol_rel_obj > 0.0 && (F - o->F_star) / std::fabs(o->F_star) <= o->tol_rel_obj) {
      double Ff;  // confirm with a fresh residual
      if ((st = report(p, o, x, &Ff, nullptr, nullptr, nullptr, s)) != SCA_OK) return st;
      done = (Ff - o->F_star) / std::fabs(o->F_star) <= o->tol_rel_obj;
      if (!done) residual_any(p, x, r, s);  // the running residual drifted: restart it
    }
    if (!done && o->tol_merit > 0.0) {
      double mer;
      if ((st = report(p, o, x, nullptr, &mer, nullptr, nullptr, s)) != SCA_OK) return st;
      done = mer <= o->tol_merit;
    }
    if (done) {
      result = SCA_OK;
      break;
    }
  }
  p->profiling = false;
  if (o->max_rounds == 0 || (o->tol_rel_obj <= 0.0 && o->tol_merit <= 0.0 && result == SCA_ENOTCONV))
    result = SCA_OK;  // no tolerance asked: running the budget is success
  double Ff = NAN, mer = NAN, mf = NAN;
  int64_t nnz = 0;
  if (result != SCA_ENONFINITE) {
    if ((st = report(p, o, x, &Ff, &mer, &mf, &nnz, s)) != SCA_OK) return st;
  }
  int64_t counters[2] = {0, 0};  // coord_updates, moved_updates (adjacent in RoundState)
  if (hipMemcpyAsync(counters, (char*)p->d_state + offsetof(RoundState, coord_updates),
                     2 * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "solve: %s", hipGetErrorString(hipGetLastError()));
  if (stats) {
    stats->rounds = k;
    stats->coord_updates = counters[0];
    stats->moved_updates = counters[1];
    stats->F = Ff;
    stats->merit = mer;
    stats->MF = mf;
    stats->rel_err = (o->F_star != 0.0 && std::isfinite(o->F_star))
                         ? (Ff - o->F_star) / std::fabs(o->F_star)
                         : 0.0;
    stats->nnz = nnz;
    stats->status = result;
    stats->checks = checks;
    stats->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (result == SCA_ENONFINITE) return set_error(SCA_ENONFINITE, "objective became non-finite");
  if (result == SCA_ENOTCONV) return set_error(SCA_ENOTCONV, "max_rounds reached");
  return SCA_OK;
}
