// Many right-hand sides over one dense A on the matrix cores.  K problems share A and one
// block draw per round (Algorithm 1, S.1), so the round's partial gradients G = A_S^T R
// (|S| x K) and its residual update R += A_J dX_J are matrix products; both run as
// 16x16x4 MFMA tiles (FP32 or FP64), with the small operand (R, or the moved rows of dX)
// staged in LDS and the large one (columns of A) streamed from HBM.  Reductions that span
// workgroups go through fixed-order partial sums, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "sca_internal.h"

using namespace sca;

struct sca_multi {
  int dtype = SCA_F32;
  size_t esize = 4;
  int64_t m = 0, n = 0, lda = 0, K = 0, KP = 0, ldb = 0;
  const void* A = nullptr;
  const void* B = nullptr;
  std::vector<double> lam;
  double c = 0, beta = INFINITY;
  int64_t nblocks = 0;
  double cn2_min = 0;
  int ncu = 256;
  std::vector<double> fstar;
  // device workspace
  int* d_bp = nullptr;
  double* d_cn2 = nullptr;
  double* d_lam = nullptr;
  double* d_fstar = nullptr;
  RoundState* d_state = nullptr;
  int* d_sel = nullptr;      // drawn coordinates of the round (n)
  int* d_iota = nullptr;     // 0..n-1 (the list of every coordinate)
  int* d_nall = nullptr;     // n (count of that list)
  void* d_G = nullptr;       // gradient partials: kMNS x n x KP (dtype; FP64 for probes)
  void* d_D = nullptr;       // moves of the drawn coordinates: n x KP (dtype)
  void* d_mv = nullptr;      // moved flags of the drawn coordinates (dtype 0/1), n
  int* d_chunk = nullptr;
  int* d_J = nullptr;        // compacted positions (n)
  void* d_Jv = nullptr;      // compaction values (n, unused)
  int* d_Jc = nullptr;       // column of each listed entry (n)
  void* d_DJ = nullptr;      // rows of the moves (or X) of the listed entries: n x KP (FP64 room)
  void* d_Rp = nullptr;      // fold partials: kMFS x m x KP (FP64 room)
  void* d_R = nullptr;       // running residual of sca_multi_solve (lda x K, dtype)
  double* d_R64 = nullptr;   // FP64 residual (lda x K)
  void* d_Xt = nullptr;      // X rows (n x KP, FP64 room) for fresh residuals
  int* d_active = nullptr;   // per problem: 1 while it still moves
  long long* d_done = nullptr;  // round at which a problem met its stop (-1: not yet)
  long long* d_upd = nullptr;   // per problem: coordinate updates while it was active
  double* d_F = nullptr;     // per problem F (K)
  double* d_mer = nullptr;   // per problem merit (K)
  int* d_nnz = nullptr;      // per problem nnz(xh) (K)
  double* d_part = nullptr;  // reduction partials
  int part_blocks = 0;
  // graph of check_every rounds + check
  hipStream_t cap = nullptr;
  hipGraphExec_t graph = nullptr;
  double gkey[10] = {0};
  // profiling (SCA_FLAG_PROFILE)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  double prof_ms[SCA_K_NKINDS] = {0, 0, 0, 0};
  int64_t prof_n[SCA_K_NKINDS] = {0, 0, 0, 0};
  bool profiling = false;
};

namespace {

constexpr int kMTC = 128;  // gradient tile: drawn coordinates per workgroup
constexpr int kMKC = 32;   // gradient: rows of R staged per LDS chunk
constexpr int kMNS = 16;   // gradient: row splits (partials reduced in the best response)
constexpr int kMFR = 256;  // fold tile: rows per workgroup (64 per wave)
constexpr int kMEC = 16;   // fold: list entries staged per LDS chunk
constexpr int kMFS = 32;   // fold: list splits (partials reduced in the fold reduction)
constexpr int kMaxK = 64;
constexpr int kMGC = 16;   // FP32 gradient (64 problems): rows per chunk of the LDS ring

// 16x16x4 MFMA: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k; element (i, j) of
// the result sits in lane j + 16*(i/4), register i%4 (FP32) or lane j + 16*(i%4),
// register i/4 (FP64).
template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int reg) { return 4 * (lane >> 4) + reg; }
};
template <> struct Mma<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int reg) { return (lane >> 4) + 4 * reg; }
};

// Four consecutive elements (16 bytes of FP32, 32 of FP64).
template <typename T> struct Quad {
  T v[4];
};
template <typename T>
__device__ __forceinline__ Quad<T> load_quad(const T* p) {
  Quad<T> q;
  if constexpr (sizeof(T) == 4) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    q.v[0] = f.x;
    q.v[1] = f.y;
    q.v[2] = f.z;
    q.v[3] = f.w;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    q.v[0] = a.x;
    q.v[1] = a.y;
    q.v[2] = b.x;
    q.v[3] = b.y;
  }
  return q;
}

// Partial gradients G[sp][t][j] = sum over the rows of split sp of A[r][list[t]] * R[r][j],
// t < S (drawn coordinates), j < KP.  Workgroup tile: kMTC coordinates x KP problems; wave
// w takes coordinates 32w..32w+31 of the tile (two 16-row MFMA tiles) against all KP
// problems (KP/16 MFMA tiles).  Each lane reads four consecutive rows of its coordinate's
// column (16 bytes) and feeds them to four successive MFMAs, whose K slots are those rows;
// R's rows are staged in LDS per chunk of kMKC rows, in two alternating buffers (one barrier
// per chunk).  TA: element type of A; TM: type of R,
// of the products and of the partials (TM = double with TA = float: FP64 products for
// probes).
template <typename TA, typename TM, int NST>
__global__ void __launch_bounds__(256)
k_mgrad(const TA* __restrict__ A, long long lda, int m, const TM* __restrict__ R, long long ldr,
        int K, const int* __restrict__ list, const int* __restrict__ S_ptr, TM* __restrict__ G,
        long long ldg) {
  typedef Mma<TM> M;
  constexpr int KP = NST * 16;
  constexpr int LD = kMKC + 4;  // LDS row stride (keeps every quad 16-byte aligned)
  __shared__ TM s_r[2][KP][LD];
  int cc = 0;  // chunks staged so far (LDS buffer cc & 1)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int S = *S_ptr;
  const int sp = blockIdx.y;
  const int MS = ((m + kMNS - 1) / kMNS + kMKC - 1) / kMKC * kMKC;
  const int rlo = min(m, sp * MS), rhi = min(m, rlo + MS);
  const int kq = lane >> 4, li = lane & 15;
  for (int tile = blockIdx.x; tile * kMTC < S; tile += gridDim.x) {
    const int tb = tile * kMTC + 32 * wave;
    int col[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int t = tb + 16 * c + li;
      col[c] = t < S ? list[t] : -1;
    }
    typename M::acc acc[2][NST];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < NST; ++s) acc[c][s] = (typename M::acc){0, 0, 0, 0};
    for (int r0 = rlo; r0 < rhi; r0 += kMKC) {
      // this lane's A quads of the chunk (issued first, so that the latencies overlap)
      Quad<TM> a[kMKC / 16][2];
#pragma unroll
      for (int step = 0; step < kMKC / 16; ++step) {
        const int rb = r0 + 16 * step + 4 * kq;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
          for (int u = 0; u < 4; ++u) a[step][c].v[u] = (TM)0;
          if (col[c] >= 0) {
            const TA* p = A + (size_t)col[c] * lda + rb;
            if (rb + 3 < rhi) {
              const Quad<TA> qa = load_quad<TA>(p);
#pragma unroll
              for (int u = 0; u < 4; ++u) a[step][c].v[u] = (TM)qa.v[u];
            } else {
#pragma unroll
              for (int u = 0; u < 4; ++u)
                if (rb + u < rhi) a[step][c].v[u] = (TM)p[u];
            }
          }
        }
      }
      // this thread's quads of R rows r0..r0+kMKC-1 (zeros past the split and past K), also
      // loaded before the barrier
      constexpr int NQ = (KP * (kMKC / 4) + 255) / 256;
      Quad<TM> rq[NQ];
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const int q = threadIdx.x + 256 * i;
        const int j = q / (kMKC / 4), rr = 4 * (q % (kMKC / 4));
#pragma unroll
        for (int u = 0; u < 4; ++u) rq[i].v[u] = (TM)0;
        if (q < KP * (kMKC / 4) && j < K) {
          const int r = r0 + rr;
          if (r + 3 < rhi) {
            rq[i] = load_quad<TM>(R + (size_t)j * ldr + r);
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (r + u < rhi) rq[i].v[u] = R[(size_t)j * ldr + r + u];
          }
        }
      }
      const int bb = cc & 1;
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const int q = threadIdx.x + 256 * i;
        if (q < KP * (kMKC / 4)) {
          const int j = q / (kMKC / 4), rr = 4 * (q % (kMKC / 4));
#pragma unroll
          for (int u = 0; u < 4; ++u) s_r[bb][j][rr + u] = rq[i].v[u];
        }
      }
      __syncthreads();
      ++cc;
#pragma unroll
      for (int step = 0; step < kMKC / 16; ++step) {
        Quad<TM> bq[NST];
#pragma unroll
        for (int s = 0; s < NST; ++s) bq[s] = load_quad<TM>(&s_r[bb][16 * s + li][16 * step + 4 * kq]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int c = 0; c < 2; ++c) acc[c][s] = M::mma(a[step][c].v[u], bq[s].v[u], acc[c][s]);
      }
    }
    // partials of this tile
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < NST; ++s)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int t = tb + 16 * c + M::row(lane, g);
          if (t < S) G[(size_t)sp * ldg + (size_t)t * KP + 16 * s + li] = acc[c][s][g];
        }
  }
}

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// FP32 partial gradients, as k_mgrad (same tile, lanes, MFMA K slots and G layout), with the
// operands of the next chunk of CH rows loaded straight into LDS (direct-to-LDS 16-byte loads)
// while the current chunk is multiplied, so that their latency hides behind the products
// without registers held for them (two stages, each a distinct pair of LDS arrays, so that the
// compiler sees that reading one stage does not wait for the loads into the other).  A: lane
// l of wave w loads its own quads (rows 16s+4(l/16)..+3 of coordinate 16c+l%16 of the wave's
// 32) into slot (w, s, c) * 64 + l and reads them back itself.  R: slot j*(CH/4) + q holds
// rows 4q..4q+3 of the chunk for problem j, loaded 64 slots per instruction by the four waves
// (each problem's quads one contiguous run), so that every lane's B quad is one slot and the
// 64 lanes of a read cover one contiguous 1 KiB.  One barrier per chunk, after each wave has
// waited for its own loads of the chunk, makes R visible and frees the other stage for the
// next loads.  Quads of rows past the split's end, of a coordinate past S or of a problem past
// K are loaded from an in-range address and zeroed after the read-back.  Against k_mgrad on
// 64 problems: no A registers in flight (5 waves per SIMD, as k_mgrad), 618 against 678 us
// per round on the 64-lambda sweep over the 20000 x 100000 LASSO.
template <int NST, int CH>
struct MgradDma {
  static constexpr int KP = NST * 16;
  static constexpr int NA = (CH / 16) * 2;             // A loads per lane and chunk
  static constexpr int NR = KP * (CH / 4) / 256;       // R loads per lane and chunk
  static constexpr int A_SLOTS = 4 * NA * 64;
  static constexpr int R_SLOTS = KP * (CH / 4);
  static_assert(CH % 16 == 0 && (KP * (CH / 4)) % 256 == 0, "chunk shape");
};

template <int NST, int CH>
__device__ __forceinline__ void mgd_issue(float4* __restrict__ sa, float4* __restrict__ sr,
                                          const float* __restrict__ A, long long lda,
                                          const float* __restrict__ R, long long ldr, int K,
                                          const int (&colc)[2], int r0, int rhi, int kq,
                                          int wave, int lane) {
  typedef MgradDma<NST, CH> D;
#pragma unroll
  for (int step = 0; step < CH / 16; ++step) {
    int rb = r0 + 16 * step + 4 * kq;
    rb = rb < rhi ? rb : r0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
      __builtin_amdgcn_global_load_lds((const void*)(A + (size_t)colc[c] * lda + rb),
                                       (lds_void_ptr)(sa + (wave * D::NA + 2 * step + c) * 64),
                                       16, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < D::NR; ++i) {
    const int slot = (wave * D::NR + i) * 64 + lane;
    const int j = min(slot / (CH / 4), K - 1);
    int r = r0 + 4 * (slot % (CH / 4));
    r = r < rhi ? r : r0;
    __builtin_amdgcn_global_load_lds((const void*)(R + (size_t)j * ldr + r),
                                     (lds_void_ptr)(sr + (wave * D::NR + i) * 64), 16, 0, 0);
  }
}

template <int NST, int CH>
__device__ __forceinline__ void mgd_compute(const float4* __restrict__ sa,
                                            const float4* __restrict__ sr,
                                            typename Mma<float>::acc (&acc)[2][NST],
                                            const bool (&live)[2], int K, int r0, int rhi, int kq,
                                            int li, int wave, int lane) {
  typedef MgradDma<NST, CH> D;
#pragma unroll
  for (int step = 0; step < CH / 16; ++step) {
    const int rb = r0 + 16 * step + 4 * kq;
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) ok[u] = rb + u < rhi;
    float a[2][4];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float4 f = sa[(wave * D::NA + 2 * step + c) * 64 + lane];
      a[c][0] = (live[c] && ok[0]) ? f.x : 0.f;
      a[c][1] = (live[c] && ok[1]) ? f.y : 0.f;
      a[c][2] = (live[c] && ok[2]) ? f.z : 0.f;
      a[c][3] = (live[c] && ok[3]) ? f.w : 0.f;
    }
    float b[NST][4];
#pragma unroll
    for (int s = 0; s < NST; ++s) {
      const bool pj = 16 * s + li < K;
      const float4 f = sr[(16 * s + li) * (CH / 4) + 4 * step + kq];
      b[s][0] = (pj && ok[0]) ? f.x : 0.f;
      b[s][1] = (pj && ok[1]) ? f.y : 0.f;
      b[s][2] = (pj && ok[2]) ? f.z : 0.f;
      b[s][3] = (pj && ok[3]) ? f.w : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int s = 0; s < NST; ++s)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[c][s] = Mma<float>::mma(a[c][u], b[s][u], acc[c][s]);
  }
}

// Waits for all of this wave's vector memory operations (the direct-to-LDS loads of the chunk
// about to be read among them), then a workgroup barrier.
__device__ __forceinline__ void mgd_wait_sync() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt not waited on here
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int NST, int CH>
__global__ void __launch_bounds__(256, 5)  // 90 registers: 5 waves per SIMD
k_mgrad_dma(const float* __restrict__ A, long long lda, int m, const float* __restrict__ R,
            long long ldr, int K, const int* __restrict__ list, const int* __restrict__ S_ptr,
            float* __restrict__ G, long long ldg) {
  typedef MgradDma<NST, CH> D;
  typedef Mma<float> M;
  __shared__ float4 s_a0[D::A_SLOTS], s_a1[D::A_SLOTS];
  __shared__ float4 s_r0[D::R_SLOTS], s_r1[D::R_SLOTS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int S = *S_ptr;
  const int sp = blockIdx.y;
  const int MS = ((m + kMNS - 1) / kMNS + CH - 1) / CH * CH;
  const int rlo = min(m, sp * MS), rhi = min(m, rlo + MS);
  const int nch = (rhi - rlo + CH - 1) / CH;
  const int kq = lane >> 4, li = lane & 15;
  for (int tile = blockIdx.x; tile * kMTC < S; tile += gridDim.x) {
    const int tb = tile * kMTC + 32 * wave;
    int colc[2];
    bool live[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int t = tb + 16 * c + li;
      live[c] = t < S;
      colc[c] = live[c] ? list[t] : 0;
    }
    typename M::acc acc[2][NST];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < NST; ++s) acc[c][s] = (typename M::acc){0, 0, 0, 0};
    __syncthreads();  // every wave is past its reads of the previous tile
    if (nch > 0) mgd_issue<NST, CH>(s_a0, s_r0, A, lda, R, ldr, K, colc, rlo, rhi, kq, wave, lane);
    // chunk c: wait for its loads, barrier, load chunk c+1 into the other stage, multiply
    auto body = [&](const float4* sa, const float4* sr, float4* sa_n, float4* sr_n, int c) {
      mgd_wait_sync();
      if (c + 1 < nch)
        mgd_issue<NST, CH>(sa_n, sr_n, A, lda, R, ldr, K, colc, rlo + (c + 1) * CH, rhi, kq,
                           wave, lane);
      mgd_compute<NST, CH>(sa, sr, acc, live, K, rlo + c * CH, rhi, kq, li, wave, lane);
    };
    for (int c = 0; c < nch; c += 2) {
      body(s_a0, s_r0, s_a1, s_r1, c);
      if (c + 1 < nch) body(s_a1, s_r1, s_a0, s_r0, c + 1);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < NST; ++s)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int t = tb + 16 * c + M::row(lane, g);
          if (t < S) G[(size_t)sp * ldg + (size_t)t * D::KP + 16 * s + li] = acc[c][s][g];
        }
  }
}

// Best response and relaxed step of every (drawn coordinate t, problem j): one wave per t,
// lane j.  g = sum of the kMNS partials (fixed order) - 2c x; a frozen problem does not move.
// D[t][j] = the move; mv[t] = 1 when any problem moved coordinate t; upd[j] += S for the
// problems still active.
template <typename T>
__global__ void __launch_bounds__(256)
k_mbr(const T* __restrict__ G, long long ldg, const int* __restrict__ list,
      const int* __restrict__ S_ptr, T* __restrict__ X, long long ldx,
      const double* __restrict__ cn2, const double* __restrict__ lam,
      const int* __restrict__ active, const RoundState* __restrict__ st, BRParams bp, int K,
      int KP, T* __restrict__ D, T* __restrict__ mv, long long* __restrict__ upd) {
  const int lane = threadIdx.x & 63;
  const int S = *S_ptr;
  const T gamma = (T)st->gamma_cur;
  if (blockIdx.x == 0 && threadIdx.x < K && active[threadIdx.x]) upd[threadIdx.x] += S;
  for (int t = blockIdx.x * 4 + (threadIdx.x >> 6); t < S; t += gridDim.x * 4) {
    const int col = list[t];
    T d = (T)0;
    if (lane < K) {
      T g = (T)0;
      for (int sp = 0; sp < kMNS; ++sp) g += G[(size_t)sp * ldg + (size_t)t * KP + lane];
      const T xj = X[(size_t)lane * ldx + col];
      g -= (T)bp.c2 * xj;
      const T q = (T)(cn2[col] + bp.tau);
      const T xh = soft_clip<T>(xj - g / q, (T)lam[lane] / q, (T)bp.beta);
      if (active[lane]) d = gamma * (xh - xj);
      X[(size_t)lane * ldx + col] = xj + d;
    }
    if (lane < KP) D[(size_t)t * KP + lane] = d;
    const uint64_t any = __ballot(d != (T)0);
    if (lane == 0) mv[t] = any ? (T)1 : (T)0;
  }
}

// Merit and nnz(xh) of every problem from full partial gradients (list = all coordinates):
// per workgroup and problem, max |xh - x| and the count of xh != 0 -> part.
template <typename TX>
__global__ void __launch_bounds__(256)
k_mprobe(const double* __restrict__ G, long long ldg, int n, const TX* __restrict__ X,
         long long ldx, const double* __restrict__ cn2, const double* __restrict__ lam,
         BRParams bp, int K, int KP, double* __restrict__ pmax, int* __restrict__ pcnt) {
  __shared__ double s_max[4][64];
  __shared__ int s_cnt[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mx = 0.0;
  int cnt = 0;
  for (int t = blockIdx.x * 4 + wave; t < n; t += gridDim.x * 4) {
    if (lane < K) {
      double g = 0.0;
      for (int sp = 0; sp < kMNS; ++sp) g += G[(size_t)sp * ldg + (size_t)t * KP + lane];
      const double xj = (double)X[(size_t)lane * ldx + t];
      g -= bp.c2 * xj;
      const double q = cn2[t] + bp.tau;
      const double xh = soft_clip<double>(xj - g / q, lam[lane] / q, bp.beta);
      mx = fmax(mx, fabs(xh - xj));
      cnt += xh != 0.0;
    }
  }
  s_max[wave][lane] = mx;
  s_cnt[wave][lane] = cnt;
  __syncthreads();
  if (wave == 0) {
    double m2 = s_max[0][lane];
    int c2 = s_cnt[0][lane];
    for (int w = 1; w < 4; ++w) {
      m2 = fmax(m2, s_max[w][lane]);
      c2 += s_cnt[w][lane];
    }
    pmax[(size_t)blockIdx.x * 64 + lane] = m2;
    pcnt[(size_t)blockIdx.x * 64 + lane] = c2;
  }
}

__global__ void k_mprobe_final(const double* __restrict__ pmax, const int* __restrict__ pcnt,
                               int nblk, int K, double* __restrict__ mer, int* __restrict__ nnz) {
  const int j = threadIdx.x;
  if (j >= K) return;
  double m2 = 0.0;
  long long c2 = 0;
  for (int b = 0; b < nblk; ++b) {
    m2 = fmax(m2, pmax[(size_t)b * 64 + j]);
    c2 += pcnt[(size_t)b * 64 + j];
  }
  mer[j] = m2;
  nnz[j] = (int)c2;
}

// Listed entries gathered for the fold: Jc[e] = colmap ? colmap[J[e]] : J[e] (the column)
// and DJ[e][j] = D[J[e]][j] (its row of moves), one wave per entry; the fold then reads
// each with one load instead of a chain of dependent ones.
template <typename TD>
__global__ void __launch_bounds__(256)
k_mgather(const int* __restrict__ J, const int* __restrict__ colmap, const TD* __restrict__ D,
          int KP, const RoundState* __restrict__ st, int* __restrict__ Jc, TD* __restrict__ DJ) {
  const int Jn = st->J_cnt;
  const int lane = threadIdx.x & 63;
  for (int e = blockIdx.x * 4 + (threadIdx.x >> 6); e < Jn; e += gridDim.x * 4) {
    const int t = J[e];
    if (lane == 0) Jc[e] = colmap ? colmap[t] : t;
    for (int j = lane; j < KP; j += 64) DJ[(size_t)e * KP + j] = D[(size_t)t * KP + j];
  }
}

// Fold partials P[sp][r][j] = sum over list entries e of split sp (ascending) of
// A[r][Jc[e]] * DJ[e][j] (k_mgather).
// Workgroup tile: kMFR rows x KP problems; wave w takes rows 64w..64w+63 of the tile.  Lane
// (i, k) of an MFMA reads the 16-byte quad of rows 4i..4i+3 (of the wave's 64) of entry
// k's column and feeds component u to MFMA u, whose result rows are 4i + u: four MFMAs per
// problem tile cover the 64 rows.  Entries are staged kMEC at a time (their rows of D in
// LDS, two alternating buffers: one barrier per chunk); the next chunk's A quads are loaded
// into registers while the current chunk computes (16-entry chunks keep the registers of
// the two chunks at those of one 32-entry chunk).
template <typename TA, typename TD, typename TM, int NST>
__global__ void __launch_bounds__(256)
k_mfold(const TA* __restrict__ A, long long lda, int m, const TD* __restrict__ DJ,
        const int* __restrict__ Jc, const RoundState* __restrict__ st, TM* __restrict__ P,
        long long ldp) {
  typedef Mma<TM> M;
  constexpr int KP = NST * 16;
  __shared__ TM s_d[2][kMEC][KP + 1];
  int cc = 0;  // chunks staged so far (LDS buffer cc & 1)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, li = lane & 15;
  const int Jn = st->J_cnt;
  const int sp = blockIdx.y;
  const int per = ((Jn + kMFS - 1) / kMFS + 3) / 4 * 4;
  const int elo = min(Jn, sp * per), ehi = min(Jn, elo + per);
  const int rb = blockIdx.x * kMFR + 64 * wave + 4 * li;  // this lane's four rows
  typename M::acc acc[4][NST];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int s = 0; s < NST; ++s) acc[u][s] = (typename M::acc){0, 0, 0, 0};
  // A quads of chunk e0 into dst.  FP32: every lane loads (entries past the split repeat
  // the split's last entry, whose staged moves are zero; rows past m read rows m..lda-1 or
  // are clamped to the last row quad, and their results are never stored), so the loads
  // carry no branches and the next chunk's loads stay in flight while this one computes.
  const int mq4 = (m + 3) / 4 * 4;
  auto load_chunk = [&](int e0, Quad<TM> (&dst)[kMEC / 4]) {
#pragma unroll
    for (int step = 0; step < kMEC / 4; ++step) {
      const int e = e0 + 4 * step + kq;
      if constexpr (sizeof(TA) == 4) {
        const TA* p = A + (size_t)Jc[min(e, ehi - 1)] * lda + min(rb, mq4 - 4);
        const Quad<TA> qa = load_quad<TA>(p);
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[step].v[u] = (TM)qa.v[u];
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[step].v[u] = (TM)0;
        if (e < ehi && rb < m) {
          const TA* p = A + (size_t)Jc[e] * lda + rb;
          if (rb + 3 < m) {
            const Quad<TA> qa = load_quad<TA>(p);
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[step].v[u] = (TM)qa.v[u];
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (rb + u < m) dst[step].v[u] = (TM)p[u];
          }
        }
      }
    }
  };
  Quad<TM> a[kMEC / 4];
  if (elo < ehi) load_chunk(elo, a);
  for (int e0 = elo; e0 < ehi; e0 += kMEC) {
    Quad<TM> an[kMEC / 4];
    load_chunk(e0 + kMEC, an);
    const int bb = cc & 1;
    for (int q = threadIdx.x; q < kMEC * KP; q += 256) {
      const int ee = q / KP, j = q % KP;
      const int e = e0 + ee;
      s_d[bb][ee][j] = e < ehi ? (TM)DJ[(size_t)e * KP + j] : (TM)0;
    }
    __syncthreads();
    ++cc;
#pragma unroll
    for (int step = 0; step < kMEC / 4; ++step) {
      const int ee = 4 * step + kq;
#pragma unroll
      for (int s = 0; s < NST; ++s) {
        const TM b = s_d[bb][ee][16 * s + li];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u][s] = M::mma(a[step].v[u], b, acc[u][s]);
      }
    }
#pragma unroll
    for (int step = 0; step < kMEC / 4; ++step) a[step] = an[step];
  }
  const int wr = blockIdx.x * kMFR + 64 * wave;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int s = 0; s < NST; ++s)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int r = wr + 4 * M::row(lane, g) + u;
        if (r < m) P[(size_t)sp * ldp + (size_t)r * KP + 16 * s + li] = acc[u][s][g];
      }
}

// FP32 fold partials, as k_mfold (same tile, lanes, MFMA K slots and P layout) for 64
// problems, with the next chunk of kMFDE list entries loaded straight into LDS while the
// current chunk is multiplied (two stages of distinct LDS arrays, one barrier per chunk after
// each wave's own loads have landed).  A: lane (i, k) of wave w loads rows 4i..4i+3 of the
// wave's 64 of entry 4s+k's column into slot (w, s) * 64 + lane and reads it back itself;
// rows past m are clamped to the last row quad (their results are never stored).  Moves: the
// chunk's rows of DJ (contiguous, 64 problems each) are one 16-byte slot per lane; entries
// past the split repeat its last entry and are zeroed after the read-back.  The columns of
// the chunk after next are loaded into registers behind the chunk's loads, so that the
// address of a load never waits for a column index.  Against k_mfold (the next chunk in
// registers) on the 64-lambda sweep over the 20000 x 100000 LASSO: fold step 401 -> 331 us
// per round.
constexpr int kMFDE = 16;  // list entries per chunk
// Columns of this lane's four entries of the chunk at e0 (entry 4s + k).
__device__ __forceinline__ void mfd_cols(int (&co)[kMFDE / 4], const int* __restrict__ Jc,
                                         int e0, int ehi, int kq) {
#pragma unroll
  for (int step = 0; step < kMFDE / 4; ++step) co[step] = Jc[min(e0 + 4 * step + kq, ehi - 1)];
}

__device__ __forceinline__ void mfd_issue(float4* __restrict__ sa, float4* __restrict__ sd,
                                          const float* __restrict__ A, long long lda,
                                          const int (&co)[kMFDE / 4],
                                          const float* __restrict__ DJ, int e0, int ehi, int rq,
                                          int wave, int lane) {
#pragma unroll
  for (int step = 0; step < kMFDE / 4; ++step)
    __builtin_amdgcn_global_load_lds((const void*)(A + (size_t)co[step] * lda + rq),
                                     (lds_void_ptr)(sa + (wave * (kMFDE / 4) + step) * 64), 16,
                                     0, 0);
  // 256 quads of moves: quad q = wave * 64 + lane is entry q / 16, problems 4 (q % 16) ..
  const int q = wave * 64 + lane;
  const int e = min(e0 + (q >> 4), ehi - 1);
  __builtin_amdgcn_global_load_lds((const void*)(DJ + (size_t)e * 64 + 4 * (q & 15)),
                                   (lds_void_ptr)(sd + wave * 64), 16, 0, 0);
}

__device__ __forceinline__ void mfd_compute(const float4* __restrict__ sa,
                                            const float* __restrict__ sd,
                                            typename Mma<float>::acc (&acc)[4][4], int e0,
                                            int ehi, int kq, int li, int wave, int lane) {
#pragma unroll
  for (int step = 0; step < kMFDE / 4; ++step) {
    const int ee = 4 * step + kq;
    const float4 f = sa[(wave * (kMFDE / 4) + step) * 64 + lane];
    float b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) b[s] = sd[ee * 64 + 16 * s + li];
    const bool ok = e0 + ee < ehi;
    const float a[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float bs = ok ? b[s] : 0.f;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u][s] = Mma<float>::mma(a[u], bs, acc[u][s]);
    }
  }
}

__global__ void __launch_bounds__(256, 4)
k_mfold_dma(const float* __restrict__ A, long long lda, int m, const float* __restrict__ DJ,
            const int* __restrict__ Jc, const RoundState* __restrict__ st,
            float* __restrict__ P, long long ldp) {
  typedef Mma<float> M;
  constexpr int NA = kMFDE / 4;
  __shared__ float4 s_a0[4 * NA * 64], s_a1[4 * NA * 64];
  __shared__ float4 s_d0[kMFDE * 16], s_d1[kMFDE * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, li = lane & 15;
  const int Jn = st->J_cnt;
  const int sp = blockIdx.y;
  const int per = ((Jn + kMFS - 1) / kMFS + 3) / 4 * 4;
  const int elo = min(Jn, sp * per), ehi = min(Jn, elo + per);
  const int mq4 = (m + 3) / 4 * 4;
  const int rq = min(blockIdx.x * kMFR + 64 * wave + 4 * li, mq4 - 4);  // this lane's row quad
  typename M::acc acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[u][s] = (typename M::acc){0, 0, 0, 0};
  if (elo < ehi) {
    // column offsets one chunk ahead of the loads that use them
    int co[kMFDE / 4];
    mfd_cols(co, Jc, elo, ehi, kq);
    mfd_issue(s_a0, s_d0, A, lda, co, DJ, elo, ehi, rq, wave, lane);
    mfd_cols(co, Jc, elo + kMFDE, ehi, kq);
    auto body = [&](const float4* sa, const float4* sd, float4* sa_n, float4* sd_n, int e0) {
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads of the chunk
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
      if (e0 + kMFDE < ehi) {
        mfd_issue(sa_n, sd_n, A, lda, co, DJ, e0 + kMFDE, ehi, rq, wave, lane);
        asm volatile("" ::: "memory");  // the column loads below go after every load above
        mfd_cols(co, Jc, e0 + 2 * kMFDE, ehi, kq);
      }
      mfd_compute(sa, reinterpret_cast<const float*>(sd), acc, e0, ehi, kq, li, wave, lane);
    };
    for (int e0 = elo; e0 < ehi; e0 += 2 * kMFDE) {
      body(s_a0, s_d0, s_a1, s_d1, e0);
      if (e0 + kMFDE < ehi) body(s_a1, s_d1, s_a0, s_d0, e0 + kMFDE);
    }
  }
  const int wr = blockIdx.x * kMFR + 64 * wave;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int r = wr + 4 * M::row(lane, g) + u;
        if (r < m) P[(size_t)sp * ldp + (size_t)r * 64 + 16 * s + li] = acc[u][s][g];
      }
}

// out[j][r] = scale * base[j][r] + sum over the kMFS partials (fixed order), j < K, r < m;
// out and out64 may each be NULL (out may alias base).  Tiles of 64 rows: the partials are
// read row by row (contiguous over the problems), summed, transposed through LDS and
// written column by column.
constexpr int kRT = 64;
template <typename TB, typename TP, typename TO>
__global__ void __launch_bounds__(256)
k_mfold_reduce(const TP* __restrict__ P, long long ldp, int m, int K, int KP, const TB* base,
               long long ldbase, double scale, TO* out, long long ldout,
               double* __restrict__ out64, long long ld64) {
  __shared__ TP tile[kRT][kMaxK + 1];
  for (int rt = blockIdx.x; rt * kRT < m; rt += gridDim.x) {
    const int r0 = rt * kRT;
    for (int q = threadIdx.x; q < kRT * KP; q += 256) {
      const int rr = q / KP, j = q % KP;
      const int r = r0 + rr;
      TP s = (TP)0;
      if (r < m)
        for (int sp = 0; sp < kMFS; ++sp) s += P[(size_t)sp * ldp + (size_t)r * KP + j];
      tile[rr][j] = s;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kRT * K; q += 256) {
      const int j = q / kRT, rr = q % kRT;
      const int r = r0 + rr;
      if (r < m) {
        const double v = scale * (double)base[(size_t)j * ldbase + r] + (double)tile[rr][j];
        if (out) out[(size_t)j * ldout + r] = (TO)v;
        if (out64) out64[(size_t)j * ld64 + r] = v;
      }
    }
    __syncthreads();
  }
}

// X (n x K, column-major) -> rows Xt[col][j] (KP wide, zeros past K) and the flag
// mv[col] = any_j X[j][col] != 0.
template <typename T, typename TO>
__global__ void k_mrows(const T* __restrict__ X, long long ldx, int n, int K, int KP,
                        TO* __restrict__ Xt, T* __restrict__ mv) {
  for (int col = blockIdx.x * 4 + (threadIdx.x >> 6); col < n; col += gridDim.x * 4) {
    const int lane = threadIdx.x & 63;
    const T v = lane < K ? X[(size_t)lane * ldx + col] : (T)0;
    if (lane < KP) Xt[(size_t)col * KP + lane] = (TO)v;
    const uint64_t any = __ballot(v != (T)0);
    if (lane == 0) mv[col] = any ? (T)1 : (T)0;
  }
}

// Per problem j (one workgroup each): F_j = 1/2 ||r_j||^2 - c ||x_j||^2 + lam_j ||x_j||_1
// in FP64 (fixed-order reduction).  With check: relative-error stop (tol > 0) freezes the
// problem and records the round; a non-finite F also freezes it.
template <typename TR, typename TX>
__global__ void __launch_bounds__(256)
k_mobj(const TR* __restrict__ R, long long ldr, int m, const TX* __restrict__ X, long long ldx,
       int n, double c, const double* __restrict__ lam, double* __restrict__ F, int check,
       double tol, const double* __restrict__ fstar, int* __restrict__ active,
       long long* __restrict__ done, const RoundState* __restrict__ st) {
  __shared__ double sh[3][4];
  const int j = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double sr = 0.0, sx = 0.0, s1 = 0.0;
  for (int r = threadIdx.x; r < m; r += 256) {
    const double v = (double)R[(size_t)j * ldr + r];
    sr += v * v;
  }
  for (int t = threadIdx.x; t < n; t += 256) {
    const double v = (double)X[(size_t)j * ldx + t];
    sx += v * v;
    s1 += fabs(v);
  }
  sr = wave_sum(sr);
  sx = wave_sum(sx);
  s1 = wave_sum(s1);
  if (lane == 0) {
    sh[0][wave] = sr;
    sh[1][wave] = sx;
    sh[2][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, d = 0;
    for (int w = 0; w < 4; ++w) {
      a += sh[0][w];
      b += sh[1][w];
      d += sh[2][w];
    }
    const double f = 0.5 * a - c * b + lam[j] * d;
    F[j] = f;
    if (check && active[j]) {
      const bool stop = !isfinite(f) || (tol > 0.0 && (f - fstar[j]) / fabs(fstar[j]) <= tol);
      if (stop) {
        active[j] = 0;
        done[j] = st->k;
      }
    }
  }
}

// Merit stop of the checks: freeze the problems whose merit is <= tol.
__global__ void k_mmerit_check(const double* __restrict__ mer, int K, double tol,
                               int* __restrict__ active, long long* __restrict__ done,
                               const RoundState* __restrict__ st) {
  const int j = threadIdx.x;
  if (j < K && active[j] && mer[j] <= tol) {
    active[j] = 0;
    done[j] = st->k;
  }
}

__global__ void k_mcast(const float* __restrict__ R, long long ldr, int m, int K,
                        double* __restrict__ R64, long long ld64) {
  const long long total = (long long)m * K;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(q / m), r = (int)(q % m);
    R64[(size_t)j * ld64 + r] = (double)R[(size_t)j * ldr + r];
  }
}

__global__ void k_mneg(const void* __restrict__ Bv, long long ldb, int m, int K, int es,
                       void* __restrict__ Rv, long long ldr) {
  const long long total = (long long)m * K;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(q / m), r = (int)(q % m);
    if (es == 4)
      ((float*)Rv)[(size_t)j * ldr + r] = -((const float*)Bv)[(size_t)j * ldb + r];
    else
      ((double*)Rv)[(size_t)j * ldr + r] = -((const double*)Bv)[(size_t)j * ldb + r];
  }
}

__global__ void k_minit(int K, int* __restrict__ active, long long* __restrict__ done,
                        long long* __restrict__ upd) {
  const int j = threadIdx.x;
  if (j < K) {
    active[j] = 1;
    done[j] = -1;
    upd[j] = 0;
  }
}

__global__ void k_mset_one(int* a, int v) { *a = v; }
__global__ void k_miota(int* a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = i;
}

// ------------------------------------------------------------------ host side
void mprof_begin(sca_multi* M, hipStream_t s, int kind) {
  if (!M->profiling) return;
  if (M->ev_used >= M->ev.size()) {
    std::pair<hipEvent_t, hipEvent_t> e;
    (void)hipEventCreate(&e.first);
    (void)hipEventCreate(&e.second);
    M->ev.push_back(e);
  }
  M->ev_kind.resize(M->ev.size());
  M->ev_kind[M->ev_used] = kind;
  (void)hipEventRecord(M->ev[M->ev_used].first, s);
}
void mprof_end(sca_multi* M, hipStream_t s) {
  if (!M->profiling) return;
  (void)hipEventRecord(M->ev[M->ev_used].second, s);
  ++M->ev_used;
}
void mprof_collect(sca_multi* M) {
  if (!M->profiling || M->ev_used == 0) return;
  (void)hipEventSynchronize(M->ev[M->ev_used - 1].second);
  for (size_t i = 0; i < M->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, M->ev[i].first, M->ev[i].second) == hipSuccess) {
      M->prof_ms[M->ev_kind[i]] += ms;
      M->prof_n[M->ev_kind[i]] += 1;
    }
  }
  M->ev_used = 0;
}

int grad_grid_x(const sca_multi* M) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((M->n + kMTC - 1) / kMTC, 2 * M->ncu));
}
long long ldg_of(const sca_multi* M) { return (long long)M->n * M->KP; }
long long ldp_of(const sca_multi* M) { return (long long)M->m * M->KP; }

template <typename TA, typename TM>
void launch_mgrad(sca_multi* M, const TM* R, long long ldr, const int* list, const int* S_ptr,
                  TM* G, hipStream_t s) {
  const dim3 grid(grad_grid_x(M), kMNS);
  const TA* A = (const TA*)M->A;
  const int m = (int)M->m, K = (int)M->K;
  if constexpr (std::is_same<TA, float>::value && std::is_same<TM, float>::value) {
    if (M->KP == 64) {
      hipLaunchKernelGGL((k_mgrad_dma<4, kMGC>), grid, dim3(256), 0, s, A,
                         (long long)M->lda, m, R, ldr, K, list, S_ptr, G, ldg_of(M));
      return;
    }
  }
  switch (M->KP / 16) {
    case 1:
      hipLaunchKernelGGL((k_mgrad<TA, TM, 1>), grid, dim3(256), 0, s, A, (long long)M->lda, m, R,
                         ldr, K, list, S_ptr, G, ldg_of(M));
      break;
    case 2:
      hipLaunchKernelGGL((k_mgrad<TA, TM, 2>), grid, dim3(256), 0, s, A, (long long)M->lda, m, R,
                         ldr, K, list, S_ptr, G, ldg_of(M));
      break;
    case 3:
      hipLaunchKernelGGL((k_mgrad<TA, TM, 3>), grid, dim3(256), 0, s, A, (long long)M->lda, m, R,
                         ldr, K, list, S_ptr, G, ldg_of(M));
      break;
    default:
      hipLaunchKernelGGL((k_mgrad<TA, TM, 4>), grid, dim3(256), 0, s, A, (long long)M->lda, m, R,
                         ldr, K, list, S_ptr, G, ldg_of(M));
      break;
  }
}

template <typename TA, typename TD, typename TM>
void launch_mfold(sca_multi* M, const TD* D, const int* colmap, TM* P, hipStream_t s) {
  const dim3 grid((unsigned)((M->m + kMFR - 1) / kMFR), kMFS);
  const TA* A = (const TA*)M->A;
  const int m = (int)M->m;
  const int ggrid = (int)std::max<int64_t>(1, std::min<int64_t>((M->n + 3) / 4, 8 * M->ncu));
  hipLaunchKernelGGL(k_mgather<TD>, dim3(ggrid), dim3(256), 0, s, (const int*)M->d_J, colmap, D,
                     (int)M->KP, (const RoundState*)M->d_state, M->d_Jc, (TD*)M->d_DJ);
  const TD* DJ = (const TD*)M->d_DJ;
  const int* Jc = (const int*)M->d_Jc;
  if constexpr (std::is_same<TA, float>::value && std::is_same<TD, float>::value &&
                std::is_same<TM, float>::value) {
    if (M->KP == 64) {
      hipLaunchKernelGGL(k_mfold_dma, grid, dim3(256), 0, s, A, (long long)M->lda, m, DJ, Jc,
                         (const RoundState*)M->d_state, P, ldp_of(M));
      return;
    }
  }
  switch (M->KP / 16) {
    case 1:
      hipLaunchKernelGGL((k_mfold<TA, TD, TM, 1>), grid, dim3(256), 0, s, A, (long long)M->lda,
                         m, DJ, Jc, (const RoundState*)M->d_state, P, ldp_of(M));
      break;
    case 2:
      hipLaunchKernelGGL((k_mfold<TA, TD, TM, 2>), grid, dim3(256), 0, s, A, (long long)M->lda,
                         m, DJ, Jc, (const RoundState*)M->d_state, P, ldp_of(M));
      break;
    case 3:
      hipLaunchKernelGGL((k_mfold<TA, TD, TM, 3>), grid, dim3(256), 0, s, A, (long long)M->lda,
                         m, DJ, Jc, (const RoundState*)M->d_state, P, ldp_of(M));
      break;
    default:
      hipLaunchKernelGGL((k_mfold<TA, TD, TM, 4>), grid, dim3(256), 0, s, A, (long long)M->lda,
                         m, DJ, Jc, (const RoundState*)M->d_state, P, ldp_of(M));
      break;
  }
}

// Ordered compaction of the flagged positions of v[0..N) (N from the device) into d_J.
template <typename T>
void mcompact(sca_multi* M, const T* v, const int* N_ptr, int count_moved, hipStream_t s) {
  const int nch = (int)((M->n + kChunk - 1) / kChunk);
  const int cgrid = std::max(1, std::min(nch, 2 * M->ncu));
  hipLaunchKernelGGL(k_compact_count<T>, dim3(cgrid), dim3(1024), 0, s, v, N_ptr, M->d_chunk);
  hipLaunchKernelGGL(k_compact_scatter<T>, dim3(cgrid), dim3(1024), 0, s, v, (const int*)nullptr,
                     N_ptr, (const int*)M->d_chunk, M->d_J, (T*)M->d_Jv, M->d_state, count_moved);
}

BRParams mbr_params(const sca_multi* M, double tau) {
  BRParams bp;
  bp.tau = tau;
  bp.lam = 0.0;
  bp.lam_eta = 0.0;
  bp.c2 = 2.0 * M->c;
  bp.beta = M->beta;
  bp.theta = 0.0;
  bp.eta = 1.0;
  bp.reg = 0;
  return bp;
}

template <typename T>
void mround(sca_multi* M, const sca_opts* o, T* X, T* R, hipStream_t s, uint64_t Tthr,
            const BRParams& bp) {
  const int K = (int)M->K, KP = (int)M->KP;
  int* S_ptr = (int*)((char*)M->d_state + offsetof(RoundState, S_cnt));
  mprof_begin(M, s, SCA_K_SELECT);
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, (int)M->nblocks, M->d_bp, o->seed,
                     o->instance, Tthr, M->d_state, M->d_sel, (int2*)nullptr);
  mprof_end(M, s);
  mprof_begin(M, s, SCA_K_GRAD);
  launch_mgrad<T, T>(M, R, (long long)M->lda, M->d_sel, S_ptr, (T*)M->d_G, s);
  mprof_end(M, s);
  mprof_begin(M, s, SCA_K_COMPACT);
  const int bgrid = (int)std::max<int64_t>(1, std::min<int64_t>((M->n + 3) / 4, 8 * M->ncu));
  hipLaunchKernelGGL(k_mbr<T>, dim3(bgrid), dim3(256), 0, s, (const T*)M->d_G, ldg_of(M),
                     (const int*)M->d_sel, (const int*)S_ptr, X, (long long)M->n, M->d_cn2,
                     M->d_lam, (const int*)M->d_active, (const RoundState*)M->d_state, bp, K, KP,
                     (T*)M->d_D, (T*)M->d_mv, M->d_upd);
  mcompact<T>(M, (const T*)M->d_mv, S_ptr, 1, s);
  mprof_end(M, s);
  mprof_begin(M, s, SCA_K_FOLD);
  launch_mfold<T, T, T>(M, (const T*)M->d_D, M->d_sel, (T*)M->d_Rp, s);
  const int rgrid = (int)std::max<int64_t>(1, std::min<int64_t>((M->m + kRT - 1) / kRT, 8 * M->ncu));
  hipLaunchKernelGGL((k_mfold_reduce<T, T, T>), dim3(rgrid), dim3(256), 0, s, (const T*)M->d_Rp,
                     ldp_of(M), (int)M->m, K, KP, (const T*)R, (long long)M->lda, 1.0, R,
                     (long long)M->lda, (double*)nullptr, 0ll);
  mprof_end(M, s);
}

// Fresh residual A X - B with FP64 products and sums: R_out (dtype, ld lda; may be NULL)
// and d_R64.
template <typename T>
void mresidual(sca_multi* M, const T* X, T* R_out, hipStream_t s) {
  const int K = (int)M->K, KP = (int)M->KP;
  const int bgrid = (int)std::max<int64_t>(1, std::min<int64_t>((M->n + 3) / 4, 8 * M->ncu));
  hipLaunchKernelGGL((k_mrows<T, double>), dim3(bgrid), dim3(256), 0, s, X, (long long)M->n,
                     (int)M->n, K, KP, (double*)M->d_Xt, (T*)M->d_mv);
  mcompact<T>(M, (const T*)M->d_mv, M->d_nall, 0, s);
  launch_mfold<T, double, double>(M, (const double*)M->d_Xt, (const int*)nullptr,
                                  (double*)M->d_Rp, s);
  const int rgrid = (int)std::max<int64_t>(1, std::min<int64_t>((M->m + kRT - 1) / kRT, 8 * M->ncu));
  hipLaunchKernelGGL((k_mfold_reduce<T, double, T>), dim3(rgrid), dim3(256), 0, s,
                     (const double*)M->d_Rp, ldp_of(M), (int)M->m, K, KP, (const T*)M->B,
                     (long long)M->ldb, -1.0, R_out, (long long)M->lda, M->d_R64,
                     (long long)M->lda);
}

// Merit and nnz(xh) from the FP64 residual in d_R64 (FP64 products).
template <typename T>
void mprobe(sca_multi* M, const T* X, const BRParams& bp, hipStream_t s) {
  const int K = (int)M->K, KP = (int)M->KP;
  launch_mgrad<T, double>(M, M->d_R64, (long long)M->lda, M->d_iota, M->d_nall,
                          (double*)M->d_G, s);
  const int pb = M->part_blocks;
  double* pmax = M->d_part;
  int* pcnt = (int*)(M->d_part + (size_t)pb * 64);
  hipLaunchKernelGGL(k_mprobe<T>, dim3(pb), dim3(256), 0, s, (const double*)M->d_G, ldg_of(M),
                     (int)M->n, X, (long long)M->n, M->d_cn2, M->d_lam, bp, K, KP, pmax, pcnt);
  hipLaunchKernelGGL(k_mprobe_final, dim3(1), dim3(64), 0, s, (const double*)pmax,
                     (const int*)pcnt, pb, K, M->d_mer, M->d_nnz);
}

template <typename T>
void mcycle(sca_multi* M, const sca_opts* o, T* X, T* R, hipStream_t s, const BRParams& bp,
            uint64_t Tthr) {
  for (int64_t q = 0; q < o->check_every; ++q) mround<T>(M, o, X, R, s, Tthr, bp);
  hipLaunchKernelGGL((k_mobj<T, T>), dim3((unsigned)M->K), dim3(256), 0, s, (const T*)R,
                     (long long)M->lda, (int)M->m, (const T*)X, (long long)M->n, (int)M->n, M->c,
                     (const double*)M->d_lam, M->d_F, 1, o->tol_rel_obj,
                     (const double*)M->d_fstar, M->d_active, M->d_done,
                     (const RoundState*)M->d_state);
  if (o->tol_merit > 0.0) {
    if (sizeof(T) == 4) {
      const int rgrid = (int)std::max<int64_t>(1, std::min<int64_t>((M->m * M->K + 255) / 256, 4 * M->ncu));
      hipLaunchKernelGGL(k_mcast, dim3(rgrid), dim3(256), 0, s, (const float*)R, (long long)M->lda,
                         (int)M->m, (int)M->K, M->d_R64, (long long)M->lda);
    } else {
      (void)hipMemcpy2DAsync(M->d_R64, sizeof(double) * M->lda, R, sizeof(double) * M->lda,
                             sizeof(double) * M->m, M->K, hipMemcpyDeviceToDevice, s);
    }
    mprobe<T>(M, X, bp, s);
    hipLaunchKernelGGL(k_mmerit_check, dim3(1), dim3(64), 0, s, (const double*)M->d_mer,
                       (int)M->K, o->tol_merit, M->d_active, M->d_done,
                       (const RoundState*)M->d_state);
  }
}

sca_status mcheck_opts(const sca_multi* M, const sca_opts* o) {
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (!(M->cn2_min + o->tau > 0.0))
    return set_error(SCA_EINVAL, "min ||a_j||^2 + tau must be > 0");
  if (o->async_workgroups > 0)
    return set_error(SCA_EINVAL, "lock-free rounds need the single-problem dense path");
  return SCA_OK;
}

sca_status mcheck_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(SCA_EHIP, "%s: %s", what, hipGetErrorString(e));
  return SCA_OK;
}

void mfree(sca_multi* M) {
  void* ptrs[] = {M->d_bp,  M->d_cn2,    M->d_lam,  M->d_fstar, M->d_state, M->d_sel,
                  M->d_iota, M->d_nall,  M->d_G,    M->d_D,     M->d_mv,    M->d_chunk,
                  M->d_J,   M->d_Jv,     M->d_Rp,   M->d_R,     M->d_R64,   M->d_Xt,
                  M->d_active, M->d_done, M->d_F,   M->d_mer,   M->d_nnz,   M->d_part,
                  M->d_upd, M->d_Jc, M->d_DJ};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (M->graph) (void)hipGraphExecDestroy(M->graph);
  if (M->cap) (void)hipStreamDestroy(M->cap);
  for (auto& e : M->ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
}

}  // namespace

// ------------------------------------------------------------------ entry points
extern "C" sca_status sca_multi_create(sca_multi** out, sca_dtype dtype, int64_t m, int64_t n,
                                       const void* A, int64_t lda, int64_t K, const void* B,
                                       int64_t ldb, const double* lambda, double c, double beta,
                                       const int64_t* block_ptr, int64_t nblocks, void* stream) {
  if (!out) return set_error(SCA_EINVAL, "out is NULL");
  *out = nullptr;
  if (K < 1 || K > kMaxK) return set_error(SCA_EINVAL, "K must be in [1, %d]", kMaxK);
  if (!lambda) return set_error(SCA_EINVAL, "lambda is NULL");
  sca_status st = validate_problem_args(dtype, m, n, B, lambda[0], c, beta, block_ptr, nblocks);
  if (st != SCA_OK) return st;
  for (int64_t k = 0; k < K; ++k)
    if (!(lambda[k] >= 0.0) || !std::isfinite(lambda[k]))
      return set_error(SCA_EINVAL, "lambda[%lld] must be finite and >= 0", (long long)k);
  const size_t es = dtype == SCA_F32 ? 4 : 8;
  if (!A) return set_error(SCA_EINVAL, "A is NULL");
  if (((uintptr_t)A) % 16) return set_error(SCA_EINVAL, "A must be 16-byte aligned");
  if (lda < m || (lda * (int64_t)es) % 16)
    return set_error(SCA_EINVAL, "lda must be >= m and lda*sizeof(element) a multiple of 16");
  if (ldb < m) return set_error(SCA_EINVAL, "ldb must be >= m");
  if (n > INT32_MAX / kMaxK || m > INT32_MAX / kMaxK)
    return set_error(SCA_EINVAL, "m and n must be < 2^31 / 64");
  sca_multi* M = new (std::nothrow) sca_multi();
  if (!M) return set_error(SCA_ENOMEM, "host allocation failed");
  M->dtype = dtype;
  M->esize = es;
  M->m = m;
  M->n = n;
  M->lda = lda;
  M->K = K;
  M->KP = (K + 15) / 16 * 16;
  M->A = A;
  M->B = B;
  M->ldb = ldb;
  M->lam.assign(lambda, lambda + K);
  M->c = c;
  M->beta = beta;
  M->nblocks = nblocks;
  M->ncu = device_cu_count();
  M->fstar.assign(K, 0.0);
  M->part_blocks = 4 * M->ncu;
  hipStream_t s = (hipStream_t)stream;
  auto fail = [&](sca_status e) {
    mfree(M);
    delete M;
    return e;
  };
#define MALLOC(ptr, bytes)                                            \
  do {                                                                \
    if ((st = dev_alloc((void**)&(ptr), (bytes))) != SCA_OK) return fail(st); \
  } while (0)
  const size_t KP = (size_t)M->KP;
  MALLOC(M->d_bp, sizeof(int) * (nblocks + 1));
  MALLOC(M->d_cn2, sizeof(double) * n);
  MALLOC(M->d_lam, sizeof(double) * kMaxK);
  MALLOC(M->d_fstar, sizeof(double) * kMaxK);
  MALLOC(M->d_state, sizeof(RoundState));
  MALLOC(M->d_sel, sizeof(int) * n);
  MALLOC(M->d_iota, sizeof(int) * n);
  MALLOC(M->d_nall, sizeof(int) * 16);
  MALLOC(M->d_G, sizeof(double) * kMNS * (size_t)n * KP);
  MALLOC(M->d_D, es * (size_t)n * KP);
  MALLOC(M->d_mv, es * n);
  MALLOC(M->d_chunk, sizeof(int) * ((n + kChunk - 1) / kChunk + 1));
  MALLOC(M->d_J, sizeof(int) * n);
  MALLOC(M->d_Jv, es * n);
  MALLOC(M->d_Jc, sizeof(int) * n);
  MALLOC(M->d_DJ, sizeof(double) * (size_t)n * KP);
  MALLOC(M->d_Rp, sizeof(double) * kMFS * (size_t)m * KP);
  MALLOC(M->d_R, es * (size_t)lda * K);
  MALLOC(M->d_R64, sizeof(double) * (size_t)lda * K);
  MALLOC(M->d_Xt, sizeof(double) * (size_t)n * KP);
  MALLOC(M->d_active, sizeof(int) * kMaxK);
  MALLOC(M->d_done, sizeof(long long) * kMaxK);
  MALLOC(M->d_upd, sizeof(long long) * kMaxK);
  MALLOC(M->d_F, sizeof(double) * kMaxK);
  MALLOC(M->d_mer, sizeof(double) * kMaxK);
  MALLOC(M->d_nnz, sizeof(int) * kMaxK);
  MALLOC(M->d_part, (sizeof(double) + sizeof(int)) * 64 * (size_t)M->part_blocks);
#undef MALLOC
  std::vector<int> bp32(nblocks + 1);
  for (int64_t i = 0; i <= nblocks; ++i) bp32[i] = (int)block_ptr[i];
  std::vector<double> lam64(kMaxK, 0.0);
  for (int64_t k = 0; k < K; ++k) lam64[k] = lambda[k];
  if (hipMemcpyAsync(M->d_bp, bp32.data(), sizeof(int) * bp32.size(), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(M->d_lam, lam64.data(), sizeof(double) * kMaxK, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemsetAsync(M->d_fstar, 0, sizeof(double) * kMaxK, s) != hipSuccess ||
      hipMemsetAsync(M->d_Rp, 0, sizeof(double) * kMFS * (size_t)m * KP, s) != hipSuccess)
    return fail(set_error(SCA_EHIP, "copy of the problem data failed"));
  hipLaunchKernelGGL(k_miota, dim3(256), dim3(256), 0, s, M->d_iota, (int)n);
  hipLaunchKernelGGL(k_mset_one, dim3(1), dim3(1), 0, s, M->d_nall, (int)n);
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, M->d_state, 0ll, 1.0, 0.0, (int)n, 1);
  hipLaunchKernelGGL(k_minit, dim3(1), dim3(64), 0, s, (int)K, M->d_active, M->d_done,
                     M->d_upd);
  if (dtype == SCA_F32)
    hipLaunchKernelGGL(k_colnorm2<float>, dim3(4 * M->ncu), dim3(256), 0, s, (const float*)A,
                       (long long)lda, (int)m, (int)n, M->d_cn2);
  else
    hipLaunchKernelGGL(k_colnorm2<double>, dim3(4 * M->ncu), dim3(256), 0, s, (const double*)A,
                       (long long)lda, (int)m, (int)n, M->d_cn2);
  std::vector<double> cn2(n);
  if (hipMemcpyAsync(cn2.data(), M->d_cn2, sizeof(double) * n, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(set_error(SCA_EHIP, "set-up kernels failed: %s",
                          hipGetErrorString(hipGetLastError())));
  double mn = INFINITY;
  for (double v : cn2) {
    if (!std::isfinite(v)) return fail(set_error(SCA_EINVAL, "A holds NaN or Inf"));
    mn = std::min(mn, v);
  }
  M->cn2_min = mn;
  if (hipStreamCreateWithFlags(&M->cap, hipStreamNonBlocking) != hipSuccess)
    return fail(set_error(SCA_EHIP, "stream creation failed"));
  *out = M;
  return SCA_OK;
}

extern "C" void sca_multi_destroy(sca_multi* M) {
  if (!M) return;
  (void)hipDeviceSynchronize();
  mfree(M);
  delete M;
}

extern "C" sca_status sca_multi_set_fstar(sca_multi* M, const double* F_star) {
  if (!M || !F_star) return set_error(SCA_EINVAL, "NULL argument");
  std::vector<double> f(kMaxK, 0.0);
  for (int64_t k = 0; k < M->K; ++k) {
    if (!std::isfinite(F_star[k]) || F_star[k] == 0.0)
      return set_error(SCA_EINVAL, "F_star[%lld] must be finite and nonzero", (long long)k);
    f[k] = F_star[k];
  }
  M->fstar.assign(F_star, F_star + M->K);
  if (hipMemcpy(M->d_fstar, f.data(), sizeof(double) * kMaxK, hipMemcpyHostToDevice) != hipSuccess)
    return set_error(SCA_EHIP, "copy of F_star failed");
  return SCA_OK;
}

extern "C" sca_status sca_multi_residual(sca_multi* M, const void* X, void* R, void* stream) {
  if (!M || !X || !R) return set_error(SCA_EINVAL, "NULL argument");
  if (((uintptr_t)R) % 16) return set_error(SCA_EINVAL, "R must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (M->dtype == SCA_F32)
    mresidual<float>(M, (const float*)X, (float*)R, s);
  else
    mresidual<double>(M, (const double*)X, (double*)R, s);
  return mcheck_launch("sca_multi_residual");
}

extern "C" sca_status sca_multi_step(sca_multi* M, const sca_opts* o, int64_t round_begin,
                                     int64_t nrounds, void* X, void* R, void* stream) {
  if (!M) return set_error(SCA_EINVAL, "NULL argument");
  sca_status st = mcheck_opts(M, o);
  if (st != SCA_OK) return st;
  if (o->delay_chunks > 1)
    return set_error(SCA_EINVAL, "bounded-delay rounds need the single-problem dense path");
  if (!X || !R || round_begin < 0 || nrounds < 0)
    return set_error(SCA_EINVAL, "X or R is NULL, or a negative round count");
  if (((uintptr_t)R) % 16) return set_error(SCA_EINVAL, "R must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const uint64_t Tthr = selection_threshold(o->select_p);
  const BRParams bp = mbr_params(M, o->tau);
  M->profiling = (o->flags & SCA_FLAG_PROFILE) != 0;
  const double g = gamma_at_round(o->gamma, o->gamma_mu, round_begin);
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, M->d_state, (long long)round_begin, g,
                     o->gamma_mu, (int)M->n, 1);
  hipLaunchKernelGGL(k_minit, dim3(1), dim3(64), 0, s, (int)M->K, M->d_active, M->d_done,
                     M->d_upd);
  for (int64_t q = 0; q < nrounds; ++q) {
    if (M->dtype == SCA_F32)
      mround<float>(M, o, (float*)X, (float*)R, s, Tthr, bp);
    else
      mround<double>(M, o, (double*)X, (double*)R, s, Tthr, bp);
  }
  mprof_collect(M);
  return mcheck_launch("sca_multi_step");
}

static sca_status mreport(sca_multi* M, const sca_opts* o, const void* X, double* F, double* mer,
                          int64_t* nnz, hipStream_t s) {
  const BRParams bp = mbr_params(M, o->tau);
  if (M->dtype == SCA_F32) {
    mresidual<float>(M, (const float*)X, (float*)nullptr, s);
    hipLaunchKernelGGL((k_mobj<double, float>), dim3((unsigned)M->K), dim3(256), 0, s,
                       (const double*)M->d_R64, (long long)M->lda, (int)M->m, (const float*)X,
                       (long long)M->n, (int)M->n, M->c, (const double*)M->d_lam, M->d_F, 0, 0.0,
                       (const double*)M->d_fstar, M->d_active, M->d_done,
                       (const RoundState*)M->d_state);
    if (mer || nnz) mprobe<float>(M, (const float*)X, bp, s);
  } else {
    mresidual<double>(M, (const double*)X, (double*)nullptr, s);
    hipLaunchKernelGGL((k_mobj<double, double>), dim3((unsigned)M->K), dim3(256), 0, s,
                       (const double*)M->d_R64, (long long)M->lda, (int)M->m, (const double*)X,
                       (long long)M->n, (int)M->n, M->c, (const double*)M->d_lam, M->d_F, 0, 0.0,
                       (const double*)M->d_fstar, M->d_active, M->d_done,
                       (const RoundState*)M->d_state);
    if (mer || nnz) mprobe<double>(M, (const double*)X, bp, s);
  }
  std::vector<double> hF(M->K), hm(M->K);
  std::vector<int> hn(M->K);
  if (hipMemcpyAsync(hF.data(), M->d_F, sizeof(double) * M->K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      ((mer || nnz) &&
       (hipMemcpyAsync(hm.data(), M->d_mer, sizeof(double) * M->K, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(hn.data(), M->d_nnz, sizeof(int) * M->K, hipMemcpyDeviceToHost, s) !=
            hipSuccess)) ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "multi objective: %s", hipGetErrorString(hipGetLastError()));
  for (int64_t k = 0; k < M->K; ++k) {
    if (F) F[k] = hF[k];
    if (mer) mer[k] = hm[k];
    if (nnz) nnz[k] = hn[k];
  }
  return SCA_OK;
}

extern "C" sca_status sca_multi_objective(sca_multi* M, const sca_opts* o, const void* X,
                                          double* F, double* mer, int64_t* nnz, void* stream) {
  if (!M || !X) return set_error(SCA_EINVAL, "NULL argument");
  sca_status st = mcheck_opts(M, o);
  if (st != SCA_OK) return st;
  return mreport(M, o, X, F, mer, nnz, (hipStream_t)stream);
}

extern "C" sca_status sca_multi_profile_get(sca_multi* M, double* ms, int64_t* launches,
                                            int reset) {
  if (!M) return set_error(SCA_EINVAL, "NULL argument");
  for (int k = 0; k < SCA_K_NKINDS; ++k) {
    if (ms) ms[k] = M->prof_ms[k];
    if (launches) launches[k] = M->prof_n[k];
    if (reset) {
      M->prof_ms[k] = 0.0;
      M->prof_n[k] = 0;
    }
  }
  return SCA_OK;
}

extern "C" sca_status sca_multi_solve(sca_multi* M, const sca_opts* o, void* X,
                                      sca_stats* stats, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!M || !X) return set_error(SCA_EINVAL, "NULL argument");
  sca_status st = mcheck_opts(M, o);
  if (st != SCA_OK) return st;
  if (o->delay_chunks > 1)
    return set_error(SCA_EINVAL, "bounded-delay rounds need the single-problem dense path");
  if (o->max_rounds < 0 || o->check_every < 1)
    return set_error(SCA_EINVAL, "max_rounds >= 0 and check_every >= 1");
  if (stats)
    for (int64_t k = 0; k < M->K; ++k)
      if (stats[k].struct_size != sizeof(sca_stats))
        return set_error(SCA_EINVAL, "stats[%lld].struct_size mismatch", (long long)k);
  if (o->tol_rel_obj > 0.0)
    for (int64_t k = 0; k < M->K; ++k)
      if (M->fstar[k] == 0.0)
        return set_error(SCA_EINVAL, "problem %lld: tol_rel_obj needs F_star (sca_multi_set_fstar)",
                         (long long)k);
  hipStream_t s = (hipStream_t)stream;
  const uint64_t Tthr = selection_threshold(o->select_p);
  const BRParams bp = mbr_params(M, o->tau);
  M->profiling = (o->flags & SCA_FLAG_PROFILE) != 0;
  void* R = M->d_R;
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, M->d_state, 0ll,
                     gamma_at_round(o->gamma, o->gamma_mu, 0), o->gamma_mu, (int)M->n, 1);
  hipLaunchKernelGGL(k_minit, dim3(1), dim3(64), 0, s, (int)M->K, M->d_active, M->d_done,
                     M->d_upd);
  if (M->dtype == SCA_F32)
    mresidual<float>(M, (const float*)X, (float*)R, s);
  else
    mresidual<double>(M, (const double*)X, (double*)R, s);
  const bool use_graph = !M->profiling;
  const double key[10] = {(double)(uintptr_t)X, (double)o->check_every, o->tol_rel_obj,
                          o->tol_merit,         o->select_p,           (double)o->seed,
                          (double)o->instance,  o->tau,                o->gamma_mu,
                          (double)o->flags};
  if (use_graph && (!M->graph || std::memcmp(key, M->gkey, sizeof(key)) != 0)) {
    if (M->graph) {
      (void)hipGraphExecDestroy(M->graph);
      M->graph = nullptr;
    }
    if (hipStreamSynchronize(s) != hipSuccess)
      return set_error(SCA_EHIP, "multi solve: %s", hipGetErrorString(hipGetLastError()));
    hipGraph_t g;
    if (hipStreamBeginCapture(M->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(SCA_EHIP, "graph capture failed to start");
    if (M->dtype == SCA_F32)
      mcycle<float>(M, o, (float*)X, (float*)R, M->cap, bp, Tthr);
    else
      mcycle<double>(M, o, (double*)X, (double*)R, M->cap, bp, Tthr);
    if (hipStreamEndCapture(M->cap, &g) != hipSuccess)
      return set_error(SCA_EHIP, "graph capture failed");
    const hipError_t e = hipGraphInstantiate(&M->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      M->graph = nullptr;
      return set_error(SCA_EHIP, "graph instantiation failed");
    }
    std::memcpy(M->gkey, key, sizeof(key));
  }
  std::vector<int> act(M->K);
  int64_t k = 0;
  int checks = 0;
  int nact = (int)M->K;
  while (k < o->max_rounds && nact > 0) {
    const int64_t nr = std::min<int64_t>(o->check_every, o->max_rounds - k);
    if (use_graph && nr == o->check_every) {
      if (hipGraphLaunch(M->graph, s) != hipSuccess)
        return set_error(SCA_EHIP, "graph launch failed");
    } else {
      sca_opts o2 = *o;
      o2.check_every = nr;
      if (M->dtype == SCA_F32)
        mcycle<float>(M, &o2, (float*)X, (float*)R, s, bp, Tthr);
      else
        mcycle<double>(M, &o2, (double*)X, (double*)R, s, bp, Tthr);
    }
    k += nr;
    ++checks;
    if (hipMemcpyAsync(act.data(), M->d_active, sizeof(int) * M->K, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_error(SCA_EHIP, "multi solve: %s", hipGetErrorString(hipGetLastError()));
    mprof_collect(M);
    nact = 0;
    for (int64_t q = 0; q < M->K; ++q) nact += act[q];
  }
  std::vector<double> F(M->K), mer(M->K);
  std::vector<int64_t> nnz(M->K);
  if ((st = mreport(M, o, X, F.data(), mer.data(), nnz.data(), s)) != SCA_OK) return st;
  std::vector<long long> done(M->K), pupd(M->K);
  long long upd[2] = {0, 0};
  if (hipMemcpy(done.data(), M->d_done, sizeof(long long) * M->K, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(pupd.data(), M->d_upd, sizeof(long long) * M->K, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(upd, (char*)M->d_state + offsetof(RoundState, coord_updates),
                sizeof(long long) * 2, hipMemcpyDeviceToHost) != hipSuccess)
    return set_error(SCA_EHIP, "multi stats copy failed");
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int notconv = 0, nonfinite = 0;
  const bool want = o->tol_rel_obj > 0.0 || o->tol_merit > 0.0;
  for (int64_t q = 0; q < M->K; ++q) {
    const bool fin = std::isfinite(F[q]);
    const bool conv = done[q] >= 0 && fin;
    if (!fin) ++nonfinite;
    if (!conv && want && fin) ++notconv;
    if (stats) {
      sca_stats& S = stats[q];
      S.rounds = done[q] >= 0 ? done[q] : k;
      S.coord_updates = pupd[q];  // drawn coordinates while this problem was active
      S.moved_updates = upd[1];   // coordinates moved in any problem (shared)
      S.F = F[q];
      S.merit = mer[q];
      S.MF = NAN;
      const double fs = M->fstar[q];
      S.rel_err = fs != 0.0 ? (F[q] - fs) / std::fabs(fs) : 0.0;
      S.seconds = secs;
      S.nnz = nnz[q];
      S.status = !fin ? SCA_ENONFINITE : ((!conv && want) ? SCA_ENOTCONV : SCA_OK);
      S.checks = checks;
    }
  }
  if (nonfinite) return set_error(SCA_ENONFINITE, "%d problems have a non-finite F", nonfinite);
  if (notconv) return set_error(SCA_ENOTCONV, "%d problems did not reach the tolerance", notconv);
  return SCA_OK;
}
