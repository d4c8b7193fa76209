// Host side of libfot: plan/workspace management, the iteration schedule of Algorithm 1
// (arXiv 2512.19072, Sec. 3), the phase read-out (Eq. 9-10) and the C ABI of fot.h.
#include "fot.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <limits>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include "fot_fused.hpp"
#include "fot_beam.hpp"
#include "fot_cfot.hpp"

using namespace fot;

namespace {

thread_local std::string g_err;

fot_status fail(fot_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(FOT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK()                                                                       \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess) return fail(FOT_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

// blocks of the read-out's per-pixel reductions: two pixels per thread up to eight blocks per CU
// (the reductions are latency-bound), fewer on small grids
constexpr int READOUT_BLOCKS = 2048;
inline int readout_blocks(int n) {
  return (int)std::min<long long>(READOUT_BLOCKS, ((long long)n * n + 2 * 256 - 1) / (2 * 256));
}

}  // namespace

// fused-kernel tile configurations (fot_plan_s::tcfg): 64 x 64 tiles, 32 x 32 tiles (small grids,
// 32-wide exponent blocks), 64 x 64 tiles with 32-wide exponent blocks
enum { TCFG_LARGE = 0, TCFG_SMALL = 1, TCFG_BLOCK32 = 2 };

struct fot_plan_s {
  fot_plan_desc d{};
  int n = 0, np = 0, B = 0, prec = 0, tiles = 0;
  size_t esz = 0, zsz = 0, plane = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int lds_limit = 0;   // LDS bytes per workgroup on the plan's device
  // FP64 state and scratch
  double *f = nullptr, *psi = nullptr, *lna = nullptr, *lnb = nullptr, *lnS = nullptr;
  double* mrow = nullptr;
  // T_x at column 0 ([batch][np], the one column the integration reads) and the read-out's fourth
  // FP64 plane, which holds T_y when a solve ends; with x_alias it is the loop's operand buffers
  // (FP32-sized operands, no tape, no schedule: one allocation, dead once the loop is done), whose
  // padded borders are cleared again before the next solve when x_dirty
  double *txc = nullptr, *Ty = nullptr;
  bool x_alias = false, x_dirty = false;
  double *rowsum_g = nullptr, *rowsum_G = nullptr, *rowpart = nullptr, *partials = nullptr;
  double *hist_a = nullptr, *hist_b = nullptr, *rparts = nullptr, *rsums = nullptr;
  unsigned* colkey = nullptr;
  int *kexpA = nullptr, *kexpT = nullptr;   // exponent tables of the block-normalised loop operands
  int nbA = 0, nbT = 0;
  int tcfg = 0;                             // fused kernels' tiles (TCFG_*)
  int* kexpL = nullptr;                     // LN form: [np][nbA] exponents of the block-normalised Lambda
  int* probe_flag = nullptr;                // non-finite flag of the end-of-solve probe
  // range check: per wave of the fused kernels, the lowest margin and the first iteration below the
  // level, [2 (head, tail type of a schedule)][batch][range_spt][2]
  int* range_slots = nullptr;
  int range_spt = 0;
  bool probing = false;                     // the probe's launches are not iteration kernels (no timing)
  int* flag = nullptr;
  // contraction operands (element type of the precision) and pass outputs (float / double)
  void *lam = nullptr, *opA = nullptr, *opB = nullptr, *Z = nullptr;
  // precision schedule: the last tail_iters iterations of a solve run with tail_prec operands,
  // which have their own Lambda and operand buffers (op_set[1]; op_set[0] holds the head type's).
  // lam / opA / opB point at the set of the segment being issued.
  int tail_prec = -1, tail_iters = 0;
  void* op_set[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  double* tape = nullptr;
  int n_ckpt = 0;
  // reverse mode (allocated when checkpoint_every > 0)
  double *fbar = nullptr, *psibar = nullptr, *psibar2 = nullptr, *psiprev = nullptr, *lbbar = nullptr;
  double *Tbx = nullptr, *Tby = nullptr, *wtmp = nullptr, *cbar = nullptr, *rsum_tmp = nullptr;
  double *gsums = nullptr, *gparts = nullptr, *dd_dev = nullptr;
  double *seg_f = nullptr, *seg_psi = nullptr, *seg_lnS = nullptr, *seg_lnSp = nullptr;
  // the segment buffers hold the last checkpoint segment's iterates as the last taped solve
  // computed them (fot_backward then replays that segment no more)
  bool seg_last_valid = false;
  // The phase read-out and the reverse-sweep contractions run with FP64 operands in every
  // precision (once per solve; their signed sums cancel too strongly for FP32).  For FP64 plans
  // these alias the loop's buffers, otherwise they are separate.
  // flam: Lambda's FP64 plane where one is kept (FP64 plans: the loop's own; plans with a tape: the
  // reverse sweep's operand), else null; flamT / flamHT: Toeplitz chunk tables of Lambda and
  // Lambda o H in FP64, which the read-out's GEMMs read (flamT follows flam's plane when it exists)
  double *flam = nullptr, *flamT = nullptr, *flamHT = nullptr, *fA = nullptr, *fB = nullptr, *fZ = nullptr;
  double flam_eps_sep = -1.0;
  bool flamH_valid_sep = false;
  double* flam_eps = nullptr;   // -> lam_eps (FP64 plans) or flam_eps_sep
  bool* flamH_valid = nullptr;  // -> lamH_valid or flamH_valid_sep
  double lam_eps = -1.0;
  double* pending_hist = nullptr;   // marginal-error sum still to be finished by the next row-exp
  const double* pending_parts = nullptr;  // the partials of that sum (written by the last half-step)
  int pending_tiles = 0;                  // and their count per target
  bool lamH_valid = false;
  bool has_state = false;
  bool tape_valid = false;
  int last_iters = 0;
  std::vector<double> last_eps;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // cached HIP graph of the iteration loop, keyed by (iters, eps schedule, tape)
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<double> graph_eps;
  bool graph_tape = false;
  int graph_prof = 0;          // profiler events captured inside the graph
  bool graph_broken = false;   // capture/instantiate failed once: launch eagerly from then on
  const double* graph_pending_parts = nullptr;
  int graph_pending_tiles = 0;
  bool used_graph = false;
  std::vector<hipEvent_t> prof;
  int prof_used = 0;
  // output beam and Gerchberg-Saxton workspace (allocated at the first such call): the four
  // DFT operands [np][2np], the field, the half-transformed field and the transform
  // ([batch][np][2np] each), and per-target scalars
  double *bWa = nullptr, *bWb = nullptr, *bWca = nullptr, *bWcb = nullptr;
  double *bfc = nullptr, *bHt = nullptr, *bF = nullptr;
  double *bpow = nullptr, *bsumG = nullptr, *brow = nullptr, *bl1 = nullptr;
  bool beam_ok = false;   // every buffer above allocated and the DFT operands written
  // cFOT (FOT_FLAG_CFOT): FFT length, twiddles, lambda's transform (for clam_eps), the transposed
  // intermediate of a half-step, f^T and ln a^T (the u-update's orientation), ln S^T of the last
  // u-update, and one marginal-error partial per workgroup
  bool cfot = false;
  int cN = 0;
  cplx* ctw = nullptr;
  double *clamhat = nullptr, *cY = nullptr, *cfT = nullptr, *clnaT = nullptr, *cS = nullptr, *cparts = nullptr;
  double clam_eps = -1.0;
  std::vector<void*> allocs;
  // workspace carved from a caller-independent device array instead of hipMalloc (see plan_init)
  unsigned char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  bool sizing = false;   // plan_init's sizing pass: dalloc only adds up the sizes
};

namespace {

fot_status dalloc(fot_plan_s* p, void** out, size_t bytes) {
  void* ptr = nullptr;
  if (bytes == 0) bytes = 16;
  if (p->sizing) {
    // sizing pass: the offsets are recorded, the pointers are placeholders never used
    const size_t off = (p->arena_used + 255) & ~(size_t)255;
    p->arena_used = off + bytes;
    *out = (void*)(uintptr_t)(256 + off);
    return FOT_OK;
  }
  if (p->arena) {
    // carve 256-byte aligned pieces from the static scratch array
    const size_t off = (p->arena_used + 255) & ~(size_t)255;
    if (off > p->arena_cap || bytes > p->arena_cap - off)
      return fail(FOT_E_INVALID, "the plan's workspace (over " + std::to_string(off + bytes) +
                                     " bytes) exceeds the static scratch array of " + std::to_string(p->arena_cap) +
                                     " bytes");
    p->arena_used = off + bytes;
    *out = p->arena + off;
    return FOT_OK;
  }
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) return fail(FOT_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  p->allocs.push_back(ptr);
  *out = ptr;
  return FOT_OK;
}

template <typename Ptr>
fot_status dalloc_t(fot_plan_s* p, Ptr** out, size_t count) {
  void* v = nullptr;
  fot_status s = dalloc(p, &v, count * sizeof(Ptr));
  *out = (Ptr*)v;
  return s;
}

void drop_graph(fot_plan_s* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  p->graph_eps.clear();
}

void release(fot_plan_s* p) {
  drop_graph(p);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  p->cap = nullptr;
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : p->prof) (void)hipEventDestroy(e);
  p->prof.clear();
}

// ------------------------------------------------------------------ launch helpers
// The marginal-error partials of the last potential update, to be summed by the next row-exp.
PendingSum take_pending(fot_plan_s* p) {
  PendingSum ps{nullptr, p->pending_tiles, nullptr};
  if (p->pending_hist) {
    ps.parts = p->pending_parts;
    ps.out = p->pending_hist;
    p->pending_hist = nullptr;
  }
  return ps;
}

fot_status rev_lambda(fot_plan_s* p, double eps);

// Run `loop` as a cached HIP graph replayed on p->stream (captured on a private stream), keyed by
// the eps schedule and the tape setting.  If capture or instantiation fails, the loop is
// launched eagerly (results are identical) and graphs are not tried again for this plan.
// p->used_graph tells whether the graph ran (the caller then restores the state the loop would
// have left).
template <typename LoopFn>
fot_status run_graph(fot_plan_s* p, const std::vector<double>& e, int iters, LoopFn loop) {
  const bool tape = p->tape != nullptr;
  if (!(p->gexec && p->graph_eps == e && p->graph_tape == tape)) {
    drop_graph(p);
    hipStream_t user = p->stream;
    const int prof0 = p->prof_used;
    p->stream = p->cap;
    p->pending_hist = nullptr;
    hipError_t eb = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    fot_status s = (eb == hipSuccess) ? loop(p, e, iters) : FOT_E_HIP;
    hipGraph_t g = nullptr;
    hipError_t ec = (eb == hipSuccess) ? hipStreamEndCapture(p->cap, &g) : eb;
    p->stream = user;
    hipError_t ei = hipErrorUnknown;
    if (s == FOT_OK && ec == hipSuccess && g) ei = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      p->gexec = nullptr;
      (void)hipGetLastError();
      p->graph_broken = true;
      p->prof_used = prof0;
      p->pending_hist = nullptr;
      g_err.clear();
      return loop(p, e, iters);
    }
    p->graph = g;
    p->graph_eps = e;
    p->graph_tape = tape;
    p->graph_prof = p->prof_used;
    p->graph_pending_parts = p->pending_parts;
    p->graph_pending_tiles = p->pending_tiles;
  } else {
    p->prof_used = p->graph_prof;
    p->pending_parts = p->graph_pending_parts;   // (which buffer the replayed loop leaves pending)
    p->pending_tiles = p->graph_pending_tiles;
  }
  HIP_TRY(hipGraphLaunch(p->gexec, p->stream));
  p->used_graph = true;
  return FOT_OK;
}

// One reverse half-step (see Ops<T>::adj_step):
//   out = mask ? (acc ? out : 0) + w e^{P/eps} K(v e^{-L}) : 0,   K = Lambda (x) Lambda,
// w = scale times the coordinates selected by `coords` (bit 0 rows, bit 1 columns), mask
// ln m > -inf; with lb, also lb += lb_scale out where the mask holds.  With next_L, the pass-1
// operand of the next half-step (v = the new out, L = next_L, in the type of next_eps) is written
// instead of out, which nothing else reads then.
struct AdjStep {
  const double* v;
  const double* L;
  const double* P;
  double eps;
  const double* lnm;
  long long sMarg;
  double scale;
  int coords;
  int acc;
  double* out;
  double* lb;
  double lb_scale;
  const double* next_L;
  double next_eps;
  bool have_operand;   // the previous step built this step's operand
};

template <typename T>
struct Ops {
  typedef typename Mma<T>::out_t zt;

  // Tile configuration of the contraction GEMMs: 64 x 64 output tiles, 8 waves per workgroup
  // (two per SIMD, so one wave's LDS and barrier waits are covered by the other's MFMAs).
  typedef Cfg64x64w8 GC;
  // Fused half-step kernels of grids too small to give every CU a 64 x 64 tile: 32 x 32 tiles of
  // four waves (one per SIMD), whose exponent blocks are 32 wide.  Four times the workgroups
  // and a quarter of the work each, so a launch's fixed latency (first stage, epilogue) is shorter.
  typedef Cfg<32, 32, 4, 1, 1> GS;
  // 64 x 64 tiles with 32-wide exponent blocks (FOT_FLAG_SMALL_TILES on grids that take 64 x 64
  // tiles): the range of the 32 x 32 tiles at close to the speed of the 64 x 64 ones.
  typedef Cfg<64, 64, 8, 2, 1, 2> GC2;
  // Call f with the plan's fused-kernel tile configuration (an empty tag object).
  template <typename F>
  static void with_cfg(const fot_plan_s* p, F&& f) {
    if (p->tcfg == TCFG_SMALL)
      f(GS{});
    else if (p->tcfg == TCFG_BLOCK32)
      f(GC2{});
    else
      f(GC{});
  }

  static fot_status gemm_launch(fot_plan_s* p, int epi, const GemmArgs& a) {
    dim3 grid(p->np / GC::BN, p->np / GC::BM, p->B);
    const dim3 block(GC::THREADS);
    if (epi == EPI_LOGROW)
      hipLaunchKernelGGL((k_gemm<T, EPI_LOGROW, GC>), grid, block, 0, p->stream, a);
    else
      hipLaunchKernelGGL((k_gemm<T, EPI_RAW, GC>), grid, block, 0, p->stream, a);
    LAUNCH_CHECK();
    return FOT_OK;
  }

  static GemmArgs base_args(fot_plan_s* p, const void* A, long long sA, const void* Bm, long long sB) {
    GemmArgs a{};
    a.A = A;
    a.B = Bm;
    a.sA = sA;
    a.sB = sB;
    a.n = p->n;
    a.np = p->np;
    a.nk = (int)((size_t)p->np * sizeof(T) / ROWB);
    a.xcd_swizzle = XCD_BLOCKS;
    return a;
  }

  // LN form of the fused kernels: Lambda stored block-normalised with an exponent table, used
  // once Lambda has entries below the operand type's range (eps small for n); FP64 operands hold
  // every entry that matters and never need it.
  static bool lam_ln(const fot_plan_s* p, double eps) {
    if constexpr (sizeof(T) == 8) {
      (void)p;
      (void)eps;
      return false;
    } else {
      return raw_band(p, eps) < p->n;
    }
  }

  // The LN form keeps Lambda's exponent table in LDS beside the stage buffers: whether the larger
  // of the two kernels (pass 2: static and dynamic LDS) fits at this plan's n_p and tiles.
  static bool ln_fits(fot_plan_s* p) {
    if constexpr (sizeof(T) == 8) {
      (void)p;
      return true;
    } else {
      hipFuncAttributes fa{};
      hipError_t e = hipSuccess;
      size_t dyn = 0;
      with_cfg(p, [&](auto c) {
        typedef decltype(c) C;
        e = hipFuncGetAttributes(&fa, (const void*)k_fused<T, 2, C, FUSED_NBUF, true>);
        dyn = fused_dyn_lds<2, C, true>(p->np);
      });
      int lim = 0;
      if (e != hipSuccess || hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
      return fa.sharedSizeBytes + dyn <= (size_t)lim;
    }
  }

  // Every eps of iterations [t0, t1) must be runnable with this operand type: one that needs the
  // block-normalised Lambda needs its exponent table to fit in LDS.
  static fot_status check_schedule(fot_plan_s* p, const std::vector<double>& e, int t0, int t1) {
    for (int t = t0; t < t1; ++t) {
      if (!lam_ln(p, e[t])) continue;
      if (ln_fits(p)) return FOT_OK;   // (the table's size does not depend on eps)
      {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "fot_solve: at eps %.3g and n %d Lambda needs its block exponents, whose table does not fit "
                      "in LDS with this operand type (use FOT_F64)",
                      e[t], p->n);
        return fail(FOT_E_UNSUPPORTED, msg);
      }
    }
    return FOT_OK;
  }

  static fot_status fill_lambda(fot_plan_s* p, double eps, bool /*unused*/) {
    if (lam_ln(p, eps)) {
      with_cfg(p, [&](auto c) {
        typedef decltype(c) C;
        hipLaunchKernelGGL((k_lambda_blocks<T, C::BN / C::XS>), dim3(p->np), dim3(64), 0, p->stream, p->n, p->np,
                           1.0 / eps, (T*)p->lam, p->kexpL);
      });
    } else {
      const size_t total = p->plane;
      const int blocks = (int)((total + 255) / 256);
      hipLaunchKernelGGL(k_fill_lambda<T>, dim3(blocks), dim3(256), 0, p->stream, (T*)p->lam, (T*)nullptr, p->n,
                         p->np, 1.0 / eps);
      hipLaunchKernelGGL(k_lam_chunks<T>, dim3((2 * p->np + 255) / 256), dim3(256), 0, p->stream, (T*)p->lam,
                         p->np);
    }
    LAUNCH_CHECK();
    p->lam_eps = eps;
    p->lamH_valid = false;
    return FOT_OK;
  }

  // Toeplitz form of Lambda's operand (k_fused<..., TZ = true>, see toeplitz_table_bytes): raw
  // Lambda (its Toeplitz chunks are formed with it; BF16x3: a table of the hi and one of the lo
  // halves), not switched off by FOT_FLAG_STAGED_LAMBDA, and the kernel's LDS, static and dynamic,
  // within the device's limit.
  template <typename C, int PASS, bool ADJ>
  static bool tz_fits(const fot_plan_s* p) {
    if (p->d.flags & FOT_FLAG_STAGED_LAMBDA) return false;
    static const size_t st = [] {
      hipFuncAttributes fa{};
      if (hipFuncGetAttributes(&fa, (const void*)k_fused<T, PASS, C, FUSED_NBUF, false, ADJ, true>) != hipSuccess) {
        (void)hipGetLastError();
        return (size_t)-1;
      }
      return (size_t)fa.sharedSizeBytes;
    }();
    return st != (size_t)-1 &&
           st + fused_dyn_lds<PASS, C, false, true, Mma<T>::PAIRED>(p->np) <= (size_t)p->lds_limit;
  }

  template <typename C, bool LN>
  static void fused_launch_cfg(fot_plan_s* p, int pass, const FusedArgs& a, hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid(p->np / C::BN, p->np / C::BM, p->B);
    const dim3 block(C::THREADS);
    if constexpr (!LN) {
      const uint32_t t1 = (uint32_t)fused_dyn_lds<1, C, false, true, Mma<T>::PAIRED>(p->np);
      const uint32_t t2 = (uint32_t)fused_dyn_lds<2, C, false, true, Mma<T>::PAIRED>(p->np);
      // (Lambda from its table: bands of tiles per XCD, one fetch of each operand panel)
      FusedArgs b = a;
      b.xcd_swizzle = pass == 1 ? XCD_ROWS : XCD_COLS;
      if (pass == 1 && tz_fits<C, 1, false>(p)) {
        hipExtLaunchKernelGGL((k_fused<T, 1, C, FUSED_NBUF, false, false, true>), grid, block, t1, p->stream, e0, e1,
                              0, b);
        return;
      }
      if (pass == 2 && tz_fits<C, 2, false>(p)) {
        hipExtLaunchKernelGGL((k_fused<T, 2, C, FUSED_NBUF, false, false, true>), grid, block, t2, p->stream, e0, e1,
                              0, b);
        return;
      }
    }
    if (pass == 1)
      hipExtLaunchKernelGGL((k_fused<T, 1, C, FUSED_NBUF, LN>), grid, block,
                            (uint32_t)fused_dyn_lds<1, C, LN>(p->np), p->stream, e0, e1, 0, a);
    else
      hipExtLaunchKernelGGL((k_fused<T, 2, C, FUSED_NBUF, LN>), grid, block,
                            (uint32_t)fused_dyn_lds<2, C, LN>(p->np), p->stream, e0, e1, 0, a);
  }
  static fot_status fused_launch(fot_plan_s* p, int pass, const FusedArgs& a) {
    const bool prof = !p->probing && (p->d.flags & FOT_FLAG_PROFILE) && p->prof_used + 2 <= (int)p->prof.size();
    hipEvent_t e0 = prof ? p->prof[p->prof_used] : nullptr;
    hipEvent_t e1 = prof ? p->prof[p->prof_used + 1] : nullptr;
    bool ln = false;
    if constexpr (sizeof(T) < 8) ln = a.kexpL != nullptr;
    with_cfg(p, [&](auto c) {
      typedef decltype(c) C;
      if (ln) {
        if constexpr (sizeof(T) < 8) fused_launch_cfg<C, true>(p, pass, a, e0, e1);
      } else {
        fused_launch_cfg<C, false>(p, pass, a, e0, e1);
      }
    });
    LAUNCH_CHECK();
    if (prof) p->prof_used += 2;
    return FOT_OK;
  }

  // Block-normalised pass-1 operand of a potential (start of a solve or of a replayed segment).
  static fot_status prep(fot_plan_s* p, const double* P, double eps) {
    with_cfg(p, [&](auto c) {
      typedef decltype(c) C;
      hipLaunchKernelGGL((k_prep_blocks<T, C::BN / C::XS>), dim3(p->np * p->np / (256 * PREP_U), p->B), dim3(256), 0,
                         p->stream, P, p->n, p->np, 1.0 / eps, (T*)p->opA, p->kexpA);
    });
    LAUNCH_CHECK();
    return FOT_OK;
  }

  // The largest |i - k| at which Lambda = exp(-(i - k)^2 / (2 n^2 eps)) is nonzero in the operand
  // type (n: no zero entries).  exp(-x) rounds to zero in FP64 for x > 745.2, in FP32 and BF16
  // (and the BF16x3 halves) for x > 104 at the latest, in FP16 for x > 17.4; each bound is taken
  // with a margin, so the band is never too narrow.
  static int band_for(const fot_plan_s* p, double eps, double L) {
    const double w = (double)p->n * std::sqrt(2.0 * eps * L) + 2.0;
    return w >= (double)p->n ? p->n : (int)w;
  }
  static int raw_band(const fot_plan_s* p, double eps) {
    return band_for(p, eps, sizeof(T) == 8 ? 746.0 : std::is_same<T, _Float16>::value ? 18.0 : 105.0);
  }
  // The LN form keeps every entry above FP64's underflow (exponent plus normalised mantissa).
  static int lambda_band(const fot_plan_s* p, double eps) {
    return lam_ln(p, eps) ? band_for(p, eps, 746.0) : raw_band(p, eps);
  }

  // Range check of the products (see range_margin in fot_fused.hpp): a term the operand type cannot
  // hold is off by less than 2^unit_log2 of its block's scale, so an output may lose at most
  // n 2^unit_log2 2^-margin of itself.  That bound takes every term at its block's largest scale and
  // is loose by orders of magnitude; the check fails when it exceeds 2^allowed_loss_log2, levels
  // set between the bounds of accurate and of inaccurate solves in a sweep of the two-Gaussian
  // workload over n = 65 ... 1024 and eps = 1e-2 ... 1e-4 (30 and 60 iterations) against the
  // oracle: FP32 and BF16x3 accurate up to 2.4e-4, inaccurate from 4; BF16 accurate up to 260,
  // inaccurate from 3.4e7; FP64 at 257^2 and eps 1e-4 within 1e-11 of the oracle at 1.4e11 and
  // off where outputs vanished.  FP16 (accurate up to 128, inaccurate from 64) is checked only
  // after the solve.
  static int unit_log2() {
    return sizeof(T) == 8 ? -1021 : std::is_same<T, _Float16>::value ? -23 : -125;
  }
  static int allowed_loss_log2() {
    return sizeof(T) == 8 ? 20 : std::is_same<T, __bf16>::value ? 13 : -7;
  }
  static int range_threshold(int n) {
    if (std::is_same<T, _Float16>::value) return INT_MIN;
    int lg = 0;
    while ((1 << lg) < n) ++lg;          // ceil(log2 n)
    return lg + unit_log2() - allowed_loss_log2();
  }
  // the bound n 2^unit_log2 2^-margin for a recorded margin (0 if no output was recorded)
  static double loss_bound(int n, int margin) {
    if (margin == 0x7f7f7f7f) return 0.0;
    return std::ldexp((double)n, unit_log2() - std::max(margin, -2000));
  }

  // One half-step: Pout = eps (lnm - ln(Lambda . exp(Pin/eps) . Lambda)) (Eq. 7 or Eq. 8), the
  // marginal error of the entering plan to hist[batch] (finished by the next pass 1), and, if
  // next_eps > 0, the block-normalised operand of Pout for the next half-step.  The operand of
  // Pin must be in p->opA / p->kexpA.
  static fot_status half(fot_plan_s* p, const double* Pin, double* Pout, const double* lnm, long long sMarg,
                         double* hist, double* lnS_out, double eps, double next_eps, int* flag = nullptr,
                         int iter = 0, int* range_slots = nullptr) {
    (void)Pin;
    const long long plane = (long long)p->plane;
    FusedArgs a{};
    a.n = p->n;
    a.np = p->np;
    a.nk = (int)((size_t)p->np * sizeof(T) / FROWB);
    a.nbA = p->nbA;
    a.nbT = p->nbT;
    a.xcd_swizzle = XCD_BLOCKS;
    a.band = lambda_band(p, eps);
    a.kexpL = lam_ln(p, eps) ? p->kexpL : nullptr;
    a.range_slots = range_slots;
    a.range_spt = p->range_spt;
    a.iter = iter;
    a.range_thr = range_threshold(p->n);
    // pass 1: W = At . Lambda
    a.A = p->opA;
    a.sA = plane;
    a.B = p->lam;
    a.sB = 0;
    a.kexp = p->kexpA;
    a.outT = p->opB;
    a.kexpT = p->kexpT;
    PendingSum ps = take_pending(p);
    a.pend_parts = ps.parts;
    a.pend_tiles = ps.tiles;
    a.pend_out = ps.out;
    fot_status s = fused_launch(p, 1, a);
    if (s != FOT_OK) return s;
    // pass 2: S = Lambda . Bt, potential update, next operand
    FusedArgs b{};
    b.n = p->n;
    b.np = p->np;
    b.nk = a.nk;
    b.nbA = p->nbA;
    b.nbT = p->nbT;
    b.xcd_swizzle = XCD_BLOCKS;
    b.band = a.band;
    b.kexpL = a.kexpL;
    b.range_slots = range_slots;
    b.range_spt = p->range_spt;
    b.iter = iter;
    b.range_thr = a.range_thr;
    b.A = p->lam;
    b.sA = 0;
    b.B = p->opB;
    b.sB = plane;
    b.kexp = p->kexpT;
    b.lnmarg = lnm;
    b.sMarg = sMarg;
    b.pot = Pout;
    b.lnS_out = lnS_out;
    b.eps = eps;
    b.inv_eps = 1.0 / eps;
    b.next_inv_eps = next_eps > 0.0 ? 1.0 / next_eps : 0.0;
    b.nextA = p->opA;
    b.kexpN = p->kexpA;
    b.partials = p->partials;
    b.flag = flag ? flag : p->flag;
    b.err_on = hist != nullptr;
    s = fused_launch(p, 2, b);
    p->pending_hist = hist;   // nullptr: no marginal-error sum to finish
    p->pending_parts = p->partials;
    p->pending_tiles = p->tiles;
    return s;
  }

  // Iterations [t0, t1) of a solve of `iters` iterations (Algorithm 1) on p->stream, all with
  // operands of type T in p->lam / p->opA / p->opB: the segment starts from the pass-1 operand of
  // psi and Lambda at its first eps; Lambda is regenerated whenever eps changes, psi is
  // checkpointed every k iterations if a tape exists.
  static fot_status segment(fot_plan_s* p, const std::vector<double>& e, int t0, int t1, int iters, int seg = 0) {
    const long long plane = (long long)p->plane;
    const int B = p->B;
    fot_status s = prep(p, p->psi, e[t0]);
    if (s != FOT_OK) return s;
    for (int t = t0; t < t1; ++t) {
      const double ep = e[t];
      if (t == t0 || ep != e[t - 1])
        if ((s = fill_lambda(p, ep, false)) != FOT_OK) return s;
      if (p->tape && (t % p->d.checkpoint_every) == 0) {
        const size_t cnt = (size_t)B * p->plane;
        hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, p->stream, p->psi,
                           p->tape + (size_t)(t / p->d.checkpoint_every) * cnt, cnt);
        LAUNCH_CHECK();
      }
      const bool last = (t == iters - 1);
      const bool hist = !(p->d.flags & FOT_FLAG_NO_HISTORY);
      // with a tape, the iterations of the last checkpoint segment also go to the segment buffers,
      // exactly as fot_backward's replay of that segment would write them
      const int k = p->d.checkpoint_every;
      const bool keep = p->tape && t >= (iters - 1) / k * k;
      const size_t so = keep ? (size_t)(t - (iters - 1) / k * k) * B * p->plane : 0;
      auto copy = [&](const double* src, double* dst) {
        hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, p->stream, src, dst, (size_t)B * p->plane);
      };
      // (the last V-update's ln S' is not kept: the read-out forms it again in FP64)
      double* lnS_u = last ? p->lnS : keep ? p->seg_lnS + so : nullptr;
      double* lnS_v = keep ? p->seg_lnSp + so : nullptr;
      if ((s = half(p, p->psi, p->f, p->lna, 0, hist ? p->hist_a + (size_t)t * B : nullptr, lnS_u, ep, ep, nullptr,
                    t, p->range_slots + (size_t)seg * B * p->range_spt * 2)) != FOT_OK)
        return s;
      if (keep) {
        copy(p->f, p->seg_f + so);
        if (last) copy(p->lnS, p->seg_lnS + so);
      }
      // the last half-step of a segment builds no next operand: the next segment (another type)
      // builds its own from psi
      if ((s = half(p, p->f, p->psi, p->lnb, plane, hist ? p->hist_b + (size_t)t * B : nullptr, lnS_v, ep,
                    t + 1 == t1 ? 0.0 : e[t + 1], nullptr, t, p->range_slots + (size_t)seg * B * p->range_spt * 2)) !=
          FOT_OK)
        return s;
      if (keep) {
        copy(p->psi, p->seg_psi + so);
        LAUNCH_CHECK();
      }
    }
    return FOT_OK;
  }

  // The iteration loop of Algorithm 1 with one operand type.
  static fot_status loop(fot_plan_s* p, const std::vector<double>& e, int iters) {
    fot_status s = check_schedule(p, e, 0, iters);
    if (s != FOT_OK) return s;
    return segment(p, e, 0, iters, iters);
  }

  // End-of-solve probe of the operand type's u-direction products: ln S(psi_T) formed as a u-half
  // would form it, for the read-out to compare with the FP64 value (the update goes to read-out
  // scratch, fZ, which the read-out reads before it writes there; its ln S is ln a - update / eps
  // wherever a > 0, the only pixels the comparison weighs).  The final column marginal checks
  // only the last V-half's products; a loss of range in the u-direction products (the potential
  // psi spanning more than the type holds within one operand block) would otherwise go unseen
  // while the iterates drift.  FP64 operands need no probe.  Its own range check is recorded as
  // iteration `iters` (the state after the last iteration).
  static fot_status probe(fot_plan_s* p, double eps, int iters, int seg) {
    if constexpr (sizeof(T) == 8) {
      (void)p;
      (void)eps;
      (void)iters;
      (void)seg;
      return FOT_OK;
    } else {
      fot_status s = prep(p, p->psi, eps);
      if (s != FOT_OK) return s;
      p->probing = true;
      s = half(p, p->psi, p->fZ, p->lna, 0, nullptr, nullptr, eps, 0.0, p->probe_flag, iters,
               p->range_slots + (size_t)seg * p->B * p->range_spt * 2);
      p->probing = false;
      return s;
    }
  }

  // Run the loop as a cached HIP graph replayed on p->stream (see run_graph).
  static fot_status loop_graph(fot_plan_s* p, const std::vector<double>& e, int iters) {
    fot_status s = run_graph(p, e, iters, [](fot_plan_s* q, const std::vector<double>& ee, int it) {
      return loop(q, ee, it);
    });
    if (s == FOT_OK && p->used_graph) {
      // state after the loop, as if it had been launched directly
      p->pending_hist = (p->d.flags & FOT_FLAG_NO_HISTORY) ? nullptr : p->hist_b + (size_t)(iters - 1) * p->B;
      p->lam_eps = e[iters - 1];
      p->lamH_valid = false;
    }
    return s;
  }

  // ---------------------------------------------------------------- reverse mode
  // One reverse half-step (AdjStep) on the fused kernels: k_adj_prep builds the signed
  // block-normalised operand of v e^{-L} (unless the previous step did), pass 1 forms its product
  // with Lambda and block-normalises it per column, pass 2 forms K and ends in the update.  lam:
  // raw Lambda in this type at eps; A, Bt: operand buffers of this type (their exponent tables are
  // the plan's kexpA and kexpT).
  template <typename C>
  static void adj_launch_cfg(fot_plan_s* p, int pass, const FusedArgs& a) {
    const dim3 grid(p->np / C::BN, p->np / C::BM, p->B);
    const dim3 block(C::THREADS);
    const uint32_t l1 = (uint32_t)fused_dyn_lds<1, C, false>(p->np), l2 = (uint32_t)fused_dyn_lds<2, C, false>(p->np);
    const uint32_t t1 = (uint32_t)fused_dyn_lds<1, C, false, true, Mma<T>::PAIRED>(p->np);
    const uint32_t t2 = (uint32_t)fused_dyn_lds<2, C, false, true, Mma<T>::PAIRED>(p->np);
    FusedArgs b = a;   // (Lambda from its table: bands of tiles per XCD)
    b.xcd_swizzle = pass == 1 ? XCD_ROWS : XCD_COLS;
    if (pass == 1 && tz_fits<C, 1, true>(p))
      hipLaunchKernelGGL((k_fused<T, 1, C, FUSED_NBUF, false, true, true>), grid, block, t1, p->stream, b);
    else if (pass == 2 && tz_fits<C, 2, true>(p))
      hipLaunchKernelGGL((k_fused<T, 2, C, FUSED_NBUF, false, true, true>), grid, block, t2, p->stream, b);
    else if (pass == 1)
      hipLaunchKernelGGL((k_fused<T, 1, C, FUSED_NBUF, false, true>), grid, block, l1, p->stream, a);
    else
      hipLaunchKernelGGL((k_fused<T, 2, C, FUSED_NBUF, false, true>), grid, block, l2, p->stream, a);
  }
  static fot_status adj_step(fot_plan_s* p, const void* lam, T* A, T* Bt, const AdjStep& st) {
    if constexpr (Mma<T>::PAIRED) {
      (void)p; (void)lam; (void)A; (void)Bt; (void)st;
      return fail(FOT_E_UNSUPPORTED, "reverse half-step: unsupported operand type");
    } else {
      const long long plane = (long long)p->plane;
      const double eps = st.eps;
      const dim3 pg(p->np * p->np / (256 * PREP_U), p->B);
      if (!st.have_operand)
        with_cfg(p, [&](auto c) {
          typedef decltype(c) C;
          hipLaunchKernelGGL((k_adj_prep<T, C::BN / C::XS>), pg, dim3(256), 0, p->stream, st.v, st.L, p->n, p->np, A,
                             p->kexpA);
        });
      LAUNCH_CHECK();
      FusedArgs a{};
      a.n = p->n;
      a.np = p->np;
      a.nk = (int)((size_t)p->np * sizeof(T) / FROWB);
      a.nbA = p->nbA;
      a.nbT = p->nbT;
      a.xcd_swizzle = XCD_BLOCKS;
      a.band = raw_band(p, eps);
      a.A = A;
      a.sA = plane;
      a.B = lam;
      a.sB = 0;
      a.kexp = p->kexpA;
      a.outT = Bt;
      a.kexpT = p->kexpT;
      FusedArgs b = a;
      b.A = lam;
      b.sA = 0;
      b.B = Bt;
      b.sB = plane;
      b.kexp = p->kexpT;
      b.outT = nullptr;
      b.kexpT = nullptr;
      b.lnmarg = st.lnm;
      b.sMarg = st.sMarg;
      b.pot = const_cast<double*>(st.P);   // (read only in the reverse update)
      b.eps = eps;
      b.inv_eps = 1.0 / eps;
      b.flag = p->flag;
      b.adj_out = st.out;
      b.adj_scale = st.scale;
      b.adj_coords = st.coords;
      b.adj_acc = st.acc;
      b.adj_lb = st.lb;
      b.adj_lb_scale = st.lb_scale;
      b.adj_next_L = st.next_L;
      b.nextA = A;   // (pass 1 has consumed it)
      b.kexpN = p->kexpA;
      with_cfg(p, [&](auto c) {
        typedef decltype(c) C;
        adj_launch_cfg<C>(p, 1, a);
        adj_launch_cfg<C>(p, 2, b);
      });
      LAUNCH_CHECK();
      return FOT_OK;
    }
  }

  static fot_status ensure_lambda(fot_plan_s* p, double eps) {
    if (p->lam_eps != eps) return fill_lambda(p, eps, false);
    return FOT_OK;
  }

  static fot_status backward(fot_plan_s* p, const double* dphi, double* dG) {
    const long long plane = (long long)p->plane;
    const size_t BP = (size_t)p->B * p->plane;
    const int T_ = p->last_iters, k = p->d.checkpoint_every, B = p->B, n = p->n, np = p->np;
    const std::vector<double>& e = p->last_eps;
    const int nseg = (T_ + k - 1) / k;
    fot_status s;
    const dim3 eg(256, B);
    // one reverse half-step (see adj_step): FP32 operands after an FP32 forward solve where Lambda
    // is held raw (the loop's own Lambda and operand buffers), FP64 operands otherwise.  A step may
    // also build the next one's operand when both use the same type and no replay comes between
    // (it overwrites the loop's operand buffers): `ready` tells the next step.
    auto f32_rev = [&](double eps) -> bool {
      if constexpr (std::is_same<T, float>::value) return !lam_ln(p, eps) && !(p->d.flags & FOT_FLAG_F64_REVERSE);
      (void)eps;
      return false;
    };
    bool ready = false;
    auto step = [&](AdjStep st) -> fot_status {
      if (st.next_L && f32_rev(st.next_eps) != f32_rev(st.eps)) st.next_L = nullptr;
      st.have_operand = ready;
      ready = st.next_L != nullptr;
      fot_status r;
      if constexpr (std::is_same<T, float>::value) {
        if (f32_rev(st.eps)) {
          if ((r = ensure_lambda(p, st.eps)) != FOT_OK) return r;
          return adj_step(p, p->lam, (T*)p->opA, (T*)p->opB, st);
        }
      }
      if ((r = rev_lambda(p, st.eps)) != FOT_OK) return r;
      return Ops<double>::adj_step(p, p->flam, p->fA, p->fB, st);
    };
    // seeds: fbar = dD a (the final u-update's f enters D as <f,a>), psibar = dD b
    hipLaunchKernelGGL(k_seed, dim3(256, B), dim3(256), 0, p->stream, p->dd_dev, p->lna, 0LL, n, np, p->fbar);
    hipLaunchKernelGGL(k_seed, dim3(256, B), dim3(256), 0, p->stream, p->dd_dev, p->lnb, plane, n, np, p->psibar);
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, p->stream, p->lbbar, BP, 0.0);
    LAUNCH_CHECK();
    if (dphi) {  // transpose of the integration: dL/dphi -> (dL/dTx, dL/dTy)
      hipLaunchKernelGGL(k_rowsum_dense, dim3(n, B), dim3(NTHREADS), 0, p->stream, dphi, n, p->rsum_tmp);
      hipLaunchKernelGGL(k_int_adj_rows, dim3(n, B), dim3(NTHREADS), 0, p->stream, dphi, p->rsum_tmp, p->lna, n,
                         np, p->Tby, p->cbar, p->Tbx);
      hipLaunchKernelGGL(k_int_adj_col, dim3(B), dim3(64), 0, p->stream, p->cbar, n, np, p->Tbx);
      LAUNCH_CHECK();
    }
    for (int sg = nseg - 1; sg >= 0; --sg) {
      const int t0 = sg * k, t1 = std::min(T_, t0 + k);
      const double* tape_in = p->tape + (size_t)sg * BP;
      // replay the segment from its checkpoint (bit-identical to the forward solve), unless the
      // forward solve left this one, the last, in the segment buffers
      const double* pin = tape_in;
      const bool replay = !(sg == nseg - 1 && p->seg_last_valid);
      p->seg_last_valid = false;   // (the next segments' replays overwrite the buffers)
      if (replay && (s = prep(p, tape_in, e[t0])) != FOT_OK) return s;
      for (int i = t0; i < t1 && replay; ++i) {
        const int q = i - t0;
        if ((s = ensure_lambda(p, e[i])) != FOT_OK) return s;
        // (the replay needs no marginal-error partials; the potentials do not depend on them)
        if ((s = half(p, pin, p->seg_f + q * BP, p->lna, 0, nullptr, p->seg_lnS + q * BP, e[i], e[i])) != FOT_OK)
          return s;
        if ((s = half(p, p->seg_f + q * BP, p->seg_psi + q * BP, p->lnb, plane, nullptr, p->seg_lnSp + q * BP, e[i],
                      i + 1 < t1 ? e[i + 1] : 0.0)) != FOT_OK)
          return s;
        pin = p->seg_psi + q * BP;
      }
      p->pending_hist = nullptr;
      ready = false;   // (the replay used the operand buffers)
      auto psi_in = [&](int i) -> const double* { return i > t0 ? p->seg_psi + (size_t)(i - 1 - t0) * BP : tape_in; };
      bool have_prev = false;
      if (sg == nseg - 1 && dphi) {
        // phase: Tx = Sx(V_T)/S(V_{T-1}) and Ty likewise (Eq. 9-10)
        const int i = T_ - 1, q = i - t0;
        const double ep = e[i];
        if ((s = ensure_lambda(p, ep)) != FOT_OK) return s;
        const double* lnSl = p->seg_lnS + (size_t)q * BP;
        const double* psiT = p->seg_psi + (size_t)q * BP;
        // psibar_T += (V_T / eps) [X K(Tbx / S) + Y K(Tby / S)]
        if ((s = step({p->Tbx, lnSl, psiT, ep, p->lnb, plane, 1.0 / ep, 1, 1, p->psibar})) != FOT_OK) return s;
        if ((s = step({p->Tby, lnSl, psiT, ep, p->lnb, plane, 1.0 / ep, 2, 1, p->psibar})) != FOT_OK) return s;
        // psibar_{T-1} += -(V_{T-1} / eps) K((Tbx Tx + Tby Ty) / S)
        hipLaunchKernelGGL(k_moment_weight, eg, dim3(256), 0, p->stream, p->Tbx, p->txc, p->Tby, p->Ty, n, np,
                           p->wtmp);
        LAUNCH_CHECK();
        if ((s = step({p->wtmp, lnSl, psi_in(i), ep, p->lnb, plane, -1.0 / ep, 0, 0, p->psiprev})) != FOT_OK) return s;
        have_prev = true;
      }
      for (int i = t1 - 1; i >= t0; --i) {
        const int q = i - t0;
        const double ep = e[i];
        if ((s = ensure_lambda(p, ep)) != FOT_OK) return s;
        // V-update psi_i = eps (ln b - ln S'(f_i)):  lbbar += eps psibar;  fbar += -u_i K(psibar / S')
        // (below the last iteration, the step that formed psibar has added its lbbar term)
        if (i == T_ - 1) {
          hipLaunchKernelGGL(k_axpy_masked, eg, dim3(256), 0, p->stream, p->psibar, p->lnb, n, np, ep, p->lbbar);
          LAUNCH_CHECK();
        }
        const double* lnSq = p->seg_lnS + (size_t)q * BP;
        if ((s = step({p->psibar, p->seg_lnSp + (size_t)q * BP, p->seg_f + (size_t)q * BP, ep, p->lna, 0, -1.0, 0,
                       i == T_ - 1 ? 1 : 0, p->fbar, nullptr, 0.0, i > 0 ? lnSq : nullptr, ep})) != FOT_OK)
          return s;
        // u-update f_i = eps (ln a - ln S(psi_{i-1})):  psibar_{i-1} = -V_{i-1} K(fbar / S)
        if (i > 0) {
          double* dst = p->psibar2;
          // the next step (V-update of iteration i - 1) in this segment: its operand now
          const double* nextL = i - 1 >= t0 ? p->seg_lnSp + (size_t)(q - 1) * BP : nullptr;
          if (i == T_ - 1 && have_prev) {
            if ((s = step({p->fbar, lnSq, psi_in(i), ep, p->lnb, plane, -1.0, 0, 1, p->psiprev, p->lbbar, e[i - 1],
                           nextL, e[i - 1]})) != FOT_OK)
              return s;
            dst = p->psiprev;
            p->psiprev = p->psibar;
            p->psibar = dst;
          } else {
            if ((s = step({p->fbar, lnSq, psi_in(i), ep, p->lnb, plane, -1.0, 0, 0, dst, p->lbbar, e[i - 1], nextL,
                           e[i - 1]})) != FOT_OK)
              return s;
            p->psibar2 = p->psibar;
            p->psibar = dst;
          }
        }
      }
    }
    // normalisation Jacobian: dL/dG from lbbar and the explicit dD <psi_T, b> term
    hipLaunchKernelGGL(k_grad_rows, dim3(n, B), dim3(NTHREADS), 0, p->stream, p->lbbar, p->psi, p->lnb, n, np,
                       p->gparts);
    hipLaunchKernelGGL(k_grad_sums, dim3(B), dim3(NTHREADS), 0, p->stream, p->gparts, p->dd_dev, n, p->gsums);
    hipLaunchKernelGGL(k_grad_final, dim3(256, B), dim3(256), 0, p->stream, p->rowsum_G, p->lbbar, p->psi, p->lnb,
                       p->dd_dev, p->gsums, n, np, dG);
    LAUNCH_CHECK();
    return FOT_OK;
  }

};

// ------------------------------------------------------------------ precision schedule
// Make operand set `which` (0: the head type's, 1: the tail type's) the one the kernels use.
void activate(fot_plan_s* p, int which) {
  p->lam = p->op_set[which][0];
  p->opA = p->op_set[which][1];
  p->opB = p->op_set[which][2];
}

// A solve's iterations with the precision schedule: iters - k iterations with H operands, then the
// last k = min(tail_iters, iters) with L operands (each segment builds its own operands from psi).
template <typename H, typename L>
fot_status sched_loop(fot_plan_s* p, const std::vector<double>& e, int iters) {
  const int t1 = iters - std::min(p->tail_iters, iters);
  fot_status s = FOT_OK;
  if (t1 > 0) {
    activate(p, 0);
    if ((s = Ops<H>::segment(p, e, 0, t1, iters)) != FOT_OK) return s;
  }
  activate(p, 1);
  return Ops<L>::segment(p, e, t1, iters, iters, 1);
}

template <typename H, typename L>
fot_status sched_check(fot_plan_s* p, const std::vector<double>& e, int iters) {
  const int t1 = iters - std::min(p->tail_iters, iters);
  fot_status s = Ops<H>::check_schedule(p, e, 0, t1);
  return s != FOT_OK ? s : Ops<L>::check_schedule(p, e, t1, iters);
}

// ------------------------------------------------------------------ FP64 read-out and reverse sweep
// Lambda (and Lambda o H) with FP64 elements for the read-out and the reverse sweep: Lambda's
// plane and its chunks where the plan keeps the plane, else Lambda's chunk table alone (the
// read-out's GEMMs read the tables), and Lambda o H's chunk table.
fot_status fill64(fot_plan_s* p, double eps, bool withH) {
  const bool needL = *p->flam_eps != eps;
  const bool needH = withH && (needL || !*p->flamH_valid);
  if (!needL && !needH) return FOT_OK;
  const dim3 cgrid((unsigned)((2 * p->np + 255) / 256));
  if (needL && p->flam) {
    hipLaunchKernelGGL(k_fill_lambda<double>, dim3((unsigned)((p->plane + 255) / 256)), dim3(256), 0, p->stream,
                       p->flam, (double*)nullptr, p->n, p->np, 1.0 / eps);
    hipLaunchKernelGGL(k_lam_chunks<double>, cgrid, dim3(256), 0, p->stream, p->flam, p->np);
  }
  const bool tabL = needL && !p->flam;
  if (tabL || needH)
    hipLaunchKernelGGL(k_lam_table64, cgrid, dim3(256), 0, p->stream, tabL ? p->flamT : (double*)nullptr,
                       needH ? p->flamHT : (double*)nullptr, p->n, p->np, 1.0 / eps);
  LAUNCH_CHECK();
  *p->flam_eps = eps;
  *p->flamH_valid = withH || (!needL && *p->flamH_valid);
  return FOT_OK;
}

fot_status rev_lambda(fot_plan_s* p, double eps) { return fill64(p, eps, false); }

// Phase read-out (Eq. 9-10), final marginals, dual value and transport cost, with FP64 operands,
// in four FP64 planes (fA, fB, fZ, Ty) besides the state.  f_probe: the end-of-solve probe's
// potential (in fZ) or null.
fot_status readout64(fot_plan_s* p, double eps, double* phase_out, const double* f_probe) {
  typedef Ops<double> R;
  const long long plane = (long long)p->plane;
  fot_status s;
  if ((s = fill64(p, eps, true)) != FOT_OK) return s;
  if (p->x_alias) p->x_dirty = true;
  const dim3 tgrid(p->np / TILE, p->np / TILE, p->B);
  const int rblocks = readout_blocks(p->n);
  const dim3 rgrid(rblocks, p->B), rblock(NTHREADS);
  const void* const LAM = p->flamT;
  const void* const LAMH = p->flamHT;
  // GEMM operands: a batch of planes, or Lambda / Lambda o H through their chunk tables
  auto args = [&](const void* A, const void* Bm, double* out) -> GemmArgs {
    const bool ta = A == LAM || A == LAMH, tb = Bm == LAM || Bm == LAMH;
    GemmArgs g = R::base_args(p, A, ta ? 0 : plane, Bm, tb ? 0 : plane);
    g.tzA = ta ? A : nullptr;
    g.tzB = tb ? Bm : nullptr;
    // (the 4 x 8 blocks per XCD of base_args: bands of tiles, as in the fused kernels, measured
    // slower here, 45.1 against 43.8 us per FP64 product at 1024^2)
    g.out = out;
    g.sOut = plane;
    return g;
  };
  auto gemm = [&](const void* A, const void* Bm, double* out) -> fot_status {
    return R::gemm_launch(p, EPI_RAW, args(A, Bm, out));
  };
  // Z = ln(A Lambda) with the row shifts of A's k_rowexp and the column keys gathered
  auto gemm_log = [&](const double* A, double* out) -> fot_status {
    GemmArgs g = args(A, LAM, out);
    g.mrow = p->mrow;
    g.colkey = p->colkey;
    return R::gemm_launch(p, EPI_LOGROW, g);
  };
  auto rowexp = [&](const double* P, double* out, double* out2, unsigned* keys, PendingSum ps) {
    hipLaunchKernelGGL(k_rowexp<double>, dim3(p->np, p->B), dim3(NTHREADS), 0, p->stream, P, p->n, p->np,
                       1.0 / eps, p->mrow, out, out2, keys, ps);
  };
  const PendingSum none{nullptr, 0, nullptr};
  // ln S'(f_T) = ln(Lambda . u_T . Lambda) in FP64, not the loop's value (computed with the operand
  // type), and with it the column-mass error of the returned plan: it then measures how well the
  // operand type represented the last V-update's products.
  //   A0' = exp(f/eps - m) -> fA, Z' = ln(A0' Lambda) -> Ty, B0' = colexp(Z') -> fB, S' -> fA.
  rowexp(p->f, p->fA, nullptr, p->colkey, take_pending(p));
  LAUNCH_CHECK();
  if ((s = gemm_log(p->fA, p->Ty)) != FOT_OK) return s;
  hipLaunchKernelGGL((k_colexpT<double, double, 0>), tgrid, dim3(NTHREADS), 0, p->stream, (const double*)p->Ty,
                     p->mrow, p->colkey, p->n, p->np, p->fB);
  LAUNCH_CHECK();
  if ((s = gemm(LAM, p->fB, p->fA)) != FOT_OK) return s;
  hipLaunchKernelGGL(k_colerr, rgrid, rblock, 0, p->stream, (const double*)p->fA, p->colkey, p->psi, p->lnb, p->n,
                     p->np, eps, p->rparts);
  LAUNCH_CHECK();
  // Moments of V_T (Eq. 9-10), each pass-2 output consumed (k_readout) before the next is formed:
  //   A0 = exp(psi/eps - m) -> fA, Z = ln(A0 Lambda) -> Ty (row shifts, column keys),
  //   B0 = colexp(Z) -> fB: S = Lambda B0 -> fA (consumed, with the probe's update in fZ), Scx =
  //   (Lambda o H) B0 -> fA (consumed); T_x at column 0 from Z's column 0 (k_tx_column),
  //   A0 again -> fA (keys kept), Zc = A0 (Lambda o H) -> fB, Bc = colexp(Zc) -> fZ: Scy = Lambda Bc
  //   -> fB (consumed), A2 = A0 Y -> fA, Zy = A2 Lambda -> fZ, By = colexp(Zy) -> fB: Sy = Lambda By
  //   -> Ty (T_y).
  rowexp(p->psi, p->fA, nullptr, p->colkey, none);
  LAUNCH_CHECK();
  if ((s = gemm_log(p->fA, p->Ty)) != FOT_OK) return s;
  hipLaunchKernelGGL((k_colexpT<double, double, 0>), tgrid, dim3(NTHREADS), 0, p->stream, (const double*)p->Ty,
                     p->mrow, p->colkey, p->n, p->np, p->fB);
  LAUNCH_CHECK();
  if ((s = gemm(LAM, p->fB, p->fA)) != FOT_OK) return s;
  hipLaunchKernelGGL(k_readout<RO_S>, rgrid, rblock, 0, p->stream, p->fA, p->colkey, p->lnS, p->lna, p->lnb, p->f,
                     p->psi, f_probe, p->n, p->np, eps, p->rparts);
  LAUNCH_CHECK();
  if ((s = gemm(LAMH, p->fB, p->fA)) != FOT_OK) return s;
  hipLaunchKernelGGL(k_readout<RO_CX>, rgrid, rblock, 0, p->stream, p->fA, p->colkey, p->lnS, p->lna, p->lnb, p->f,
                     p->psi, (const double*)nullptr, p->n, p->np, eps, p->rparts);
  hipLaunchKernelGGL(k_tx_column, dim3(p->n, p->B), dim3(NTHREADS), 0, p->stream, (const double*)p->Ty,
                     (const double*)p->mrow, (const unsigned*)p->colkey, (const double*)p->flamT,
                     (const double*)p->lnS, p->n, p->np, p->txc);
  rowexp(p->psi, p->fA, nullptr, (unsigned*)nullptr, none);
  LAUNCH_CHECK();
  if ((s = gemm(p->fA, LAMH, p->fB)) != FOT_OK) return s;
  hipLaunchKernelGGL((k_colexpT<double, double, 2>), tgrid, dim3(NTHREADS), 0, p->stream, (const double*)p->fB,
                     p->mrow, p->colkey, p->n, p->np, p->fZ);
  LAUNCH_CHECK();
  if ((s = gemm(LAM, p->fZ, p->fB)) != FOT_OK) return s;
  hipLaunchKernelGGL(k_readout<RO_CY>, rgrid, rblock, 0, p->stream, p->fB, p->colkey, p->lnS, p->lna, p->lnb, p->f,
                     p->psi, (const double*)nullptr, p->n, p->np, eps, p->rparts);
  // (the moment operand A2 with the row shifts of A0, which the column keys above refer to)
  rowexp(p->psi, nullptr, p->fA, p->colkey, none);
  LAUNCH_CHECK();
  if ((s = gemm(p->fA, LAM, p->fZ)) != FOT_OK) return s;
  hipLaunchKernelGGL((k_colexpT<double, double, 2>), tgrid, dim3(NTHREADS), 0, p->stream, (const double*)p->fZ,
                     p->mrow, p->colkey, p->n, p->np, p->fB);
  LAUNCH_CHECK();
  if ((s = gemm(LAM, p->fB, p->Ty)) != FOT_OK) return s;
  hipLaunchKernelGGL(k_readout<RO_TY>, rgrid, rblock, 0, p->stream, p->Ty, p->colkey, p->lnS, p->lna, p->lnb, p->f,
                     p->psi, (const double*)nullptr, p->n, p->np, eps, p->rparts);
  hipLaunchKernelGGL(k_sum_parts, dim3(READOUT_SLOTS, p->B), dim3(NTHREADS), 0, p->stream, p->rparts, rblocks,
                     p->rsums);
  hipLaunchKernelGGL(k_integrate, dim3(p->n, p->B), dim3(NTHREADS), 0, p->stream, (const double*)p->txc,
                     (const double*)p->Ty, p->lna, p->n, p->np, p->fZ, p->rowpart);
  if (phase_out)
    hipLaunchKernelGGL(k_center, dim3(p->n, p->B), dim3(NTHREADS), 0, p->stream, p->fZ, p->rowpart, p->n, p->np,
                       phase_out);
  LAUNCH_CHECK();
  return FOT_OK;
}

// ------------------------------------------------------------------ output beam (Sec. 4)
__global__ void k_flag_nonpositive(const double* v, int cnt, int* flag) {
  for (int i = threadIdx.x; i < cnt; i += blockDim.x)
    if (!(v[i] > 0.0 && v[i] < INFINITY)) atomicOr(flag, 4);
}

fot_status beam_ready(fot_plan_s* p) {
  if (p->beam_ok) return FOT_OK;   // (after a failed attempt the pointers set so far are leaked to
                                   // p->allocs and freed with the plan; a retry allocates afresh)
  const size_t wsz = (size_t)p->np * 2 * p->np, fsz = (size_t)p->B * wsz;
  fot_status s;
  double** w[4] = {&p->bWa, &p->bWb, &p->bWca, &p->bWcb};
  for (double** x : w)
    if ((s = dalloc_t(p, x, wsz)) != FOT_OK) return s;
  double** f[3] = {&p->bfc, &p->bHt, &p->bF};
  for (double** x : f) {
    if ((s = dalloc_t(p, x, fsz)) != FOT_OK) return s;
    HIP_TRY(hipMemsetAsync(*x, 0, fsz * sizeof(double), p->stream));   // padding stays zero
  }
  if ((s = dalloc_t(p, &p->bpow, (size_t)p->B)) != FOT_OK) return s;
  if ((s = dalloc_t(p, &p->bsumG, (size_t)p->B)) != FOT_OK) return s;
  if ((s = dalloc_t(p, &p->brow, (size_t)p->B * p->n)) != FOT_OK) return s;
  if ((s = dalloc_t(p, &p->bl1, (size_t)p->B)) != FOT_OK) return s;
  const size_t cells = (size_t)p->np * p->np;
  hipLaunchKernelGGL(k_dft_operands, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, p->stream, p->n, p->np,
                     p->bWa, p->bWb, p->bWca, p->bWcb);
  LAUNCH_CHECK();
  p->beam_ok = true;
  return FOT_OK;
}

// dst = F[src] (forward) or conj-F[src] (inverse, without the 1/n^2), both in the [Re | Im]
// row layout: four FP64 MFMA GEMMs with K = 2 np.
fot_status beam_dft(fot_plan_s* p, const double* src, double* dst, bool inverse) {
  const int np = p->np;
  const long long wsz = (long long)np * 2 * np;
  GemmArgs a{};
  a.n = p->n;
  a.np = np;
  a.kp = 2 * np;
  a.nk = (int)((size_t)2 * np * sizeof(double) / ROWB);
  a.ldo = 2 * np;
  a.xcd_swizzle = XCD_BLOCKS;
  a.sA = 0;
  a.sB = wsz;
  a.sOut = wsz;
  const double* Wr = inverse ? p->bWca : p->bWa;
  const double* Wi = inverse ? p->bWcb : p->bWb;
  typedef Ops<double> R;
  fot_status s;
  // step A: Ht[M][j] = sum_k W[M][k] f[j][k]
  a.B = src;
  a.A = Wr;
  a.out = p->bHt;
  if ((s = R::gemm_launch(p, EPI_RAW, a)) != FOT_OK) return s;
  a.A = Wi;
  a.out = p->bHt + np;
  if ((s = R::gemm_launch(p, EPI_RAW, a)) != FOT_OK) return s;
  // step B: F[L][M] = sum_j W[L][j] Ht[M][j]
  a.B = p->bHt;
  a.A = Wr;
  a.out = dst;
  if ((s = R::gemm_launch(p, EPI_RAW, a)) != FOT_OK) return s;
  a.A = Wi;
  a.out = dst + np;
  return R::gemm_launch(p, EPI_RAW, a);
}

// Row sums of g^2 (and of G^2 if given) with input validation, 1 / (n^2 sum g^2) per target,
// sum G^2 per target; flag bits 2 (negative or non-finite amplitude) and 4 (zero total).
fot_status beam_inputs(fot_plan_s* p, const double* g, const double* G) {
  const int n = p->n, B = p->B;
  HIP_TRY(hipMemsetAsync(p->flag, 0, sizeof(int), p->stream));
  hipLaunchKernelGGL(k_rowsumsq, dim3(n, 1), dim3(NTHREADS), 0, p->stream, g, n, p->rowsum_g, p->flag);
  hipLaunchKernelGGL(k_inv_power, dim3(1), dim3(NTHREADS), 0, p->stream, p->rowsum_g, n, B, p->bpow);
  hipLaunchKernelGGL(k_flag_nonpositive, dim3(1), dim3(NTHREADS), 0, p->stream, p->bpow, B, p->flag);
  if (G) {
    hipLaunchKernelGGL(k_rowsumsq, dim3(n, B), dim3(NTHREADS), 0, p->stream, G, n, p->rowsum_G, p->flag);
    hipLaunchKernelGGL(k_sum_rows, dim3(B), dim3(NTHREADS), 0, p->stream, p->rowsum_G, n, p->bsumG);
    hipLaunchKernelGGL(k_flag_nonpositive, dim3(1), dim3(NTHREADS), 0, p->stream, p->bsumG, B, p->flag);
  }
  LAUNCH_CHECK();
  return FOT_OK;
}

fot_status beam_flag(fot_plan_s* p, const char* who) {
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (hflag & 2) return fail(FOT_E_INVALID, std::string(who) + ": amplitudes must be finite and >= 0");
  if (hflag & 4) return fail(FOT_E_INVALID, std::string(who) + ": an image has zero (or non-finite) total intensity");
  return FOT_OK;
}

// ------------------------------------------------------------------ cFOT (Eq. 11)
// One cFOT pass, with HIP-event timing under FOT_FLAG_PROFILE (counted like the fused passes).
template <typename K, typename... Args>
fot_status cfot_launch(fot_plan_s* p, K kernel, Args... args) {
  const dim3 grid((unsigned)((p->n + 1) / 2), (unsigned)p->B);
  const bool prof = (p->d.flags & FOT_FLAG_PROFILE) && p->prof_used + 2 <= (int)p->prof.size();
  hipEvent_t e0 = prof ? p->prof[p->prof_used] : nullptr;
  hipEvent_t e1 = prof ? p->prof[p->prof_used + 1] : nullptr;
  hipExtLaunchKernelGGL(kernel, grid, dim3(CFOT_THREADS), (uint32_t)cfot_lds_bytes(p->cN), p->stream, e0, e1, 0,
                        args...);
  LAUNCH_CHECK();
  if (prof) p->prof_used += 2;
  return FOT_OK;
}

// fn(std::integral_constant<int, N>) for the plan's FFT length
template <typename F>
fot_status cfot_dispatch(int N, F&& fn) {
  switch (N) {
    case 256: return fn(std::integral_constant<int, 256>{});
    case 512: return fn(std::integral_constant<int, 512>{});
    case 1024: return fn(std::integral_constant<int, 1024>{});
    case 2048: return fn(std::integral_constant<int, 2048>{});
    case 4096: return fn(std::integral_constant<int, 4096>{});
    default: return fail(FOT_E_UNSUPPORTED, "cFOT: unsupported FFT length");
  }
}

// One half-step by convolutions: Pin (one orientation) -> Pout (the other), Eq. 7 or 8.  The
// marginal-error partials of this half-step are summed into hist by the next half-step's first
// pass (p->pending_hist), or by cfot_finish_pending at the end of the loop.
fot_status cfot_half(fot_plan_s* p, const double* Pin, double* Pout, const double* lnm, long long sMarg,
                     double* hist, double* lnS_out, double eps) {
  const long long plane = (long long)p->plane;
  double* pend_out = p->pending_hist;
  p->pending_hist = nullptr;
  const int cnt = (p->n + 1) / 2;
  fot_status s = cfot_dispatch(p->cN, [&](auto nc) -> fot_status {
    constexpr int N = decltype(nc)::value;
    fot_status r = cfot_launch(p, k_cfot_pass1<N>, Pin, plane, 1.0 / eps, p->n, p->np, (const cplx*)p->ctw,
                               (const double*)p->clamhat, p->cY, plane,
                               pend_out ? (const double*)p->cparts : (const double*)nullptr, cnt, pend_out);
    if (r != FOT_OK) return r;
    return cfot_launch(p, k_cfot_pass2<N>, (const double*)p->cY, plane, p->n, p->np, (const cplx*)p->ctw,
                       (const double*)p->clamhat, lnm, sMarg, Pout, plane, lnS_out, eps, p->cparts, p->flag,
                       hist != nullptr ? 1 : 0);
  });
  if (s != FOT_OK) return s;
  p->pending_hist = hist;
  return FOT_OK;
}

fot_status cfot_finish_pending(fot_plan_s* p) {
  if (!p->pending_hist) return FOT_OK;
  hipLaunchKernelGGL(k_cfot_sum, dim3(p->B), dim3(NTHREADS), 0, p->stream, (const double*)p->cparts,
                     (p->n + 1) / 2, p->pending_hist);
  LAUNCH_CHECK();
  p->pending_hist = nullptr;
  return FOT_OK;
}

fot_status cfot_transpose(fot_plan_s* p, const double* in, long long sIn, double* out, long long sOut, int batch) {
  const unsigned t = (unsigned)((p->n + 31) / 32);
  hipLaunchKernelGGL(k_transpose64, dim3(t, t, batch), dim3(256), 0, p->stream, in, sIn, out, sOut, p->n, p->np);
  LAUNCH_CHECK();
  return FOT_OK;
}

// The iteration loop of Algorithm 1 with convolutions: f is carried transposed (with ln a
// transposed to match) and restored to the natural layout at the end, with ln S of the last
// u-update, so the read-out and the potentials API see the same state as after the GEMM loop.
fot_status cfot_loop(fot_plan_s* p, const std::vector<double>& e, int iters) {
  const long long plane = (long long)p->plane;
  const int B = p->B;
  fot_status s;
  p->pending_hist = nullptr;
  if ((s = cfot_transpose(p, p->lna, 0, p->clnaT, 0, 1)) != FOT_OK) return s;
  if ((s = cfot_transpose(p, p->f, plane, p->cfT, plane, B)) != FOT_OK) return s;
  const bool hist = !(p->d.flags & FOT_FLAG_NO_HISTORY);
  for (int t = 0; t < iters; ++t) {
    const double ep = e[t];
    if (t == 0 || ep != e[t - 1]) {
      s = cfot_dispatch(p->cN, [&](auto nc) -> fot_status {
        constexpr int N = decltype(nc)::value;
        hipLaunchKernelGGL(k_cfot_lamhat<N>, dim3(1), dim3(CFOT_THREADS), (uint32_t)cfot_lds_bytes(N), p->stream,
                           p->n, 1.0 / ep, (const cplx*)p->ctw, p->clamhat);
        LAUNCH_CHECK();
        return FOT_OK;
      });
      if (s != FOT_OK) return s;
    }
    const bool last = t == iters - 1;
    if ((s = cfot_half(p, p->psi, p->cfT, p->clnaT, 0, hist ? p->hist_a + (size_t)t * B : nullptr,
                       last ? p->cS : nullptr, ep)) != FOT_OK)
      return s;
    if ((s = cfot_half(p, p->cfT, p->psi, p->lnb, plane, hist ? p->hist_b + (size_t)t * B : nullptr,
                       nullptr, ep)) != FOT_OK)
      return s;
  }
  if ((s = cfot_finish_pending(p)) != FOT_OK) return s;
  if ((s = cfot_transpose(p, p->cfT, plane, p->f, plane, B)) != FOT_OK) return s;
  if ((s = cfot_transpose(p, p->cS, plane, p->lnS, plane, B)) != FOT_OK) return s;
  p->clam_eps = e[iters - 1];
  return FOT_OK;
}

fot_status cfot_loop_graph(fot_plan_s* p, const std::vector<double>& e, int iters) {
  fot_status s = run_graph(p, e, iters, [](fot_plan_s* q, const std::vector<double>& ee, int it) {
    return cfot_loop(q, ee, it);
  });
  if (s == FOT_OK && p->used_graph) {
    p->clam_eps = e[iters - 1];
    p->pending_hist = nullptr;
  }
  return s;
}

fot_status sched_loop_graph_state(fot_plan_s* p, const std::vector<double>& e, int iters) {
  // state after a replayed loop, as if it had been launched directly
  p->pending_hist = (p->d.flags & FOT_FLAG_NO_HISTORY) ? nullptr : p->hist_b + (size_t)(iters - 1) * p->B;
  p->lam_eps = e[iters - 1];
  p->lamH_valid = false;
  return FOT_OK;
}

// One solve after set-up: the iteration loop (operand type H throughout, or the precision schedule
// H then L), the end-of-solve probe of the final type's products, and the FP64 read-out.
template <typename H, typename L>
fot_status solve_body(fot_plan_s* p, const std::vector<double>& e, int iters, double* phase_out) {
  constexpr bool sched = !std::is_same<H, L>::value;
  if (p->x_dirty) {
    // the last read-out used the operand buffers as an FP64 plane: the padded borders, which the
    // loop kernels read as zeros and never write, are cleared again (no borders when n = n_p)
    if (p->np > p->n &&
        hipMemsetAsync(p->op_set[0][1], 0, 2 * (size_t)p->B * p->plane * p->esz, p->stream) != hipSuccess)
      return fail(FOT_E_HIP, "fot_solve: memset failed");
    p->x_dirty = false;
  }
  if (p->ev[1]) HIP_TRY(hipEventRecord(p->ev[1], p->stream));
  const bool graph = !(p->d.flags & (FOT_FLAG_NO_GRAPH | FOT_FLAG_PROFILE)) && !p->graph_broken && p->cap;
  p->used_graph = false;
  fot_status s;
  if (p->cfot) {
    s = graph ? cfot_loop_graph(p, e, iters) : cfot_loop(p, e, iters);
  } else if constexpr (sched) {
    if (graph) {
      s = run_graph(p, e, iters, [](fot_plan_s* q, const std::vector<double>& ee, int it) {
        return sched_loop<H, L>(q, ee, it);
      });
      if (s == FOT_OK && p->used_graph) s = sched_loop_graph_state(p, e, iters);
    } else {
      s = sched_loop<H, L>(p, e, iters);
    }
    activate(p, 1);   // the final iterations' operand type (a replayed graph issues nothing here)
  } else {
    s = graph ? Ops<H>::loop_graph(p, e, iters) : Ops<H>::loop(p, e, iters);
  }
  if (s == FOT_OK && p->ev[2])
    s = (hipEventRecord(p->ev[2], p->stream) == hipSuccess) ? FOT_OK : fail(FOT_E_HIP, "event record");
  const bool probed = !p->cfot && sizeof(L) != 8;
  if (s == FOT_OK && probed) s = Ops<L>::probe(p, e[iters - 1], iters, sched ? 1 : 0);
  if (s == FOT_OK) s = readout64(p, e[iters - 1], phase_out, probed ? p->fZ : nullptr);
  if (s == FOT_OK && p->ev[3])
    s = (hipEventRecord(p->ev[3], p->stream) == hipSuccess) ? FOT_OK : fail(FOT_E_HIP, "event record");
  activate(p, 0);
  return s;
}

template <typename F>
fot_status dispatch(int prec, F&& fn) {
  switch (prec) {
    case FOT_F64: return fn((double)0);
    case FOT_F32: return fn((float)0);
    case FOT_BF16: return fn((__bf16)0);
    case FOT_F16: return fn((_Float16)0);
    case FOT_BF16X3: return fn(bf16x3{});
    default: return fail(FOT_E_UNSUPPORTED, "unknown precision");
  }
}

bool finite_positive(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

// Checks of a plan descriptor (fot_plan's argument errors); *cN_out gets the cFOT FFT length (0: none).
static fot_status validate_desc(const fot_plan_desc& d, int* cN_out) {
  if (d.n < 1 || d.n > 8192) return fail(FOT_E_INVALID, "fot_plan: n must be in [1, 8192]");
  if (d.batch < 1 || d.batch > 65535) return fail(FOT_E_INVALID, "fot_plan: batch must be in [1, 65535]");
  if (d.precision < FOT_F64 || d.precision > FOT_BF16X3) return fail(FOT_E_INVALID, "fot_plan: unknown precision");
  if (d.max_iters < 1) return fail(FOT_E_INVALID, "fot_plan: max_iters must be >= 1");
  if (d.checkpoint_every < 0) return fail(FOT_E_INVALID, "fot_plan: checkpoint_every must be >= 0");
  if (d.flags & ~(FOT_FLAG_PROFILE | FOT_FLAG_NO_GRAPH | FOT_FLAG_NO_HISTORY | FOT_FLAG_CFOT | FOT_FLAG_SMALL_TILES |
                  FOT_FLAG_F64_REVERSE | FOT_FLAG_STAGED_LAMBDA))
    return fail(FOT_E_INVALID, "fot_plan: unknown flag bits");
  if (d.tail_iters < 0) return fail(FOT_E_INVALID, "fot_plan: tail_iters must be >= 0");
  if (d.tail_iters > 0) {
    if (d.tail_precision < FOT_F64 || d.tail_precision > FOT_BF16X3)
      return fail(FOT_E_INVALID, "fot_plan: unknown tail_precision");
    if (d.tail_precision == d.precision)
      return fail(FOT_E_INVALID, "fot_plan: tail_precision equals precision (use tail_iters = 0)");
    if (d.precision == FOT_F64)
      return fail(FOT_E_UNSUPPORTED, "fot_plan: a precision schedule starts with a 32- or 16-bit operand type");
    if (d.flags & FOT_FLAG_CFOT) return fail(FOT_E_UNSUPPORTED, "fot_plan: FOT_FLAG_CFOT has no precision schedule");
    if (d.checkpoint_every > 0)
      return fail(FOT_E_UNSUPPORTED, "fot_plan: no reverse mode with a precision schedule (checkpoint_every must be 0)");
  }
  int cN = 0;
  if (d.flags & FOT_FLAG_CFOT) {
    if (d.precision != FOT_F64) return fail(FOT_E_UNSUPPORTED, "fot_plan: FOT_FLAG_CFOT needs FOT_F64 (FP64 FFTs)");
    if (d.checkpoint_every > 0)
      return fail(FOT_E_UNSUPPORTED, "fot_plan: FOT_FLAG_CFOT has no reverse mode (checkpoint_every must be 0)");
    cN = CFOT_MIN_N;
    while (cN < 2 * d.n - 1) cN <<= 1;
    if (cN > CFOT_MAX_N) return fail(FOT_E_UNSUPPORTED, "fot_plan: FOT_FLAG_CFOT supports n <= 2048");
  }
  *cN_out = cN;
  return FOT_OK;
}

// Build plan *p (default-constructed) for descriptor d (already validated; cN its FFT length) on
// `stream`.  With `arena` non-null every device buffer is carved from its `cap` bytes instead of
// hipMalloc, and no HIP event or capture stream is created (such a plan launches eagerly and
// reports no timing).  On failure the caller releases *p.
static fot_status plan_init(fot_plan_s* p, const fot_plan_desc& d, int cN, hipStream_t stream, unsigned char* arena,
                            size_t cap) {
  const bool tail = d.tail_iters > 0;
  p->arena = arena;
  p->arena_cap = cap;
  p->arena_used = 0;
  p->d = d;
  p->n = d.n;
  auto esz_of = [](int prec) -> size_t {
    return prec == FOT_F64 ? 8 : (prec == FOT_F32 || prec == FOT_BF16X3) ? 4 : 2;
  };
  p->tail_prec = tail ? d.tail_precision : -1;
  p->tail_iters = tail ? d.tail_iters : 0;
  p->esz = tail ? std::max(esz_of(d.precision), esz_of(d.tail_precision)) : esz_of(d.precision);
  const size_t esz_min = tail ? std::min(esz_of(d.precision), esz_of(d.tail_precision)) : p->esz;
  // padded side: whole 64-pixel tiles and whole K stages of the fused kernels (FROWB bytes,
  // a multiple of the read-out GEMM's ROWB) for every operand type of the plan
  static_assert(FROWB % ROWB == 0, "fused stages must also be whole read-out stages");
  const int align = std::max(TILE, (int)(FROWB / esz_min));
  p->np = ((d.n + align - 1) / align) * align;
  p->B = d.batch;
  p->prec = d.precision;
  p->zsz = (d.precision == FOT_F64 || p->tail_prec == FOT_F64) ? 8 : 4;
  p->plane = (size_t)p->np * p->np;
  p->stream = stream;
  auto bail = [](fot_status s) { return s; };
  if (hipGetDevice(&p->device) != hipSuccess) return bail(fail(FOT_E_HIP, "fot_plan: no HIP device"));
  // fused-kernel tiles: 64 x 64, or 32 x 32 when 64 x 64 tiles would occupy at most half of the
  // CUs.  Measured FP32 half-steps (pass 1 + pass 2), 32 x 32 against 64 x 64 tiles on 256 CUs:
  // 512^2 17 against 32 us, 640^2 27 against 38 us, 768^2 45 against 43 us (BF16 26 against
  // 20 us), 1024^2 73 against 57 us.  FOT_FLAG_SMALL_TILES asks for 32-wide exponent blocks: the
  // 32 x 32 tiles where they are chosen anyway, 64 x 64 tiles with two blocks per tile otherwise.
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
      hipDeviceGetAttribute(&p->lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess)
    return bail(fail(FOT_E_HIP, "fot_plan: cannot query the device"));
  const bool small = 2LL * d.batch * (p->np / Ops<float>::GC::BM) * (p->np / Ops<float>::GC::BN) <= (long long)cus;
  p->tcfg = small ? TCFG_SMALL : (d.flags & FOT_FLAG_SMALL_TILES) ? TCFG_BLOCK32 : TCFG_LARGE;
  if (p->tcfg == TCFG_BLOCK32) {
    // the block-normalised Lambda's exponent table takes twice the LDS with 32-wide blocks on 64 x 64
    // tiles: where it would not fit beside the stage buffers, the 32 x 32 tiles serve the flag
    hipFuncAttributes fa{};
    typedef Ops<float>::GC2 C;
    if (hipFuncGetAttributes(&fa, (const void*)k_fused<float, 2, C, FUSED_NBUF, true>) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(FOT_E_HIP, "fot_plan: cannot query the fused kernel"));
    }
    if (fa.sharedSizeBytes + fused_dyn_lds<2, C, true>(p->np) > (size_t)p->lds_limit) p->tcfg = TCFG_SMALL;
  }
  int tbm = 0, tbn = 0, txs = 1;
  Ops<float>::with_cfg(p, [&](auto c) {
    typedef decltype(c) C;
    tbm = C::BM;
    tbn = C::BN;
    txs = C::XS;
  });
  // one marginal-error partial per output tile of the fused pass-2 kernel
  p->tiles = (p->np / tbm) * (p->np / tbn);
  const size_t BP = (size_t)p->B * p->plane;
  const bool tape = d.checkpoint_every > 0;
  const size_t chunk64 = toeplitz_chunks_bytes(p->np) / sizeof(double);   // FP64 chunk table, in doubles
  // (the read-out's fourth plane: the loop's two operand buffers where they hold 4-byte elements
  // and nothing else needs them after the loop)
  p->x_alias = !tape && !tail && p->esz == 4;
  if (d.checkpoint_every > 0) p->n_ckpt = (d.max_iters + d.checkpoint_every - 1) / d.checkpoint_every;
  const size_t kseg = tape ? (size_t)std::min(d.checkpoint_every, d.max_iters) : 0;
  // Every device buffer of the plan, carved in order from one piece of memory (see dalloc).
  auto carve = [&]() -> fot_status {
    fot_status s = FOT_OK;
#define ALLOC(ptr, cnt)                                       \
  if ((s = dalloc_t(p, &(ptr), (cnt))) != FOT_OK) return s;
#define ALLOCV(ptr, bytes)                                    \
  if ((s = dalloc(p, &(ptr), (bytes))) != FOT_OK) return s;
    ALLOC(p->f, BP);
    ALLOC(p->psi, BP);
    ALLOC(p->lna, p->plane);
    ALLOC(p->lnb, BP);
    ALLOC(p->lnS, BP);
    ALLOC(p->mrow, (size_t)p->B * p->np);
    ALLOC(p->rowsum_g, (size_t)p->n);
    ALLOC(p->rowsum_G, (size_t)p->B * p->n);
    ALLOC(p->rowpart, (size_t)p->B * p->n);
    ALLOC(p->partials, (size_t)p->B * p->tiles);
    p->pending_parts = p->partials;
    p->pending_tiles = p->tiles;
    ALLOC(p->hist_a, (size_t)d.max_iters * p->B);
    ALLOC(p->hist_b, (size_t)d.max_iters * p->B);
    ALLOC(p->rparts, (size_t)READOUT_SLOTS * p->B * READOUT_BLOCKS);
    ALLOC(p->rsums, (size_t)READOUT_SLOTS * p->B);
    ALLOC(p->probe_flag, (size_t)1);
    // (the most waves any iteration kernel has per target: 32 x 32 tiles of 4 waves)
    p->range_spt = (p->np / 32) * (p->np / 32) * 4;
    ALLOC(p->range_slots, (size_t)2 * p->B * p->range_spt * 2);
    ALLOC(p->colkey, (size_t)p->B * p->np);
    p->nbA = p->np / (tbn / txs);
    p->nbT = p->np / (tbm / txs);
    ALLOC(p->kexpA, (size_t)p->B * p->np * p->nbA);
    ALLOC(p->kexpT, (size_t)p->B * p->np * p->nbT);
    if (d.precision != FOT_F64) ALLOC(p->kexpL, (size_t)p->np * p->nbA);
    ALLOC(p->flag, (size_t)1);
    // (each Lambda plane is followed by its Toeplitz chunks, see toeplitz_chunks_bytes)
    const bool paired = d.precision == FOT_BF16X3 || (tail && d.tail_precision == FOT_BF16X3);
    const size_t lam_bytes = p->plane * p->esz + toeplitz_chunks_bytes(p->np, paired);
    ALLOCV(p->lam, lam_bytes);
    // the two operand buffers as one piece (with x_alias also the read-out's FP64 plane Ty)
    ALLOCV(p->opA, 2 * BP * p->esz);
    p->opB = (unsigned char*)p->opA + BP * p->esz;
    p->op_set[0][0] = p->lam;
    p->op_set[0][1] = p->opA;
    p->op_set[0][2] = p->opB;
    if (tail) {
      ALLOCV(p->op_set[1][0], lam_bytes);
      ALLOCV(p->op_set[1][1], BP * p->esz);
      ALLOCV(p->op_set[1][2], BP * p->esz);
    }
    if (d.precision == FOT_F64) ALLOCV(p->Z, BP * p->zsz);   // (the FP64 read-out's fZ)
    if (d.precision == FOT_F64) {
      p->flam = (double*)p->lam;
      p->flamT = p->flam + p->plane;
      p->fA = (double*)p->opA;
      p->fB = (double*)p->opB;
      p->fZ = (double*)p->Z;
      p->flam_eps = &p->lam_eps;
      p->flamH_valid = &p->lamH_valid;
    } else {
      if (tape) {
        ALLOC(p->flam, p->plane + chunk64);
        p->flamT = p->flam + p->plane;
      } else {
        p->flam = nullptr;
        ALLOC(p->flamT, chunk64);
      }
      ALLOC(p->fA, BP);
      ALLOC(p->fB, BP);
      ALLOC(p->fZ, BP);
      p->flam_eps = &p->flam_eps_sep;
      p->flamH_valid = &p->flamH_valid_sep;
    }
    ALLOC(p->flamHT, chunk64);
    ALLOC(p->txc, (size_t)p->B * p->np);
    if (p->x_alias)
      p->Ty = (double*)p->opA;
    else
      ALLOC(p->Ty, BP);
    if (cN > 0) {
      void* tw = nullptr;
      ALLOCV(tw, sizeof(cplx) * (size_t)cfot_tw_count(cN));
      p->ctw = (cplx*)tw;
      ALLOC(p->clamhat, (size_t)cN);
      ALLOC(p->cY, BP);
      ALLOC(p->cfT, BP);
      ALLOC(p->clnaT, p->plane);
      ALLOC(p->cS, BP);
      ALLOC(p->cparts, (size_t)p->B * ((p->n + 1) / 2));
    }
    if (tape) {
      ALLOC(p->tape, (size_t)p->n_ckpt * BP);
      ALLOC(p->fbar, BP);
      ALLOC(p->psibar, BP);
      ALLOC(p->psibar2, BP);
      ALLOC(p->psiprev, BP);
      ALLOC(p->lbbar, BP);
      ALLOC(p->Tbx, BP);
      ALLOC(p->Tby, BP);
      ALLOC(p->wtmp, BP);
      ALLOC(p->cbar, (size_t)p->B * p->n);
      ALLOC(p->rsum_tmp, (size_t)p->B * p->n);
      ALLOC(p->gsums, (size_t)2 * p->B);
      ALLOC(p->gparts, (size_t)2 * p->B * p->n);
      ALLOC(p->dd_dev, (size_t)p->B);
      ALLOC(p->seg_f, kseg * BP);
      ALLOC(p->seg_psi, kseg * BP);
      ALLOC(p->seg_lnS, kseg * BP);
      ALLOC(p->seg_lnSp, kseg * BP);
    }
#undef ALLOC
#undef ALLOCV
    return s;
  };
  fot_status s = FOT_OK;
  if (!arena) {
    // one hipMalloc of the exact total (a sizing pass first): no per-buffer rounding of the
    // allocator; later buffers (the output-beam workspace) are allocated on their own
    p->sizing = true;
    s = carve();
    p->sizing = false;
    if (s != FOT_OK) return bail(s);
    void* block = nullptr;
    if ((s = dalloc(p, &block, p->arena_used)) != FOT_OK) return bail(s);
    p->arena = (unsigned char*)block;
    p->arena_cap = p->arena_used;
    p->arena_used = 0;
    s = carve();
    p->arena = nullptr;
    p->arena_cap = p->arena_used = 0;
    if (s != FOT_OK) return bail(s);
  } else if ((s = carve()) != FOT_OK) {
    return bail(s);
  }
  if (cN > 0) {
    p->cfot = true;
    p->cN = cN;
    const int lds = (int)cfot_lds_bytes(cN);
    s = cfot_dispatch(cN, [&](auto nc) -> fot_status {
      constexpr int N = decltype(nc)::value;
      if (hipFuncSetAttribute((const void*)k_cfot_pass1<N>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
              hipSuccess ||
          hipFuncSetAttribute((const void*)k_cfot_pass2<N>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
              hipSuccess ||
          hipFuncSetAttribute((const void*)k_cfot_lamhat<N>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
              hipSuccess)
        return fail(FOT_E_HIP, "fot_plan: cannot reserve LDS for the FFT kernels");
      return FOT_OK;
    });
    if (s != FOT_OK) return bail(s);
    hipLaunchKernelGGL(k_cfot_twiddles, dim3((unsigned)((cfot_tw_count(cN) + 255) / 256)), dim3(256), 0, p->stream,
                       cN, p->ctw);
    if (hipGetLastError() != hipSuccess) return bail(fail(FOT_E_HIP, "fot_plan: twiddle kernel launch failed"));
  }
  // the fused loop kernels never write the padded borders of their operands: zero them once
  for (int set = 0; set < (tail ? 2 : 1); ++set)
    for (int k = 1; k < 3; ++k)
      if (p->op_set[set][k] && hipMemsetAsync(p->op_set[set][k], 0, BP * p->esz, p->stream) != hipSuccess)
        return bail(fail(FOT_E_HIP, "fot_plan: memset failed"));
  if (hipMemsetAsync(p->kexpA, 0, sizeof(int) * p->B * p->np * p->nbA, p->stream) != hipSuccess ||
      hipMemsetAsync(p->kexpT, 0, sizeof(int) * p->B * p->np * p->nbT, p->stream) != hipSuccess ||
      hipMemsetAsync(p->colkey, 0, sizeof(unsigned) * p->B * p->np, p->stream) != hipSuccess ||
      hipMemsetAsync(p->flag, 0, sizeof(int), p->stream) != hipSuccess)
    return bail(fail(FOT_E_HIP, "fot_plan: memset failed"));
  if (!arena) {
    for (auto& e : p->ev)
      if (hipEventCreate(&e) != hipSuccess) return bail(fail(FOT_E_HIP, "fot_plan: event create failed"));
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(FOT_E_HIP, "fot_plan: stream create failed"));
  }
  if (d.flags & FOT_FLAG_PROFILE) {
    const size_t ne = 2 * ((size_t)d.max_iters * 4 + 16);
    p->prof.resize(ne, nullptr);
    for (auto& e : p->prof)
      if (hipEventCreate(&e) != hipSuccess) return bail(fail(FOT_E_HIP, "fot_plan: event create failed"));
  }
  if (hipStreamSynchronize(p->stream) != hipSuccess) return bail(fail(FOT_E_HIP, "fot_plan: sync failed"));
  return FOT_OK;
}


// ------------------------------------------------------------------ static scratch (fot_solve_noalloc)
// Device workspace for callers that cannot allocate: one array per GPU, held until the process
// ends.  Host code never uses the array's name as an address (it is a host-side stand-in); the
// device address comes from hipGetSymbolAddress, once per device with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

static fot_status scratch_of_current_device(unsigned char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(FOT_E_HIP, "fot_solve_noalloc: no usable HIP device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FOT_E_HIP, std::string("fot_solve_noalloc: hipGetSymbolAddress of the scratch array: ") +
                                 hipGetErrorString(e));
    g_scratch_ptr[dev] = (unsigned char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return FOT_OK;
}

// ====================================================================== C ABI
extern "C" {

const char* fot_last_error(void) { return g_err.c_str(); }

const char* fot_version(void) { return "fot 0.1 gfx950"; }

fot_status fot_plan(const fot_plan_desc* desc, void* stream, fot_plan_t* out) {
  g_err.clear();
  if (!desc || !out) return fail(FOT_E_INVALID, "fot_plan: null argument");
  int cN = 0;
  fot_status s = validate_desc(*desc, &cN);
  if (s != FOT_OK) return s;
  fot_plan_s* p = new (std::nothrow) fot_plan_s();
  if (!p) return fail(FOT_E_NOMEM, "fot_plan: host allocation failed");
  s = plan_init(p, *desc, cN, (hipStream_t)stream, nullptr, 0);
  if (s != FOT_OK) {
    const std::string msg = g_err;
    release(p);
    delete p;
    g_err = msg;
    return s;
  }
  *out = p;
  return FOT_OK;
}

fot_status fot_destroy(fot_plan_t p) {
  g_err.clear();
  if (!p) return fail(FOT_E_INVALID, "fot_destroy: null plan");
  (void)hipStreamSynchronize(p->stream);
  release(p);
  delete p;
  return FOT_OK;
}

fot_status fot_potentials(fot_plan_t p, double* f_out, double* psi_out, const double* f_in, const double* psi_in) {
  g_err.clear();
  if (!p) return fail(FOT_E_INVALID, "fot_potentials: null plan");
  const size_t n = p->n, np = p->np;
  const size_t rows = (size_t)p->B * n;
  // the padded planes are stacked, so one 2-D copy per batch entry keeps the pitches simple
  for (int b = 0; b < p->B; ++b) {
    const size_t po = (size_t)b * p->plane, co = (size_t)b * n * n;
    if (f_out)
      HIP_TRY(hipMemcpy2DAsync(f_out + co, n * 8, p->f + po, np * 8, n * 8, n, hipMemcpyDeviceToDevice, p->stream));
    if (psi_out)
      HIP_TRY(hipMemcpy2DAsync(psi_out + co, n * 8, p->psi + po, np * 8, n * 8, n, hipMemcpyDeviceToDevice,
                               p->stream));
  }
  (void)rows;
  if (f_in || psi_in) {
    if (!p->has_state) {
      const size_t total = (size_t)p->B * p->plane;
      const int blocks = (int)((total + 255) / 256);
      const double v0 = -INFINITY;
      if (!f_in) hipLaunchKernelGGL(k_fill_pot, dim3(blocks), dim3(256), 0, p->stream, p->f, p->n, p->np, p->B, v0);
      if (!psi_in)
        hipLaunchKernelGGL(k_fill_pot, dim3(blocks), dim3(256), 0, p->stream, p->psi, p->n, p->np, p->B, v0);
      LAUNCH_CHECK();
    }
    for (int b = 0; b < p->B; ++b) {
      const size_t po = (size_t)b * p->plane, co = (size_t)b * n * n;
      if (f_in)
        HIP_TRY(hipMemcpy2DAsync(p->f + po, np * 8, f_in + co, n * 8, n * 8, n, hipMemcpyDeviceToDevice, p->stream));
      if (psi_in)
        HIP_TRY(hipMemcpy2DAsync(p->psi + po, np * 8, psi_in + co, n * 8, n * 8, n, hipMemcpyDeviceToDevice,
                                 p->stream));
    }
    p->has_state = true;
    p->tape_valid = false;
  }
  return FOT_OK;
}

fot_status fot_solve(fot_plan_t p, const double* g, const double* G, const double* eps, int n_eps, int iters,
                     int warm_start, double* phase_out, fot_report* rep) {
  g_err.clear();
  if (!p || !g || !G || !eps) return fail(FOT_E_INVALID, "fot_solve: null argument");
  if (iters < 1 || iters > p->d.max_iters) return fail(FOT_E_INVALID, "fot_solve: iters must be in [1, max_iters]");
  if (n_eps != 1 && n_eps != iters) return fail(FOT_E_INVALID, "fot_solve: n_eps must be 1 or iters");
  for (int i = 0; i < n_eps; ++i)
    if (!finite_positive(eps[i])) return fail(FOT_E_INVALID, "fot_solve: eps must be finite and > 0");
  if (warm_start && !p->has_state) return fail(FOT_E_STATE, "fot_solve: warm start without potentials");
  std::vector<double> e(iters);
  for (int t = 0; t < iters; ++t) e[t] = eps[n_eps == 1 ? 0 : t];
  if (!p->cfot) {
    const fot_status sc =
        p->tail_iters > 0
            ? dispatch(p->prec, [&](auto h) -> fot_status {
                return dispatch(p->tail_prec, [&](auto l) -> fot_status {
                  return sched_check<decltype(h), decltype(l)>(p, e, iters);
                });
              })
            : dispatch(p->prec, [&](auto tag) -> fot_status {
                return Ops<decltype(tag)>::check_schedule(p, e, 0, iters);
              });
    if (sc != FOT_OK) return sc;
  }
  const int n = p->n, np = p->np, B = p->B;
  p->prof_used = 0;
  p->tape_valid = false;
  p->seg_last_valid = false;
  p->pending_hist = nullptr;

  if (p->ev[0]) HIP_TRY(hipEventRecord(p->ev[0], p->stream));
  HIP_TRY(hipMemsetAsync(p->flag, 0, sizeof(int), p->stream));
  HIP_TRY(hipMemsetAsync(p->probe_flag, 0, sizeof(int), p->stream));
  // 0x7f7f7f7f: nothing recorded
  HIP_TRY(hipMemsetAsync(p->range_slots, 0x7f, sizeof(int) * 2 * B * p->range_spt * 2, p->stream));
  hipLaunchKernelGGL(k_rowsumsq, dim3(n, 1), dim3(NTHREADS), 0, p->stream, g, n, p->rowsum_g, p->flag);
  hipLaunchKernelGGL(k_logmarg, dim3(np, 1), dim3(NTHREADS), 0, p->stream, g, p->rowsum_g, n, np, p->lna, p->flag);
  hipLaunchKernelGGL(k_rowsumsq, dim3(n, B), dim3(NTHREADS), 0, p->stream, G, n, p->rowsum_G, p->flag);
  hipLaunchKernelGGL(k_logmarg, dim3(np, B), dim3(NTHREADS), 0, p->stream, G, p->rowsum_G, n, np, p->lnb, p->flag);
  LAUNCH_CHECK();
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (hflag & 2) return fail(FOT_E_INVALID, "fot_solve: amplitudes must be finite and >= 0");
  if (hflag & 4) return fail(FOT_E_INVALID, "fot_solve: an image has zero (or non-finite) total intensity");

  if (!warm_start) {
    const double v0 = e[0] * std::log(1.0 / ((double)n * (double)n));  // u = V = 1/n^2
    const size_t total = (size_t)B * p->plane;
    const int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_fill_pot, dim3(blocks), dim3(256), 0, p->stream, p->f, n, np, B, v0);
    hipLaunchKernelGGL(k_fill_pot, dim3(blocks), dim3(256), 0, p->stream, p->psi, n, np, B, v0);
    LAUNCH_CHECK();
  }

  fot_status st = p->tail_iters > 0 ? dispatch(p->prec, [&](auto h) -> fot_status {
    return dispatch(p->tail_prec, [&](auto l) -> fot_status {
      return solve_body<decltype(h), decltype(l)>(p, e, iters, phase_out);
    });
  })
                                     : dispatch(p->prec, [&](auto tag) -> fot_status {
                                         return solve_body<decltype(tag), decltype(tag)>(p, e, iters, phase_out);
                                       });
  if (st != FOT_OK) return st;

  std::vector<double> ha((size_t)iters * B), hb((size_t)iters * B), rs((size_t)READOUT_SLOTS * B);
  std::vector<int> riter((size_t)B, 0x7f7f7f7f), rmin((size_t)2 * B, 0x7f7f7f7f);
  std::vector<int> slots((size_t)2 * B * p->range_spt * 2);
  int pflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(&pflag, p->probe_flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(slots.data(), p->range_slots, sizeof(int) * slots.size(), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(ha.data(), p->hist_a, ha.size() * 8, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(hb.data(), p->hist_b, hb.size() * 8, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(rs.data(), p->rsums, rs.size() * 8, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->has_state = true;
  p->last_iters = iters;
  p->last_eps = e;
  p->tape_valid = (p->tape != nullptr);
  p->seg_last_valid = p->tape_valid;
  for (int seg = 0; seg < 2; ++seg)
    for (int b = 0; b < B; ++b)
      for (int w = 0; w < p->range_spt; ++w) {
        const int* sl = &slots[2 * (((size_t)seg * B + b) * p->range_spt + w)];
        rmin[(size_t)seg * B + b] = std::min(rmin[(size_t)seg * B + b], sl[0]);
        riter[b] = std::min(riter[b], sl[1]);
      }
  for (int& r : riter)
    if (r == 0x7f7f7f7f) r = -1;

  if (rep) {
    const double epT = e[iters - 1];
    for (int b = 0; b < B; ++b) {
      const double err_a = rs[0 * B + b], mass = rs[1 * B + b], cost = rs[2 * B + b] + rs[6 * B + b], dots = rs[3 * B + b],
                   err_b = rs[4 * B + b];
      if (rep->err_a) rep->err_a[b] = err_a;
      if (rep->err_b) rep->err_b[b] = err_b;
      if (rep->err_products) rep->err_products[b] = (rs[5 * B + b] != rs[5 * B + b]) ? rs[5 * B + b] : std::max(err_b, rs[5 * B + b]);
      if (rep->dual) rep->dual[b] = dots - epT * mass;
      if (rep->transport_cost) rep->transport_cost[b] = cost;
      if (rep->range_iter) rep->range_iter[b] = riter[b];
      if (rep->range_loss && !p->cfot) {
        auto bound = [&](auto tag, int m) { return Ops<decltype(tag)>::loss_bound(p->n, m); };
        double lb = 0.0;
        (void)dispatch(p->prec, [&](auto tag) -> fot_status {
          lb = std::max(lb, bound(tag, rmin[b]));
          return FOT_OK;
        });
        if (p->tail_iters > 0)
          (void)dispatch(p->tail_prec, [&](auto tag) -> fot_status {
            lb = std::max(lb, bound(tag, rmin[B + b]));
            return FOT_OK;
          });
        rep->range_loss[b] = lb;
      } else if (rep->range_loss) {
        rep->range_loss[b] = 0.0;
      }
    }
    if (p->d.flags & FOT_FLAG_NO_HISTORY) {
      std::fill(ha.begin(), ha.end(), std::numeric_limits<double>::quiet_NaN());
      std::fill(hb.begin(), hb.end(), std::numeric_limits<double>::quiet_NaN());
    }
    if (rep->err_a_history) std::memcpy(rep->err_a_history, ha.data(), ha.size() * 8);
    if (rep->err_b_history) std::memcpy(rep->err_b_history, hb.data(), hb.size() * 8);
    rep->iters_done = iters;
    rep->nonfinite = (hflag & 1) ? 1 : 0;
    float ms = 0.f;
    rep->ms_total = rep->ms_iterations = 0.0;   // (no events in a plan on the static scratch array)
    if (p->ev[0]) {
      HIP_TRY(hipEventElapsedTime(&ms, p->ev[0], p->ev[3]));
      rep->ms_total = ms;
      HIP_TRY(hipEventElapsedTime(&ms, p->ev[1], p->ev[2]));
      rep->ms_iterations = ms;
    }
    double tot = 0.0;
    int cnt = 0;
    for (int i = 0; i + 1 < p->prof_used; i += 2) {
      HIP_TRY(hipEventElapsedTime(&ms, p->prof[i], p->prof[i + 1]));
      tot += ms;
      if (rep->ms_launches && cnt < 4 * iters) rep->ms_launches[cnt] = ms;
      ++cnt;
    }
    rep->ms_contract = tot;
    rep->n_contract = cnt;
    rep->graph = p->used_graph ? 1 : 0;
  }
  if (hflag & 1) return fail(FOT_E_NONFINITE, "fot_solve: a potential became non-finite");
  for (int b = 0; b < B; ++b)
    if (riter[b] >= 0) {
      char msg[512];
      std::snprintf(msg, sizeof msg,
                    "fot_solve: target %d: at iteration %d%s a product of the Gibbs factor fell below what "
                    "the operand type holds at eps %.3g (terms lost to underflow could matter; use FOT_F64, "
                    "FOT_FLAG_SMALL_TILES or a larger eps)",
                    b, riter[b], riter[b] == iters ? " (the check after the last one)" : "", e[riter[b] < iters ? riter[b] : iters - 1]);
      return fail(FOT_E_RANGE, msg);
    }
  if (pflag & 1)
    return fail(FOT_E_RANGE, "fot_solve: one more u-update in the operand type at the final potentials gave a "
                             "non-finite potential: the products lost range at this eps");
  {
    // the final products (column marginal, and the probe's row discrepancy) are exact up to the
    // operand type's rounding.  Bounds from sweeps against the oracle over n and eps: above each
    // type's largest value in accurate solves (FP16 3.1e-4, BF16 7.8e-4) and below the values of
    // solves whose potentials had drifted (FP16 from 7.5e-4, BF16 1.3e-2).  FP16's range loss is
    // systematic (a biased error), so its bound is the tightest of the 16-bit types.
    const int fprec = p->tail_iters > 0 ? p->tail_prec : p->prec;   // the final iterations' type
    const double bound = p->cfot                 ? 1e-6
                         : fprec == FOT_F64    ? 1e-8
                         : fprec == FOT_F32    ? 1e-5
                         : fprec == FOT_BF16X3 ? 1e-4
                         : fprec == FOT_F16    ? 5e-4
                                               : 5e-3;
    for (int b = 0; b < B; ++b) {
      // the larger of the final column-marginal L1 (the last V-half's products) and the probe's
      // row-marginal discrepancy (the u-direction products at the final potentials)
      const double err_b = std::max(rs[4 * B + b], rs[5 * B + b]);
      if (!(err_b <= bound) || rs[5 * B + b] != rs[5 * B + b]) {
        char msg[512];
        std::snprintf(msg, sizeof msg,
                      p->cfot ? "fot_solve: target %d: final column-marginal L1 %.3g exceeds %.0e: the FFT "
                                "convolutions lost the small values at eps %.3g (use the matrix-product "
                                "contraction or a larger eps)"
                              : "fot_solve: target %d: marginal L1 of the operand type's products %.3g (final "
                                "column marginal, or the row marginal of one more u-update) exceeds %.0e: the "
                                "Gibbs products underflowed in the operand type at eps %.3g (FOT_FLAG_SMALL_TILES "
                                "reaches about half the eps; otherwise use FOT_F64 or a larger eps)",
                      b, err_b, bound, e[iters - 1]);
        return fail(FOT_E_RANGE, msg);
      }
    }
  }
  return FOT_OK;
}

fot_status fot_solve_noalloc(const fot_plan_desc* desc, void* stream, const double* g, const double* G,
                             const double* eps, int n_eps, int iters, double* f_out, double* psi_out,
                             double* phase_out, fot_report* rep) {
  g_err.clear();
  if (!desc) return fail(FOT_E_INVALID, "fot_solve_noalloc: null descriptor");
  fot_plan_desc d = *desc;
  if (d.checkpoint_every != 0)
    return fail(FOT_E_INVALID, "fot_solve_noalloc: no reverse mode (checkpoint_every must be 0)");
  if (d.flags & FOT_FLAG_PROFILE) return fail(FOT_E_INVALID, "fot_solve_noalloc: FOT_FLAG_PROFILE needs events");
  d.flags |= FOT_FLAG_NO_GRAPH;   // (a graph's instantiation would allocate)
  int cN = 0;
  fot_status s = validate_desc(d, &cN);
  if (s != FOT_OK) return s;
  unsigned char* base = nullptr;
  if ((s = scratch_of_current_device(&base)) != FOT_OK) return s;
  fot_plan_s plan;
  s = plan_init(&plan, d, cN, (hipStream_t)stream, base, NOALLOC_SCRATCH_BYTES);
  if (s == FOT_OK) s = fot_solve(&plan, g, G, eps, n_eps, iters, 0, phase_out, rep);
  // the potentials are written also when the solve reports FOT_E_RANGE or FOT_E_NONFINITE
  if (s == FOT_OK || s == FOT_E_RANGE || s == FOT_E_NONFINITE) {
    const std::string msg = g_err;
    const fot_status sp = fot_potentials(&plan, f_out, psi_out, nullptr, nullptr);
    if (sp != FOT_OK) s = sp;
    else g_err = msg;
    if (hipStreamSynchronize(plan.stream) != hipSuccess && s == FOT_OK)
      s = fail(FOT_E_HIP, "fot_solve_noalloc: stream synchronisation failed");
  }
  const std::string msg = g_err;
  release(&plan);   // (frees nothing: no device buffer of this plan came from hipMalloc)
  g_err = msg;
  return s;
}

fot_status fot_backward(fot_plan_t p, const double* dL_dDual, const double* dL_dphase, double* dL_dG) {
  g_err.clear();
  if (!p) return fail(FOT_E_INVALID, "fot_backward: null plan");
  if (!dL_dG) return fail(FOT_E_INVALID, "fot_backward: null output");
  if (!p->tape) return fail(FOT_E_STATE, "fot_backward: the plan has no tape (checkpoint_every = 0)");
  if (!p->tape_valid) return fail(FOT_E_STATE, "fot_backward: no taped solve to differentiate");
  std::vector<double> dd((size_t)p->B, 0.0);
  if (dL_dDual)
    for (int b = 0; b < p->B; ++b) {
      if (!std::isfinite(dL_dDual[b])) return fail(FOT_E_INVALID, "fot_backward: dL/dD must be finite");
      dd[b] = dL_dDual[b];
    }
  HIP_TRY(hipMemcpyAsync(p->dd_dev, dd.data(), sizeof(double) * p->B, hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemsetAsync(p->flag, 0, sizeof(int), p->stream));
  fot_status st = dispatch(p->prec, [&](auto tag) -> fot_status {
    typedef decltype(tag) T;
    return Ops<T>::backward(p, dL_dphase, dL_dG);
  });
  if (st != FOT_OK) return st;
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (hflag & 1) return fail(FOT_E_NONFINITE, "fot_backward: a replayed potential became non-finite");
  return FOT_OK;
}

fot_status fot_output_beam(fot_plan_t p, const double* g, const double* phase, const double* G, double* intensity,
                           double* l1) {
  g_err.clear();
  if (!p || !g || !phase) return fail(FOT_E_INVALID, "fot_output_beam: null argument");
  if (l1 && !G) return fail(FOT_E_INVALID, "fot_output_beam: the L1 loss needs the target G");
  const int n = p->n, np = p->np, B = p->B;
  fot_status s;
  if ((s = beam_ready(p)) != FOT_OK) return s;
  if ((s = beam_inputs(p, g, G)) != FOT_OK) return s;
  hipLaunchKernelGGL(k_beam_field, dim3(n, B), dim3(NTHREADS), 0, p->stream, g, phase, n, np, p->bfc);
  LAUNCH_CHECK();
  if ((s = beam_dft(p, p->bfc, p->bF, false)) != FOT_OK) return s;
  hipLaunchKernelGGL(k_beam_intensity, dim3(n, B), dim3(NTHREADS), 0, p->stream, p->bF, n, np, p->bpow, G,
                     p->bsumG, intensity, p->brow);
  if (G) hipLaunchKernelGGL(k_sum_rows, dim3(B), dim3(NTHREADS), 0, p->stream, p->brow, n, p->bl1);
  LAUNCH_CHECK();
  if ((s = beam_flag(p, "fot_output_beam")) != FOT_OK) return s;
  if (l1) {
    HIP_TRY(hipMemcpyAsync(l1, p->bl1, sizeof(double) * B, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  return FOT_OK;
}

fot_status fot_polish_gs(fot_plan_t p, const double* g, const double* G, double* phase, int iters) {
  g_err.clear();
  if (!p || !g || !G || !phase) return fail(FOT_E_INVALID, "fot_polish_gs: null argument");
  if (iters < 0) return fail(FOT_E_INVALID, "fot_polish_gs: iters must be >= 0");
  const int n = p->n, np = p->np, B = p->B;
  fot_status s;
  if ((s = beam_ready(p)) != FOT_OK) return s;
  if ((s = beam_inputs(p, g, G)) != FOT_OK) return s;
  if ((s = beam_flag(p, "fot_polish_gs")) != FOT_OK) return s;
  hipLaunchKernelGGL(k_beam_field, dim3(n, B), dim3(NTHREADS), 0, p->stream, g, phase, n, np, p->bfc);
  LAUNCH_CHECK();
  for (int it = 0; it < iters; ++it) {
    if ((s = beam_dft(p, p->bfc, p->bF, false)) != FOT_OK) return s;
    hipLaunchKernelGGL(k_gs_project, dim3(n, B), dim3(NTHREADS), 0, p->stream, p->bF, G, n, np, p->bfc);
    LAUNCH_CHECK();
    if ((s = beam_dft(p, p->bfc, p->bF, true)) != FOT_OK) return s;
    hipLaunchKernelGGL(k_gs_phase, dim3(n, B), dim3(NTHREADS), 0, p->stream, p->bF, g, n, np, phase, p->bfc);
    LAUNCH_CHECK();
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  return FOT_OK;
}

}  // extern "C"
