/*
 * fot.h -- C ABI of the MI355X (gfx950) Fast Optimal Transport library (libfot.so).
 *
 * The library solves the entropic optimal-transport problem of holographic beam shaping
 * of arXiv 2512.19072: given an input-beam amplitude g_jk and target amplitudes G_LM on
 * n x n grids (Sec. 2), it runs the Sinkhorn-Knopp dual iteration of Algorithm 1 with the
 * separable Gibbs kernel exp(-c/eps) = Lambda_jL Lambda_kM (Sec. 3, Eq. 6-8), returns the
 * dual potentials, the marginal errors, the dual value and transport cost, and the phase
 * obtained from the first moments of the plan (Sec. 3, Eq. 9-10) by trapezoid integration.
 * fot_backward differentiates the dual value and the phase with respect to G through the
 * unrolled iterations (reverse mode with checkpoints).
 *
 * Conventions shared by every entry point
 *   - Arrays are row-major [n][n] per image, j (row) = x axis, k (column) = y axis;
 *     batches are [batch][n][n].  X_L = (L - floor(n/2)) / sqrt(n) (Sec. 2).
 *   - Every array argument except the fot_report fields is a DEVICE pointer owned by the
 *     caller (for example a torch tensor's data pointer); the library never frees it.
 *     The plan owns all its workspace, allocated once in fot_plan (the output-beam
 *     workspace of fot_output_beam / fot_polish_gs at the first such call).
 *   - Potentials are FP64: f = eps ln u and psi = eps ln V (Eq. 6), -inf at zero-mass pixels.
 *   - Work is issued on the plan's stream in stream order.  fot_solve synchronises once at
 *     its end to fill the report; fot_backward synchronises once at its end to report errors.
 *   - Every call returns a status; nothing aborts or throws across the ABI.  On failure,
 *     fot_last_error() gives a message (thread-local, valid until the next call on the
 *     same thread).
 *   - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef FOT_H
#define FOT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fot_plan_s* fot_plan_t;

typedef enum {
  FOT_OK = 0,
  FOT_E_INVALID = 1,     /* bad argument: size, eps <= 0, negative/non-finite amplitude, zero mass */
  FOT_E_NOMEM = 2,       /* device allocation failed in fot_plan */
  FOT_E_HIP = 3,         /* a HIP runtime call failed */
  FOT_E_NONFINITE = 4,   /* a potential of a positive-mass pixel became non-finite */
  FOT_E_STATE = 5,       /* call order violated (e.g. backward without a taped solve) */
  FOT_E_UNSUPPORTED = 6, /* option not available in this library (or, from fot_solve, an eps that
                            needs the block-normalised Gibbs factor at an n whose exponent
                            table does not fit in LDS: n > 4096 with 32- and 16-bit types) */
  FOT_E_RANGE = 7        /* fot_solve finished and filled its outputs, but the Gibbs products
                            may have lost values below the operand type's range at this eps.
                            Two checks: (1) in every iteration each output of the per-axis
                            products is compared with the largest block scale it was formed
                            from, which bounds what terms dropped below the type's range could
                            have cost it (fot_report.range_loss, a worst case); the check fails
                            when the bound exceeds 2^-7 (FP32, BF16x3), 2^13 (BF16) or 2^20
                            (FP64), levels calibrated against the oracle between accurate and
                            inaccurate solves (fot_report.range_iter gives the first such
                            iteration; FP16 has no such check); (2) after the
                            solve, fot_report.err_products (the larger of the final column-
                            marginal L1, evaluated in FP64, and the discrepancy of one more
                            u-direction product at the final potentials against FP64) must stay
                            within the type's bound (FP64 1e-8, FP32 1e-5, BF16x3 1e-4, BF16
                            5e-3, FP16 5e-4).  Use FOT_F64, FOT_FLAG_SMALL_TILES or a larger eps */
} fot_status;

/* Element type of the contraction operands (the Gibbs factor and the shifted exponentials
 * that the per-axis matrix products consume).  Accumulation is FP32 (FP64 for FOT_F64);
 * potentials, logarithms of the marginals, and all reductions are FP64 in every mode.
 * Every operand is stored in blocks normalised by an integer power of two that the products
 * rescale exactly in FP64; the Gibbs factor too once eps is small enough that it has entries
 * below the type's range.  The 32-bit and 16-bit types then reach down to eps = 2e-4 on
 * 1024 x 1024 grids (the paper's regime; 1e-4 with FOT_FLAG_SMALL_TILES; FP16 to about 1e-3);
 * below that FOT_E_RANGE reports the loss and FOT_F64 applies.
 * FOT_BF16X3 splits each operand value v into hi = bf16(v) and lo = bf16(v - hi) and forms
 * every product as hi.hi + hi.lo + lo.hi with three BF16 matrix-core operations: about 16
 * significant bits per operand (between BF16's 8 and FP32's 24) at BF16 matrix-core rates,
 * with FP32's exponent range and FP32's memory footprint (4 bytes per operand value). */
typedef enum { FOT_F64 = 0, FOT_F32 = 1, FOT_BF16 = 2, FOT_F16 = 3, FOT_BF16X3 = 4 } fot_precision;

enum {
  FOT_FLAG_PROFILE = 1,  /* time every launch of the iteration kernels (the fused per-axis
                            contractions of Eq. 7-8) with HIP events (fot_report.ms_contract);
                            the iteration loop is then launched kernel by kernel (events
                            recorded inside a graph cannot be timed) */
  FOT_FLAG_NO_GRAPH = 2, /* launch the iteration loop kernel by kernel instead of replaying a
                            HIP graph of it (the results are bit-identical either way) */
  FOT_FLAG_NO_HISTORY = 4, /* do not evaluate the per-iteration marginal errors (the paper's
                            practice of running a fixed number of iterations without a loss,
                            Sec. 3 after Algorithm 1): err_*_history is filled with NaN; the
                            potentials, phase and final report values are bit-identical */
  FOT_FLAG_CFOT = 8,     /* cFOT (Sec. 3, convolutional speedup, Eq. 11): apply Lambda . X .
                            Lambda in the iterations as two 1-D linear convolutions with
                            lambda_j = exp(-j^2 / (2 n^2 eps)) by FP64 FFTs of length N =
                            2^ceil(log2(2n - 1)), O(n^2 log n) per half-step instead of the
                            O(n^3) matrix products.  Requires FOT_F64, n <= 2048 and
                            checkpoint_every = 0 (no reverse mode); otherwise fot_plan returns
                            FOT_E_UNSUPPORTED.  The read-out (Eq. 9-10, the report) is the same
                            FP64 computation as without the flag.  An FFT's rounding is relative
                            to each whole row, so convolution values far below their row's
                            largest lose accuracy: at small eps fot_solve may return
                            FOT_E_NONFINITE, or FOT_E_RANGE when the final column-marginal L1
                            exceeds 1e-6 */
  FOT_FLAG_SMALL_TILES = 16, /* normalise the iteration kernels' operands in 32-wide instead of
                            64-wide blocks.  fot_plan runs the kernels on 32 x 32 output tiles,
                            whose blocks are 32 wide anyway, when 64 x 64 tiles would occupy at
                            most half of the GPU's compute units (small grids); on larger grids
                            the flag keeps the 64 x 64 tiles with two blocks each (up to
                            n_p = 3584, beyond which the block-normalised Lambda's exponent table
                            needs the 32 x 32 tiles) and trades speed (about 1.12x the time per
                            iteration at 1024 x 1024 and eps 2e-4) for range: the 32- and 16-bit operand types then reach
                            about half the eps (FP32: 1e-4 instead of 2e-4 on the two-Gaussian
                            1024 x 1024 workload).  The two tilings give bit-identical
                            potentials.  No effect with FOT_FLAG_CFOT */
  FOT_FLAG_F64_REVERSE = 32, /* fot_backward after an FP32 solve: run the reverse half-steps with FP64
                            operands, as for the other precisions.  Without the flag they use FP32
                            operands wherever the solve held the Gibbs factor raw in FP32: on 8
                            targets of 512 x 512 with 100 iterations (checkpoints every 10) the
                            backward pass takes 28 ms instead of 37 ms, and the gradient's error
                            grows from 1.6e-5 to 5.7e-5 relative to the FP64 oracle's gradient and
                            from 3e-6 to 1.6e-5 relative to central differences of FP64 solves */
  FOT_FLAG_STAGED_LAMBDA = 64 /* stage the Gibbs factor's tiles through LDS with every K stage of the
                            per-axis contractions, as the other operand is, instead of reading
                            them from one Toeplitz table per workgroup (Lambda[i][k] depends on
                            i - k only).  The results are bit-identical; the table halves the
                            bytes each workgroup fetches per stage.  The table is used wherever
                            Lambda is held raw (not block-normalised for small eps) with FP64,
                            FP32, BF16 or FP16 operands and its first row fits in a stage
                            buffer (n_p * element size <= 32 KiB on 64 x 64 tiles, 16 KiB on
                            32 x 32 tiles) */
};

typedef struct {
  int n;                 /* grid side, 1 <= n <= 8192 */
  int batch;             /* number of targets sharing one input amplitude, >= 1 */
  int precision;         /* fot_precision */
  int max_iters;         /* largest iteration count fot_solve will be given, >= 1 */
  int checkpoint_every;  /* > 0: keep psi every k iterations so fot_backward can replay;
                            0: no tape (fot_backward then returns FOT_E_STATE) */
  int flags;             /* FOT_FLAG_* */
  int tail_precision;    /* precision schedule (with tail_iters > 0): the operand type of the last
                            tail_iters iterations of every fot_solve; the first iters - tail_iters
                            use `precision` (Algorithm 1 is unchanged; only the type of the
                            contraction operands changes between the two segments, and each
                            segment builds its operands from the potentials it starts from).
                            Must differ from `precision`; `precision` must not be FOT_F64; no
                            FOT_FLAG_CFOT and no reverse mode (checkpoint_every = 0), else
                            FOT_E_UNSUPPORTED.  The end-of-solve range check uses the tail type.
                            Example: BF16 iterations then one or two FP32 ones reach FP32's
                            marginal error at BF16's iteration cost */
  int tail_iters;        /* >= 0; 0 = no schedule (zero-initialised descriptors keep one type) */
} fot_plan_desc;

/* Results of fot_solve.  All pointers are HOST arrays owned by the caller; any may be NULL. */
typedef struct {
  double* err_a;          /* [batch] sum_p |sum_q Gamma_pq - a_p| of the final plan (Sec. 3, conv. criterion) */
  double* err_b;          /* [batch] sum_q |sum_p Gamma_pq - b_q| of the final plan, in FP64: after
                             the final V-update it measures the operand type's error in that
                             update's products (FP32 ~1e-7, BF16 ~5e-4 on well-posed inputs) */
  double* dual;           /* [batch] <f,a> + <psi,b> - eps sum Gamma, a = g^2/sum g^2, b = G^2/sum G^2 */
  double* transport_cost; /* [batch] sum Gamma_pq c_pq (Sec. 2, Eq. 2-3) */
  double* err_a_history;  /* [iters][batch] row-marginal L1 of the plan entering each u-update
                             (NaN with FOT_FLAG_NO_HISTORY) */
  double* err_b_history;  /* [iters][batch] column-marginal L1 of the plan entering each V-update */
  int iters_done;         /* iterations run */
  int nonfinite;          /* 1 if a non-finite potential appeared (status FOT_E_NONFINITE) */
  double ms_total;        /* HIP-event time of the whole solve on the plan's stream */
  double ms_iterations;   /* HIP-event time of the iteration loop only */
  double ms_contract;     /* FOT_FLAG_PROFILE: summed HIP-event time of the iteration kernels */
  int n_contract;         /* FOT_FLAG_PROFILE: number of iteration-kernel launches timed */
  int graph;              /* 1 if the iteration loop was replayed as a HIP graph */
  double* err_products;   /* [batch] or NULL: the check of the operand type's products at the
                             final potentials against FP64, the larger of err_b and the row-
                             marginal L1 that one more u-update would make through its products
                             alone; FOT_E_RANGE when it exceeds the type's bound (0 beyond err_b
                             for FOT_F64 and cFOT, whose products need no probe) */
  int* range_iter;        /* [batch] or NULL: the first iteration (0-based; iters = the check
                             after the last one) in which an output of the operand type's
                             products fell below its range floor (see FOT_E_RANGE), or -1 */
  double* range_loss;     /* [batch] or NULL: the largest relative loss that terms dropped below
                             the operand type's range could have caused in any output of the
                             per-axis products during the solve (a bound: n 2^-125 times 2 to the
                             output's distance below the largest block scale it was formed from;
                             2^-1021 for FP64, 2^-23 for FP16); see FOT_E_RANGE */
  double* ms_launches;    /* [4 * iters] or NULL: FOT_FLAG_PROFILE: the HIP-event time of each
                             timed iteration-kernel launch in issue order (pass 1 and pass 2 of
                             the u-half, then of the V-half, per iteration); n_contract entries */
} fot_report;

/* Create a plan: validates desc, allocates O(n^2 * batch) device workspace once, as one device
 * allocation (no later allocation in fot_solve or fot_backward; without a tape at most
 * (68 batch + 12) bytes per padded pixel for 32- and 16-bit operands, (64 batch + 16) for FP64,
 * plus a few MB), and binds it to `stream` (a hipStream_t; NULL = the null stream) on the current
 * device.  *out is set only on FOT_OK (FOT_E_NOMEM when the allocation fails). */
fot_status fot_plan(const fot_plan_desc* desc, void* stream, fot_plan_t* out);

/* Run Algorithm 1 (Sec. 3): normalise a = g^2/sum g^2 and b = G^2/sum G^2 (Eq. 2 marginals,
 * unit mass), start from u = V = 1/n^2 (or, with warm_start != 0, from the potentials the
 * plan holds), do `iters` iterations of the u-update (Eq. 7) then the V-update (Eq. 8), then
 * compute Eq. 9-10 with the final u and V, integrate by the trapezoid rule from phi_00 = 0
 * (along j at k = 0, then along k), remove the a-weighted mean, and fill `rep`.
 *   g         device [n][n] FP64 input amplitude, finite, >= 0, positive total
 *   G         device [batch][n][n] FP64 target amplitudes, same requirements per target
 *   eps       HOST array of n_eps values: n_eps == 1 (constant) or n_eps == iters (eps_t of
 *             iteration t; the potentials are carried across changes), each finite and > 0
 *   iters     1 <= iters <= max_iters
 *   phase_out device [batch][n][n] FP64 phase in cycles, or NULL to skip writing it
 *   rep       host report, or NULL
 * Returns FOT_E_INVALID for bad arguments or amplitudes (nothing is run), FOT_E_UNSUPPORTED
 * (nothing is run) if an eps of the schedule needs the block-normalised Gibbs factor at an n whose
 * exponent table does not fit in LDS (32- and 16-bit types with n > 4096),
 * FOT_E_NONFINITE if a positive-mass potential overflowed (outputs undefined, the plan
 * stays usable), FOT_E_RANGE if the operand type could not represent the products at this
 * eps (outputs written but inaccurate; see FOT_E_RANGE), FOT_E_HIP on a runtime error. */
fot_status fot_solve(fot_plan_t plan, const double* g, const double* G,
                     const double* eps, int n_eps, int iters, int warm_start,
                     double* phase_out, fot_report* rep);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): one solve as fot_plan + fot_solve + fot_potentials + fot_destroy would do it, with
 * the same kernels and bit-identical results, but with every device buffer carved from a static
 * array of 32 MiB per GPU that the library holds until the process ends.  Nothing is allocated
 * (no hipMalloc, no graph, no events); the iteration loop is launched kernel by kernel and the
 * report's timing fields are 0.
 *   desc      as for fot_plan; checkpoint_every must be 0 and FOT_FLAG_PROFILE unset
 *             (FOT_E_INVALID otherwise); a plan whose workspace exceeds 32 MiB (n_p <= 640 for one
 *             target with FP64, FP32 or BF16x3 operands, n_p <= 512 with 16-bit ones) is rejected
 *             with FOT_E_INVALID before anything runs
 *   stream..rep as for fot_plan / fot_solve (a cold start: u = V = 1/n^2)
 *   f_out, psi_out  device [batch][n][n] FP64 final potentials, or NULL; written also when the
 *             status is FOT_E_RANGE or FOT_E_NONFINITE
 * Every call on a GPU uses that GPU's one array and leaves its contents behind (each call clears
 * what must start at zero): calls that overlap on one GPU (other streams or threads) race and
 * must be serialised by the caller.  Synchronises the stream before returning. */
fot_status fot_solve_noalloc(const fot_plan_desc* desc, void* stream, const double* g, const double* G,
                             const double* eps, int n_eps, int iters, double* f_out, double* psi_out,
                             double* phase_out, fot_report* rep);

/* Read and/or write the potentials held by the plan (device [batch][n][n] FP64 each).
 * Outputs are written before inputs are read, so the same call can swap states.
 * Any pointer may be NULL to skip it.  Writing potentials invalidates the backward tape. */
fot_status fot_potentials(fot_plan_t plan, double* f_out, double* psi_out,
                          const double* f_in, const double* psi_in);

/* Reverse mode of the last fot_solve (which must have run with checkpoint_every > 0 and
 * without warm_start changes since): given dL/dD per target (HOST [batch], NULL = 0) and
 * dL/dphase (device [batch][n][n] FP64, NULL = 0), write dL/dG (device [batch][n][n] FP64).
 * The iterations are replayed from the stored checkpoints segment by segment; the replay is
 * bit-identical to the forward solve.  Each reverse half-step is one signed contraction
 * Lambda (v e^{-ln S}) Lambda run on the fused iteration kernels (signed block-normalised operands,
 * FP64 block sums), with FP32 operands after an FP32 solve unless FOT_FLAG_F64_REVERSE is set
 * (FP64 operands otherwise).  Zero-amplitude target pixels get gradient 0. */
fot_status fot_backward(fot_plan_t plan, const double* dL_dDual, const double* dL_dphase,
                        double* dL_dG);

/* Output beam of a phase and its L1 intensity loss (Sec. 4; Eq. 1 for the beam).
 *   g          [n][n]        input amplitude (>= 0, not all zero), shared by the batch
 *   phase      [batch][n][n] phase in cycles (for example fot_solve's phase_out)
 *   G          [batch][n][n] target amplitude, or NULL when no loss is wanted
 *   intensity  [batch][n][n] output, or NULL: the unit-power far-field intensity
 *              I_LM = |F[g e^{2 pi i phase}]_LM|^2 / (n^2 sum g^2), with the centred transform
 *              F[f]_LM = sum_jk f_jk exp(-2 pi i ((j-c)(L-c) + (k-c)(M-c)) / n), c = floor(n/2)
 *              (x_j X_L of Sec. 2; this sign sends light to where the phase gradient points)
 *   l1         HOST double[batch], or NULL: sum_LM |I_LM - G_LM^2 / sum G^2| (needs G)
 * The transform runs as FP64 matrix-core products (about 16 n^3 flop per target).  Returns
 * FOT_E_INVALID for null g or phase, l1 without G, or amplitudes that are negative,
 * non-finite or all zero.  Synchronises the plan's stream before returning. */
fot_status fot_output_beam(fot_plan_t plan, const double* g, const double* phase, const double* G,
                           double* intensity, double* l1);

/* Gerchberg-Saxton polishing of a phase (the textbook step that Sec. 4 names as the usual
 * follow-up to an OT phase), in place: iters rounds of
 *   F = F[g e^{2 pi i phase}];  F <- G F / |F|  (G where F = 0);
 *   f = conj-transform of F;    phase <- arg(f) / (2 pi) in (-1/2, 1/2]  (0 where f = 0)
 * with the transform of fot_output_beam.  g [n][n], G and phase [batch][n][n] as there.
 * iters = 0 leaves the phase unchanged.  Returns FOT_E_INVALID for null arguments, iters < 0
 * or invalid amplitudes (the phase is then unchanged).  Synchronises before returning. */
fot_status fot_polish_gs(fot_plan_t plan, const double* g, const double* G, double* phase, int iters);

/* Release the plan and all its device memory (after finishing its stream's work). */
fot_status fot_destroy(fot_plan_t plan);

/* Message for the last failed call on this thread ("" if none). */
const char* fot_last_error(void);

/* Library version string, e.g. "fot 0.1 gfx950". */
const char* fot_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FOT_H */
