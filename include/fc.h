/*
 * fc.h - C ABI of the MI355X (gfx950) fast-convolution filtered CP-OFDM library.
 *
 * Implements the fast-convolution (FC) synthesis and analysis filter banks of
 * Yli-Kaakinen et al., "Frequency-Domain Signal Processing for Spectrally-
 * Enhanced CP-OFDM Waveforms in 5G New Radio" (arXiv 2008.00672):
 *   - continuous FC with overlap-add (OLA) or overlap-save (OLS) blocks
 *     (Sec. III-B, block operators F^(OLA), F^(OLS); Sec. IV, G^(OLA), G^(OLS));
 *   - symbol-synchronised FC whose blocks align with every OFDM symbol and its
 *     NR cyclic prefix, with CP truncation/extrapolation (Sec. III-C..III-E)
 *     and the synchronised receiver with CP removal (Sec. IV); the
 *     synchronised transmitter as OLA or as OLS with hard or smoothed output
 *     window edges (Sec. III-D);
 *   - the synchronised receiver with OFDM demodulation in the simplified
 *     joint form (Sec. V-A), the transmitter from QAM grids with the OFDM
 *     modulation in the kernels, the adjoint and the weight gradient, HIP
 *     graph capture and an autotuner for the work split.
 *
 * Conventions (all arguments are plain C types; no framework types cross this
 * boundary):
 *   - Samples are complex, stored interleaved (I, Q) in one of the I/O types
 *     below. Arithmetic is always FP32 on the device; twiddles and block phases
 *     are computed in FP64 on the host and rounded once to FP32.
 *   - Naming: n_short is the paper's L_m (short transform, equal to the OFDM
 *     IFFT length L_OFDM,m), n_long is the paper's N (long transform);
 *     I = n_long / n_short is the interpolation factor.
 *   - Every device pointer is owned by the caller and must stay valid until the
 *     work queued on the given stream has completed. The plan owns its own
 *     device tables (descriptors, twiddles, weights) and scratch (the
 *     demodulating receiver's and the weight gradient's per-task slots).
 *   - Calls that take a stream are asynchronous on that stream (a hipStream_t
 *     passed as void*; NULL means the default stream) and never synchronise the
 *     host, except where a function says so (weights from host memory,
 *     tuning, autotuning). A plan must not be used on two streams
 *     concurrently or from two host threads at once; different plans are
 *     independent.
 *   - Every function returns an fc_status and never aborts or throws across
 *     the ABI. Argument and shape errors are detected on the host before any
 *     device work is queued. HIP runtime failures surface as FC_E_DEVICE.
 */
#ifndef FC_H_
#define FC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fc_status;
enum {
  FC_OK = 0,
  FC_E_ARG = -1,          /* invalid argument value or NULL pointer          */
  FC_E_SHAPE = -2,        /* inconsistent sizes (e.g. n_short does not divide n_long) */
  FC_E_UNSUPPORTED = -3,  /* valid per the paper but not implemented here    */
  FC_E_NOMEM = -4,        /* host or device allocation failed                */
  FC_E_DEVICE = -5,       /* a HIP runtime call failed                       */
  FC_E_STATE = -6,        /* operation not valid for this plan               */
  FC_E_LIMIT = -7         /* needs more than the fixed no-allocation scratch */
};

/* Size of the fixed device scratch of fc_tx_weight_grad_noalloc (per GPU). */
#define FC_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* Processing model of a subband (Sec. III-B, III-C, IV). */
enum {
  FC_CONT_OLA = 0,   /* continuous, fixed overlap, overlap-add                 */
  FC_CONT_OLS = 1,   /* continuous, fixed overlap, overlap-save                */
  FC_SYNC_OLA = 2,   /* symbol-synchronised: OLA transmitter, CP-removing receiver */
  FC_SYNC_OLS = 3    /* symbol-synchronised: OLS transmitter (output windows), same receiver */
};

/* Storage type of the interleaved I/Q samples in device memory. */
enum {
  FC_IO_C64 = 0,     /* 2 x float32                                    */
  FC_IO_F16 = 1,     /* 2 x IEEE binary16, round-to-nearest-even       */
  FC_IO_BF16 = 2     /* 2 x bfloat16, round-to-nearest-even            */
};

/* Operation selector for layout queries. */
enum {
  FC_OP_TX = 0,      /* fc_tx_synthesize: low-rate CP-OFDM in, high-rate out            */
  FC_OP_RX = 1,      /* fc_rx_analyze:    high-rate in, low-rate out                    */
  FC_OP_ADJ = 2,     /* fc_tx_adjoint:    high-rate in, low-rate CP-OFDM-shaped out     */
  FC_OP_RXD = 3,     /* fc_rx_demodulate: high-rate in, subcarriers out (synchronised)   */
  FC_OP_TXG = 4      /* fc_tx_modulate:   QAM grid in, high-rate out (synchronised)      */
};

/*
 * One subband (Sec. III-A/III-B; the paper's subband m).
 *   scs_khz       subcarrier spacing 15 * 2^mu kHz (selects the NR CP rule)
 *   first_symbol  index of the first symbol within its subframe (long-CP symbols
 *                 are l = 0 and l = 7 * 2^mu of the subframe)
 *   n_symbols     B_OFDM,m, number of OFDM symbols in the burst (>= 1)
 *   n_active      L_act,m, active subcarriers K (even); passband kappa in [-K/2, K/2)
 *   n_tb          transition-band bins per side (default weights, validation)
 *   n_short       L_m = L_OFDM,m: a power of two in [16, 4096], or 3 x 2^k in
 *                 [768, 3072] (mixed radix, e.g. the 768 = 3 x 256 of Sec. VI-C)
 *   n_long        N in the same set, >= n_short, with N / n_short a power of
 *                 two (FC_E_SHAPE otherwise); other lengths FC_E_UNSUPPORTED
 *   center_bin    c_m, subband centre in long-transform bins (signed)
 *   overlap_num/overlap_den  overlap factor lambda; synchronised modes need 1/2,
 *                 continuous modes need 0 < lambda <= 1/2 with lambda*L_m even
 *   mode          FC_CONT_OLA .. FC_SYNC_OLS
 *   stream        index of the high-rate stream this subband is summed into /
 *                 analysed from; streams are numbered 0..n_streams-1 densely
 *   ncp_high      optional per-symbol high-rate CP lengths N_CP,n (n_symbols
 *                 entries, read during fc_plan_create only); NULL selects the
 *                 NR normal CP at rate n_long * SCS
 *   taper         FC_SYNC_OLS only (0 otherwise): length T (even, high-rate
 *                 samples) of the smooth outer edges of the TX output windows
 *                 (Sec. III-D): the rising edge of s_0 and the falling edge of
 *                 s_1 become raised-cosine ramps w_i = sin^2(pi (i + 1/2)/(2T))
 *                 over the T samples centred on the hard edge, so the edges of
 *                 neighbouring symbols cross-fade; T/2 <= N_L - N_CP,n for every
 *                 symbol and T/2 <= N_T; 0 keeps the hard edges. The receiver
 *                 does not depend on it.
 */
typedef struct fc_subband {
  int32_t scs_khz;
  int32_t first_symbol;
  int32_t n_symbols;
  int32_t n_active;
  int32_t n_tb;
  int32_t n_short;
  int32_t n_long;
  int32_t center_bin;
  int32_t overlap_num;
  int32_t overlap_den;
  int32_t mode;
  int32_t stream;
  const int32_t* ncp_high;
  int32_t taper;
} fc_subband;

typedef struct fc_plan fc_plan;

/*
 * Build a plan for n_sb subbands on device `device` with I/O type io_type.
 * device = -1 builds a host-only plan: schedules, layouts and validation
 * without device memory; compute calls on it return FC_E_STATE.
 * Validates every subband (Sec. III-B/III-E constraints: n_short | n_long,
 * K + 2 n_tb <= n_short, |c| + n_short/2 <= n_long/2, integer low-rate CP in
 * continuous modes, truncated low-rate CP <= n_short/4 in synchronised modes,
 * equal numerology, symbol count and CP schedule among subbands sharing a
 * stream and n_long in one processing group). Initialises every subband's
 * weights to a raised-cosine transition of n_tb bins. *plan receives the plan
 * (or NULL on failure). Device memory for the plan's tables is allocated here,
 * and, when every subband is synchronised, the scratch of fc_rx_demodulate:
 * 8 bytes per subband bin per workgroup task (sum_m n_short_m x 8 bytes for
 * each task, a task holding run_len / 2 symbols of one processing group),
 * reallocated when fc_plan_set_tuning changes FC_OP_RXD.
 */
fc_status fc_plan_create(const fc_subband* sb, int32_t n_sb, int32_t io_type, int32_t device,
                         fc_plan** plan);

/* Release the plan and its device tables (after the queued work completed). */
void fc_plan_destroy(fc_plan* plan);

/* Number of subbands and streams of the plan. */
fc_status fc_plan_counts(const fc_plan* plan, int32_t* n_sb, int32_t* n_streams);

/*
 * Buffer layout for operation `op`, in complex samples (not bytes):
 *   lowrate_off[n_sb + 1]       subband m's low-rate samples are
 *                               [lowrate_off[m], lowrate_off[m+1])
 *   highrate_off[n_streams + 1] stream s's high-rate samples are
 *                               [highrate_off[s], highrate_off[s+1])
 * Low-rate layout: FC_OP_TX / FC_OP_ADJ and continuous FC_OP_RX use the
 * concatenated CP-OFDM symbols (sum_n n_short + L_CP,n); synchronised FC_OP_RX
 * returns n_symbols * n_short samples (CP removed, Sec. IV concatenation), and
 * FC_OP_RXD n_symbols * n_short subcarrier values, FC_OP_TXG (input) the
 * QAM grid, n_symbols * n_active values.
 * Either pointer may be NULL.
 */
fc_status fc_plan_layout(const fc_plan* plan, int32_t op, int64_t* lowrate_off,
                         int64_t* highrate_off);

/*
 * Per-symbol CP schedule of subband sb: ncp_high[n] = N_CP,n (high rate),
 * ncp_low[n] = L_CP,n (low rate; floor(N_CP,n / I) in synchronised modes,
 * Sec. III-E). Arrays of n_symbols entries; either may be NULL.
 * offset (may be NULL) receives the position, in its stream, of sample 0 of
 * this subband's local high-rate axis (groups on one stream are aligned so that
 * their first CPs start together).
 */
fc_status fc_plan_symbols(const fc_plan* plan, int32_t sb, int32_t* ncp_high, int32_t* ncp_low,
                          int64_t* offset);

/*
 * Frequency-domain window D_m of subband sb (Sec. III-B): n == n_short real
 * weights in fftshifted order (index p is subcarrier kappa = p - n_short/2).
 * Host pointer, copied; the device copy is updated on `stream` and the call
 * returns once that copy has completed. Non-finite weights are rejected.
 */
fc_status fc_set_weights(fc_plan* plan, int32_t sb, const float* w_host, int32_t n, void* stream);

/*
 * Same as fc_set_weights with a device pointer w_dev: an asynchronous
 * device-to-device copy on `stream`; the host is not synchronised and
 * fc_get_weights reads the device copy. sb >= 0: n == that subband's
 * n_short floats; sb == -1: every subband's weights at once, concatenated in
 * plan order (n == sum_m n_short_m, the layout of fc_tx_weight_grad's
 * grad_w). The values are not read on the host and NOT checked for
 * finiteness: the caller must pass finite weights (a NaN or Inf reaches
 * every output sample of its subband and grad_w). Errors: FC_E_ARG,
 * FC_E_SHAPE, FC_E_STATE (host-only plan), FC_E_DEVICE.
 */
fc_status fc_set_weights_device(fc_plan* plan, int32_t sb, const float* w_dev, int32_t n, void* stream);

/* Copy subband sb's current weights (n == n_short) to host memory w_host
 * (waits for the device). */
fc_status fc_get_weights(const fc_plan* plan, int32_t sb, float* w_host, int32_t n);

/*
 * FC synthesis filter bank (Sec. III-B, eq. for x_FC-F-OFDM; Sec. III-C..III-E):
 * lowrate_in (device, FC_OP_TX layout) -> highrate_out (device, all streams).
 * Every sample of every stream is written (zeros where no block contributes);
 * subbands on one stream are summed. All four modes; FC_SYNC_OLS is the
 * synchronised scheme's OLS alternative (Sec. III-D: no input windows, each
 * filtered block kept on s_0 = [0; 1_{N_S + N_CP,n}; 0] from the CP start or
 * s_1 = [0_{N_L}; 1_{N_S}; 0_{N_T}]; hard edges, or smooth outer edges of the
 * subband's taper length, see fc_subband).
 */
fc_status fc_tx_synthesize(fc_plan* plan, const void* lowrate_in, void* highrate_out, void* stream);

/*
 * FC analysis filter bank (Sec. IV): highrate_in (device) -> lowrate_out
 * (device, FC_OP_RX layout). FC_CONT_OLS / FC_CONT_OLA use G^(OLS) / G^(OLA)
 * with conj(phi) and scale 1/sqrt(I); synchronised modes use two blocks per
 * symbol and return the CP-free symbols (Sec. IV concatenation).
 */
fc_status fc_rx_analyze(fc_plan* plan, const void* highrate_in, void* lowrate_out, void* stream);

/*
 * CP-OFDM modulation and synchronised FC synthesis in one pass (Sec. III-A
 * modulation with L_OFDM = n_short and the truncated low-rate CP of
 * Sec. III-E, then the Sec. III-C/D synthesis): the kernels run each symbol's
 * L-point IFFT in LDS and take the FC blocks from it, so the low-rate
 * CP-OFDM signal never goes to memory.
 *   grid_in       device, FC_OP_TXG layout: per subband n_symbols rows of
 *                 n_active values (subcarriers kappa = -K/2 .. K/2-1), the
 *                 plan's I/O type; x_n = sqrt(L) W_L^{-1} X_n.
 *   highrate_out  device, high-rate layout, as fc_tx_synthesize.
 * Every subband must be synchronised (FC_SYNC_OLA or FC_SYNC_OLS), else
 * FC_E_STATE. Asynchronous on `stream`; errors as fc_tx_synthesize.
 */
fc_status fc_tx_modulate(fc_plan* plan, const void* grid_in, void* highrate_out, void* stream);

/*
 * Synchronised FC analysis followed by OFDM demodulation (Sec. IV, with
 * L_OFDM = n_short): for every symbol n of every subband,
 * x_hat_n = (1/sqrt(L)) W_L x_hat_OFDM,n, the subcarrier values, computed in
 * the simplified joint form of Sec. V-A (one short IFFT and one FFT per symbol
 * instead of two IFFTs and an FFT): with g0, g1 the two blocks' weighted and
 * phase-rotated bins, x = C(A - B) + B, A[k] = g0[k] j^k, B[k] = g1[k] (-j)^k,
 * C the half-band matrix W_L diag(1_{L/2}, 0_{L/2}) W_L^{-1}.
 *   highrate_in      device, high-rate layout, the plan's I/O type.
 *   subcarriers_out  device, FC_OP_RXD layout (per subband n_symbols * n_short
 *                    values, symbol by symbol; subcarrier kappa of a symbol at
 *                    index kappa mod n_short), the plan's I/O type.
 * Every subband must be synchronised (FC_SYNC_OLA or FC_SYNC_OLS), else
 * FC_E_STATE. Asynchronous on `stream`; errors as fc_rx_analyze. Each task
 * keeps its symbols' B terms in its own slot of plan-owned device scratch
 * (allocated with the plan's tables): calls on one plan that overlap in time
 * on different streams race on it.
 */
fc_status fc_rx_demodulate(fc_plan* plan, const void* highrate_in, void* subcarriers_out, void* stream);

/*
 * Exact adjoint of fc_tx_synthesize (used for gradients): highrate_in ->
 * lowrate_out in the FC_OP_TX low-rate layout, so that
 * <tx(x), y> = <x, adjoint(y)> for the plan's current weights (the RX block
 * operators with the OLA / OLS roles swapped, Sec. IV). Every lowrate_out
 * sample is written. Not provided for plans with an FC_SYNC_OLS subband
 * (FC_E_STATE). Asynchronous on `stream`; errors as fc_rx_analyze.
 */
fc_status fc_tx_adjoint(fc_plan* plan, const void* highrate_in, void* lowrate_out, void* stream);

/*
 * Gradient of the real functional J = Re<g, tx(x)> with respect to every
 * subband's real weights D (Sec. III: the output is linear in D, so
 * dJ/dD_p = Re<g, b_p> with b_p the output for a unit weight at bin p; this
 * is also the weight gradient of any real loss whose complex output gradient,
 * in PyTorch's conjugate-Wirtinger convention, is g).
 *   lowrate_in  device, FC_OP_TX low-rate layout, the plan's I/O type: the
 *               forward input x.
 *   grad_out    device, high-rate layout (all streams), the plan's I/O type: g.
 *   grad_w      device float array of sum_m n_short_m entries (subbands in
 *               plan order, fftshifted order within a subband, as
 *               fc_set_weights): overwritten with
 *               sum over blocks of Re(conj(G_q) * phase * X_p),
 *               X the block's short FFT of x, G the long FFT of the matching
 *               block of g scaled like the adjoint, q = Xi(p).
 * Buffers are owned by the caller. Asynchronous on `stream`; the result does
 * not depend on the plan's current weights. Scheduled over the adjoint's
 * blocks in tasks of four consecutive blocks of a group (a fixed split); the
 * FC_OP_ADJ concurrency (fc_plan_set_tuning) sets its launches in flight.
 * Each task stores its per-bin sums in its own slot of a plan-owned scratch
 * buffer (4 bytes x the sum over tasks of the n_short of the task's
 * subbands), and a reduction adds every weight's slots in block order: the
 * summation tree is fixed, so the result is bitwise the same for every tuning
 * and every call. The scratch is allocated (hipMalloc) by the first call and
 * kept until fc_plan_destroy, so a graph capture (fc_graph_begin) may record
 * this call only after one uncaptured call on the plan (or use
 * fc_tx_weight_grad_noalloc). Errors:
 * FC_E_ARG (null pointer), FC_E_STATE (host-only plan, a plan with an
 * FC_SYNC_OLS subband, which has no adjoint, or a first call on a capturing
 * stream), FC_E_NOMEM (scratch), FC_E_DEVICE (launch failure).
 */
fc_status fc_tx_weight_grad(fc_plan* plan, const void* lowrate_in, const void* grad_out,
                            float* grad_w, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * computation as fc_tx_weight_grad, with the same kernels and the same fixed
 * summation tree (bitwise the same result), but the per-task partial sums go
 * to a fixed device array of FC_NOALLOC_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends, instead of plan-owned
 * scratch. It calls no hipMalloc, hipFree or other allocating routine; the
 * caller passes every input and output, as for fc_tx_weight_grad.
 * The array is shared by every call on one GPU: calls that overlap in time on
 * one GPU (from any plan, stream or host thread) race and give wrong results;
 * calls ordered on one stream, or otherwise serialised, are safe. Nothing in
 * it needs clearing between calls (every slot is written before it is read).
 * Errors: as fc_tx_weight_grad (no FC_E_NOMEM), and FC_E_LIMIT when the
 * plan's partial sums (4 bytes x the sum over the gradient's tasks of their
 * subbands' n_short) exceed FC_NOALLOC_SCRATCH_BYTES; nothing is queued then.
 */
fc_status fc_tx_weight_grad_noalloc(fc_plan* plan, const void* lowrate_in, const void* grad_out,
                                    float* grad_w, void* stream);

/* Work decomposition of operation op: FC blocks, tasks (workgroup work
 * items) and kernel launches per call. Either pointer may be NULL. */
fc_status fc_plan_stats(const fc_plan* plan, int32_t op, int64_t* n_blocks, int64_t* n_tasks,
                        int64_t* n_launches);

/*
 * Tuning of operation op (FC_OP_TX .. FC_OP_TXG; FC_OP_ADJ's conc also
 * applies to the weight gradient, whose blocks per task are fixed):
 *   run_len  FC blocks per workgroup task (consecutive blocks of one group;
 *            0 = the planner's choice from the total block count; TX runs of
 *            synchronised groups are rounded up to whole symbols; RX tasks
 *            that accumulate into shared samples always hold one block);
 *   conc     1..4: how many launches of one independent set (kernel classes
 *            writing disjoint outputs) may run at once, on the caller's
 *            stream plus side streams owned by the plan.
 * Results do not depend on run_len or conc (same arithmetic per block).
 * fc_plan_set_tuning waits for the plan's device to go idle and rebuilds the
 * op's work tables (freeing the old ones): graphs captured before hold the
 * old tables' addresses and must be captured again. Errors: FC_E_ARG (out
 * of range), FC_E_STATE (op not available for this plan), FC_E_NOMEM /
 * FC_E_DEVICE.
 */
fc_status fc_plan_set_tuning(fc_plan* plan, int32_t op, int32_t run_len, int32_t conc);
fc_status fc_plan_get_tuning(const fc_plan* plan, int32_t op, int32_t* run_len, int32_t* conc);

/*
 * Transform plan of operation op (FC_OP_TX .. FC_OP_TXG), 0 (default) or 1,
 * a choice between precompiled kernels: for the TX operations, the other
 * placement of the short FFTs of single-subband groups with a pruned long
 * IFFT and n_short <= 1024 (one wave per block, blocks in groups, against
 * the whole workgroup, one block at a time); for FC_OP_RX, FC_OP_ADJ and
 * FC_OP_RXD, the long FFT with the next lower radix (radix-8 passes at
 * n_long = 4096, radix 4 at 2048). Elsewhere both plans are the same kernel.
 * Plan 1 changes the order of the FP32 operations, so results differ from
 * plan 0 by rounding. Set like fc_plan_set_tuning (device idle, tables
 * rebuilt, graphs must be captured again); setting it applies to every
 * kernel class of the op. fc_plan_autotune chooses it too, and then, kernel
 * class by kernel class (one launch per class), the other plan where that
 * makes the whole call faster; fc_plan_get_transform_plan returns the op's
 * plan, fc_plan_get_class_plans how many of the op's kernel classes have two
 * plans (*n_classes) and how many of those run plan 1 (*n_plan1).
 * Errors: FC_E_ARG (op or plan out of range, NULL result pointer),
 * FC_E_STATE, FC_E_NOMEM, FC_E_DEVICE.
 */
fc_status fc_plan_set_transform_plan(fc_plan* plan, int32_t op, int32_t tplan);
fc_status fc_plan_get_transform_plan(const fc_plan* plan, int32_t op, int32_t* tplan);
fc_status fc_plan_get_class_plans(const fc_plan* plan, int32_t op, int32_t* n_classes, int32_t* n_plan1);

/*
 * Autotuner: times op on the caller's buffers (in / out as for the op's
 * call; out is overwritten) for run_len in {0, 8, 16, 32, 64} (TX) or
 * {0, 1, 2, 4, 8, 16} (RX, adjoint; {0, 2, 4, 8, 16} demodulating RX) and
 * conc in {1, 4}, and the transform plans 0 and 1 where they differ for
 * this op (fc_plan_set_transform_plan), each by one warm-up call and three
 * bursts of four calls back to back (HIP events on `stream`, the shortest
 * burst's time per call kept; on a stream other than the legacy null stream
 * the call is captured once as a HIP graph and the replays are timed, so
 * host launch gaps do not enter the choice), then applies the
 * fastest. With conc > 1 each candidate is timed twice: with the launches
 * spread over the streams longest first by the planner's work estimate, and
 * by their measured times (every kernel launch of the op timed on its own);
 * the better order is kept (until the next fc_plan_set_tuning). Last, class by
 * class (largest first), it keeps the other transform plan for a kernel
 * class where the whole call then times at least 1.5 % faster. Synchronous.
 * The chosen values and time per call (ms) are written to the non-NULL
 * result pointers; the chosen transform plans are read back with
 * fc_plan_get_transform_plan and fc_plan_get_class_plans.
 */
fc_status fc_plan_autotune(fc_plan* plan, int32_t op, const void* in, void* out, void* stream,
                           int32_t* best_run_len, int32_t* best_conc, float* best_ms);

/*
 * HIP graphs of FC calls. fc_graph_begin starts a capture of `stream` (not
 * the legacy null stream); every fc_* call issued on it until fc_graph_end
 * is recorded (kernel launches, fills, fork/join of the side streams; none
 * allocates or synchronises), and fc_graph_end instantiates the graph.
 * Issue the calls on `stream` itself: calls issued on other streams that
 * joined the capture through events are not supported.
 * fc_graph_launch replays it on any stream. Plans and buffers are recorded
 * by address and must outlive the graph, and so must the plans' work tables:
 * fc_plan_set_tuning and fc_plan_autotune rebuild them, so capture after
 * tuning. Weights changed later with fc_set_weights* are used by later
 * replays. Errors: FC_E_ARG, FC_E_DEVICE (capture or instantiation failed,
 * e.g. a non-capturable call in between).
 */
typedef struct fc_graph fc_graph;
fc_status fc_graph_begin(void* stream);
fc_status fc_graph_end(void* stream, fc_graph** graph);
fc_status fc_graph_launch(fc_graph* graph, void* stream);
void fc_graph_destroy(fc_graph* graph);

/* Human-readable name of a status code (static string). */
const char* fc_status_str(fc_status s);

/* Library version string, e.g. "fc 0.1 gfx950". */
const char* fc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FC_H_ */
