/*
 * polyspec.h -- C ABI of the MI355X (gfx950) polyspectrum library.
 *
 * The library computes the unbiased polyspectrum estimates of
 * Sifft, Ghorbanietemad, Wagner and Haegele, "Correct Estimation of
 * Higher-Order Spectra" (arXiv 2505.01231):
 *
 *   a_k(f)      = dt sum_{i<N} g_i z_{fN+i} exp(+2 pi j i k / N)   (Section 3, eq. a_k;
 *                                                                  +j sign of Appendix A)
 *   S2_ab(k)    = c2(a_k, b*_k)          / (dt sum g^2)            (Section 3; Section 7)
 *   S3_abc(k,l) = c3(a_k, b_l, c*_{k+l}) / (dt sum g^3)            (Section 4; Section 7)
 *   S4_abcd(k,l)= c4(a_k, b*_k, c_l, d*_l)/ (dt sum g^4)           (Section 4 cut; Section 7)
 *
 * with c2..c4 the multivariate k-statistics of Section 4.1 evaluated over the
 * m consecutive frames of one chunk, averaged over the Np chunks of a record,
 * with error bars sigma = sqrt(Var/Np), Var = Np/(Np-1)(mean(x^2)-mean(x)^2)
 * taken separately for the real and imaginary parts (Section 4.2).
 *
 * Frames are contiguous, non-overlapping blocks of N samples; a chunk is m
 * consecutive frames; Np = floor(floor(L / N) / m); leftover samples are not
 * used.  The output grid is k, l = 0..N_f-1 (frequency k / (N dt)).
 *
 * Conventions shared by every entry point:
 *  - Every pointer named d_* is a device (HBM) pointer on the current HIP
 *    device; every other pointer is host memory.  The caller owns all device
 *    buffers it passes (inputs, workspace, outputs).  The library allocates
 *    memory only in these calls, each freed by the matching destroy:
 *      ps_plan_create        window, twiddle and tile tables (device) and, on
 *                            the first execute, a pinned host staging area for
 *                            the work tables (grown when an execute needs more)
 *                            -> ps_plan_destroy;
 *      ps_graph_create       the graph's work tables (device) -> ps_graph_destroy;
 *      ps_streamer_create(_multi)  staging slots and workspace (device)
 *                            -> ps_streamer_destroy;
 *      ps_stream_begin       accumulator state, carry buffer, workspace and work
 *                            tables (device) -> ps_stream_destroy.
 *    ps_execute, ps_execute_sequential, ps_coefficients, ps_full_plane,
 *    ps_spectra_zscore and the push / launch / end calls allocate no device
 *    memory; ps_plan_autotune creates two events and destroys them before it
 *    returns.
 *  - Calls that take a stream only enqueue work on it and return; results are
 *    valid after the caller synchronises that stream.  A plan must not be used
 *    by two streams at the same time.
 *  - Errors are reported by return code only; nothing unwinds across the ABI.
 *    ps_last_error() returns a thread-local description of the last failure.
 *    Argument errors are detected before anything is enqueued.  Device faults
 *    surface at the caller's synchronisation (and as PS_E_HIP from a later call).
 */
#ifndef POLYSPEC_H
#define POLYSPEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PS_ABI_VERSION 1

typedef struct ps_plan_s* ps_plan_t;
typedef void* ps_stream_t; /* a hipStream_t; NULL is the null stream */

typedef enum ps_status {
    PS_OK = 0,
    PS_E_INVALID_ARG = 1, /* a parameter is out of range, a pointer is NULL or misaligned */
    PS_E_UNSUPPORTED = 2, /* valid per the paper but not implemented here (e.g. complex records at N not a power of two) */
    PS_E_WORKSPACE = 3,   /* workspace smaller than ps_workspace_size() */
    PS_E_HIP = 4,         /* a HIP runtime call failed */
    PS_E_INTERNAL = 5
} ps_status;

typedef enum ps_dtype {
    PS_F32 = 0, PS_F64 = 1, PS_I16 = 2,
    PS_C64 = 3,   /* complex: interleaved float32 (re, im); plans with complex_signal = 1 */
    PS_C128 = 4   /* complex: interleaved float64 */
} ps_dtype;
typedef enum ps_estimator { PS_EST_KSTAT = 0, PS_EST_NATURAL = 1, PS_EST_C3OPT = 2 } ps_estimator;

/* Window g_i, i = 0..N-1.  HANN: symmetric sin^2(pi i/(N-1)); HANN_PERIODIC:
 * sin^2(pi i/N); ACG: the approximate confined Gaussian of Appendix B with
 * sigma_t = window_param (the paper's default 0.14, Section 3). */
typedef enum ps_window { PS_WIN_HANN = 0, PS_WIN_HANN_PERIODIC = 1, PS_WIN_ACG = 2 } ps_window;

/* Arithmetic of the S4 frame contractions (Sections 4 and 4.1):
 *  FP32    plain FP32 vector arithmetic;
 *  BF16X3  each FP32 operand split into three bfloat16 terms, six cross products
 *          on the matrix cores with FP32 accumulation;
 *  FP16X2S each operand scaled per chunk and frequency by a power of two and split
 *          into two float16 terms, three cross products on the matrix cores
 *          (requires m <= 10, else PS_E_UNSUPPORTED).
 * The k-statistic combination and the chunk average are FP64 in every mode. */
typedef enum ps_precision { PS_PREC_FP32 = 0, PS_PREC_BF16X3 = 1, PS_PREC_FP16X2S = 2 } ps_precision;

/* BATCHED: every chunk of a record in one pass of each kernel.
 * PER_CHUNK: one short-time estimate (one chunk) per launch, the structure the
 * paper describes for its own library (Section 10); kept as the reference
 * "plain" schedule. */
typedef enum ps_schedule { PS_SCHED_BATCHED = 0, PS_SCHED_PER_CHUNK = 1 } ps_schedule;

#define PS_ORDER_S1 (1u << 1) /* first-order spectrum: the windowed mean (Section 3) */
#define PS_ORDER_S2 (1u << 2)
#define PS_ORDER_S3 (1u << 3)
#define PS_ORDER_S4 (1u << 4)

/* Per-record flags returned by ps_record_info. */
#define PS_FLAG_EMPTY 1u     /* no complete chunk: every output is NaN */
#define PS_FLAG_NO_ERRBAR 2u /* Np == 1: error bars are NaN */

typedef struct ps_config {
    uint32_t struct_size; /* sizeof(ps_config) */
    uint32_t orders;      /* PS_ORDER_* bitmask, non-zero */
    int32_t n_channels;   /* 1..4 (Section 7) */
    int32_t frame_len;    /* N: 256..8192; a power of two takes the FFT, any other length the direct transform */
    int32_t n_freq;       /* N_f; 0 => floor(f_max * N * dt) + 1 */
    int32_t m;            /* frames per chunk: >= 1 (S1), >= 2 (S2), >= 3 (S3), >= 4 (S4) */
    double f_max;         /* used only when n_freq == 0 */
    double dt;            /* sampling step, > 0 */
    double window_param;  /* sigma_t for PS_WIN_ACG (> 0) */
    int32_t window;       /* ps_window */
    int32_t precision;    /* ps_precision */
    int32_t schedule;     /* ps_schedule */
    int32_t n_combos2;    /* channel combinations; 0 => every orbit (see below) */
    int32_t n_combos3;
    int32_t n_combos4;
    const int8_t* combos2; /* host [n_combos2][2]: (a, b) -> C2(a_k, b*_k) */
    const int8_t* combos3; /* host [n_combos3][3]: (a, b, c) -> C3(a_k, b_l, c*_{k+l}) */
    const int8_t* combos4; /* host [n_combos4][4]: (a, b, c, d) -> C4(a_k, b*_k, c_l, d*_l) */
    int32_t interlaced;    /* 0 or 1: interlaced windows (see below); PS_SCHED_BATCHED only */
    int32_t estimator;     /* ps_estimator */
    int32_t complex_signal; /* 0: real records; 1: complex records (PS_C64 / PS_C128), see below */
    int32_t s4_shift;      /* q: S4 on a plane parallel to the cut (complex_signal = 1), see below */
    int32_t frame_len_set; /* further frame lengths records may carry: bit q (8..13) admits N = 2^q (see below) */
} ps_config;
/* Several frame lengths in one execute (frame_len_set != 0; real signals,
 * power-of-two frame_len): a record whose ps_record.frame_len is 2^q with bit
 * q set is cut into frames of that length; frame_len 0 means the plan's.
 * Each frame length has its own window (same kind and sigma_t), Fourier
 * coefficients and grid: N_f scales with the frame length when n_freq is
 * given (n_freq * 2^q / frame_len, which must be an integer), else follows
 * f_max as for the plan's (floor(f_max 2^q dt) + 1); the constraints on N_f
 * hold per frame length.  Every record's spectra use its own grid (outputs
 * sized by ps_plan_frame_info).  All records of an execute, whatever their
 * frame length, share each stage's launch.  ps_full_plane, the streamer and
 * the running accumulation take the plan's frame length only. */
/* Complex-valued signals (complex_signal = 1; frame_len up to 4096): without
 * a_{-k} = a_k* the negative frequencies carry their own information, so every
 * spectrum is computed on the signed grid k, l in (-N_f, N_f): S2 has 2 N_f - 1
 * points, S3 and S4 (2 N_f - 1)^2, index k + N_f - 1 (ps_plan_info.grid), and
 * S1 is complex.  Same definitions (Sections 3, 4 and 7) and constraints on
 * N_f; ps_full_plane does not apply (the grid is already the full plane).
 * The conjugated arguments are those of the real-signal formulas, so S2_ab of
 * complex records is C2(a_k, b*_k) (the power spectrum for a = b); the
 * unconjugated negative-frequency components of the general definition are
 * obtained by passing conj(b) as channel b.
 *
 * Planes of the three-dimensional fourth-order spectrum (Appendix on the full
 * S4): s4_shift = q != 0 computes every S4 combination on the plane parallel
 * to the cut, S4_abcd(k, l) = C4(a_{k+q}, b*_{k-q}, c_{l-q}, d*_{l+q}), i.e. the
 * full spectrum at (k + q, -k + q, l - q) for real data; it needs
 * complex_signal = 1 (pass real records as complex), N_f - 1 + |q| <= N/2, and
 * then uses every channel combination (no symmetry maps a plane onto itself
 * for q != 0; explicit lists are taken as given). */
/* Cumulant estimator per chunk.  PS_EST_KSTAT: the unbiased k-statistics of
 * Section 4.1.  PS_EST_NATURAL: the natural (plug-in) estimator of Section 6,
 * the cumulant's moment expression with sample means (biased by O(1/m); for
 * comparisons).  PS_EST_C3OPT: S3 by c3^(opt), the estimator of the closing
 * remark of Section 4.1 for zero-mean data, symmetrised over the three
 * factors: mean(xyz) - (m-1)/(m+1) [U(xy,z) + U(xz,y) + U(yz,x)], U(p, r) the
 * average of p_i r_j over distinct frames i != j; of least variance for
 * Gaussian-dominated data, unbiased where every factor has mean zero (away
 * from bin 0 and the bins the window leaks a mean into) and biased elsewhere;
 * S3 then needs m >= 2, and S2 and S4 keep the k-statistics.  It costs one
 * more row per chunk in S3 and C * chunks * (m + 1) * K * 8 bytes of
 * workspace.  S1 (the mean) is the same under all. */
/* Interlaced windows (Section 3): the centre of a window weighs the signal more
 * than its edges; the same spectra computed on windows shifted by T/2 weigh it
 * the other way.  With interlaced = 1 every record (or streamer window) is
 * processed twice, as the frame set starting at sample 0 and as the set
 * starting at sample N/2, each cut into its own chunks, and the output is the
 * average of the two spectra.  Its error bar is the average of the two error
 * bars: the sets overlap, so their estimates are positively correlated, and
 * this average is never below the error of the averaged spectrum.  When the
 * shifted set has no complete chunk the output is the first set's alone.
 * ps_record_info reports the first set (Np, flags). */
/* "Every orbit": combinations related by the symmetries of Section 9 that keep
 * the output grid are computed once.  S2: (a,b) with a <= b (S2_ba = conj S2_ab).
 * S3: (a,b,c) with a <= b (S3_bac(k,l) = S3_abc(l,k)).  S4: the lexicographically
 * smallest of {abcd, badc, cdab, dcba} (S4_badc = conj S4_abcd,
 * S4_cdab(k,l) = S4_abcd(l,k)).  For 4 channels: 10, 40 and 76 combinations. */

typedef struct ps_record {
    const void* d_data;     /* sample 0 of channel 0; element type `dtype`, 4/8/2-byte aligned */
    int64_t n_samples;      /* samples per channel (L) */
    int64_t channel_stride; /* elements from one channel's sample 0 to the next's */
    int32_t dtype;          /* ps_dtype; int16 samples are used in LSB units */
    int32_t frame_len;      /* 0: the plan's frame_len; else a frame length of the plan's frame_len_set */
} ps_record;

/* Output of one record.  Spectra are FP64 interleaved complex (re, im); error
 * bars are (sigma_re, sigma_im) pairs.  Layouts: S2 [n_combos2][N_f],
 * S3 and S4 [n_combos][N_f][N_f] with index [k][l], S1 [n_channels] (one value
 * per channel: S1_a = C1(a_0) / (dt sum g), the windowed mean; real, so its
 * imaginary part and sigma_im are 0).  Any pointer may be NULL if its order
 * was not requested.  Units: (input unit)^n * dt^(n-1). */
typedef struct ps_output {
    double* d_s2;
    double* d_s2_err;
    double* d_s3;
    double* d_s3_err;
    double* d_s4;
    double* d_s4_err;
    double* d_s1;     /* PS_ORDER_S1 */
    double* d_s1_err;
} ps_output;

typedef struct ps_plan_info {
    int32_t frame_len;  /* N */
    int32_t n_freq;     /* N_f */
    int32_t n_coef;     /* coefficients kept per frame: 2 N_f - 1 with S3, else N_f */
    int32_t m;
    int32_t n_combos2, n_combos3, n_combos4;
    int32_t grid;       /* points per output axis: N_f, or 2 N_f - 1 for complex signals */
    double f_max;       /* (N_f - 1) / (N dt) */
    double sum_g[5];    /* sum_i g_i^n, n = 0..4, as used by the normalisation */
    const int8_t* combos2; /* host, owned by the plan */
    const int8_t* combos3;
    const int8_t* combos4;
} ps_plan_info;

/* Validate `cfg`, build the window (FP64 on the host: Hann, or the confined
 * Gaussian of Appendix B) and the FFT tables of eq. a_k (Section 3), enumerate
 * the channel-combination orbits (Section 9) and pick launch shapes.
 * Validation follows the estimator's definitions: m >= order (the
 * denominators of eq. c2..c4, Section 4.1); 2 (N_f - 1) <= N/2 when S3 is
 * requested (its third factor a_{k+l}, Section 4), else N_f - 1 <= N/2;
 * N in 256..8192.  The paper takes N a power of two, or at least a product of
 * small primes, for the FFT (Section 3); a power of two here runs the FFT,
 * any other length the direct transform of eq. a_k (FP64 accumulation, in
 * two stages N = N1 N2 when N has a divisor 8 <= N1 <= sqrt(N), else in one;
 * slower than the FFT; real records, one frame length per plan).  Allocates the plan's small device tables on the current device
 * (synchronous).  On failure *out is NULL and the status is PS_E_INVALID_ARG
 * (a parameter out of range), PS_E_UNSUPPORTED (allowed by the paper, not
 * built here, e.g. complex records at a frame length that is not a power of
 * two) or PS_E_HIP. */
ps_status ps_plan_create(const ps_config* cfg, ps_plan_t* out);

/* Free the plan and its device tables (synchronous).  NULL is accepted. */
ps_status ps_plan_destroy(ps_plan_t plan);

ps_status ps_plan_query(ps_plan_t plan, ps_plan_info* info);

/* Np and PS_FLAG_* for a record of n_samples samples per channel at the
 * plan's frame length (with interlaced windows: of the frame set that starts
 * at sample 0). */
ps_status ps_record_info(ps_plan_t plan, int64_t n_samples, int64_t* n_chunks, uint32_t* flags);

/* The same for a record at its own frame length (rec->frame_len). */
ps_status ps_record_chunks(ps_plan_t plan, const ps_record* rec, int64_t* n_chunks, uint32_t* flags);

/* ps_plan_query for one of the plan's frame lengths (frame_len 0 or the
 * plan's: ps_plan_query): its N_f, coefficient count, grid, f_max and window
 * sums.  PS_E_INVALID_ARG for a frame length the plan does not hold. */
ps_status ps_plan_frame_info(ps_plan_t plan, int32_t frame_len, ps_plan_info* info);

/* Device workspace (bytes) that ps_execute needs for these records: the
 * FP32 Fourier coefficients of every frame of every complete chunk (eq. a_k,
 * K = 2 N_f - 1 per frame with S3, else N_f; chunks as in Section 4.2), the
 * work tables and the FP64 partial sums over chunks.  Host only; records are
 * validated as by ps_execute (PS_E_INVALID_ARG). */
ps_status ps_workspace_size(ps_plan_t plan, const ps_record* recs, int32_t n_rec, size_t* bytes);

/* Enqueue the whole estimator for n_rec records on `stream`: windowed real FFT
 * per frame (Section 3, eq. a_k), per-chunk centring and moment sums, the
 * k-statistics of Section 4.1 (eq. c2..c4; multichannel arguments of
 * Section 7), the spectra's normalisation (Sections 3 and 4), and the FP64
 * chunk average with the error bars of Section 4.2.  recs[i] is read-only;
 * outs[i] (caller-owned, layouts of ps_output) receives record i; a record
 * without a complete chunk gets NaN outputs.  d_ws must be 256-byte aligned
 * and at least ps_workspace_size() bytes; its contents are scratch.
 * Errors (nothing enqueued): PS_E_INVALID_ARG for NULL, misaligned or
 * inconsistent arguments, PS_E_UNSUPPORTED for a record of more than 2^31 - 1
 * chunks, PS_E_WORKSPACE for a small workspace, PS_E_HIP when a launch fails. */
ps_status ps_execute(ps_plan_t plan, const ps_record* recs, int32_t n_rec, void* d_ws,
                     size_t ws_bytes, const ps_output* outs, ps_stream_t stream);

/* Allocation-free form of ps_execute, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same estimator and outputs as ps_execute, with the
 * workspace taken from a static device array of PS_STATIC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends (its
 * address is resolved for a device when the first plan is created there).
 * The call allocates nothing: no device memory, no pinned host memory, no
 * events (stage timing is not recorded).  Limits: ps_workspace_size() of the
 * records must not exceed PS_STATIC_SCRATCH_BYTES, and their work tables must
 * fit the plan's pinned staging (4 MiB; about 30,000 record-combination
 * segments); otherwise PS_E_WORKSPACE and nothing is enqueued.
 * PS_E_INVALID_ARG when no plan was ever created on the current device.  All
 * calls on one GPU share its array, which keeps the last call's contents
 * (nothing in it needs to start at zero): calls that overlap on one GPU
 * (two streams, or two host threads) race and must be serialised by the
 * caller. */
#define PS_STATIC_SCRATCH_BYTES (256u * 1024u * 1024u)
ps_status ps_execute_static(ps_plan_t plan, const ps_record* recs, int32_t n_rec, const ps_output* outs,
                            ps_stream_t stream);

/* Sequential spectra (the short-time estimates of Section 8, kept instead of
 * averaged): the spectra of chunks [chunk_lo, chunk_lo + n_chunks) of one
 * record, each chunk on its own.  `out` holds, for each requested order, an
 * array of n_chunks consecutive blocks in the layout of ps_output (chunk
 * chunk_lo + i in block i, e.g. S3 as [n_chunks][n_combos3][N_f][N_f] complex);
 * error bars are NaN (one chunk has no spread).  All chunks run in the same
 * launches as ps_execute's records (each chunk is one record of m N samples;
 * interlaced windows leave a one-chunk record as it is).
 * Errors: PS_E_INVALID_ARG if the range is not inside [0, Np) of the record or
 * n_chunks > 2^31 - 1; otherwise as ps_workspace_size / ps_execute.  n_chunks
 * == 0 enqueues nothing. */
ps_status ps_sequential_workspace_size(ps_plan_t plan, const ps_record* rec, int64_t chunk_lo,
                                       int64_t n_chunks, size_t* bytes);
ps_status ps_execute_sequential(ps_plan_t plan, const ps_record* rec, int64_t chunk_lo, int64_t n_chunks,
                                void* d_ws, size_t ws_bytes, const ps_output* out, ps_stream_t stream);

/* Full frequency plane (Section 9): the spectrum of one channel combination
 * on the signed grid k, l in (-N_f, N_f), gathered from a record's
 * positive-quadrant outputs.  For real signals a_{-k} = a_k*, so each signed
 * point is a positive-quadrant value of a related combination, possibly
 * conjugated or transposed (S2_ab(-k) = S2_ab(k)*; S3_abc takes values of
 * S3_abc, S3_acb and S3_bca; S4_abcd(-k, l) = S4_bacd(k, l),
 * S4_abcd(k, -l) = S4_abdc(k, l), S4_abcd(-k, -l) = S4_badc(k, l)); the plan
 * must hold those combinations' orbits (it does with the default "every
 * orbit").  order: 2, 3 or 4.  combo: host, `order` channel indices.  in: the
 * record's ps_output as filled by ps_execute (device arrays).  d_out, d_err
 * (device, either may be NULL): S2 [2 N_f - 1], S3 / S4 [2 N_f - 1][2 N_f - 1]
 * complex FP64 (and sigma pairs) at index k + N_f - 1 (, l + N_f - 1).
 * Enqueued on `stream`, after the execute that wrote `in` when on the same
 * stream.  Errors: PS_E_INVALID_ARG for a bad order, channel or pointer, or an
 * order the plan did not compute; PS_E_UNSUPPORTED when a needed combination
 * is not among the plan's. */
ps_status ps_full_plane(ps_plan_t plan, int32_t order, const int8_t* combo, const ps_output* in, double* d_out,
                        double* d_err, ps_stream_t stream);

/* Graph form of ps_execute for repeated runs over the same buffers: the whole
 * launch sequence (one launch per stage over every record and combination) is
 * captured once into a HIP graph, with its work tables built and copied
 * synchronously into device memory owned by the graph; ps_graph_launch then
 * replays it with a single hipGraphLaunch on any stream.  The records' device
 * data (whose contents may change between launches), the workspace and the
 * outputs given here must stay allocated while the graph exists, and the
 * workspace must not be used by other calls while a launch is in flight.
 * Contains no memset nodes (clears are kernels).  ps_graph_create synchronises
 * with the device; errors as for ps_execute. */
typedef struct ps_graph_s* ps_graph_t;
ps_status ps_graph_create(ps_plan_t plan, const ps_record* recs, int32_t n_rec, void* d_ws, size_t ws_bytes,
                          const ps_output* outs, ps_graph_t* out);
ps_status ps_graph_launch(ps_graph_t graph, ps_stream_t stream);
ps_status ps_graph_destroy(ps_graph_t graph);

/* Streaming form (quasi-polyspectra of non-stationary signals, Section 8):
 * time-resolved spectra of consecutive windows of a host-resident stream.
 * ps_streamer_create allocates, once, `depth` device staging slots of
 * window_samples samples per channel, one workspace and a copy stream
 * (default priority).  ps_streamer_push takes one window from pinned host
 * memory (channels contiguous, channel c at c * window_samples): it enqueues
 * the host-to-device copy into the next slot on the copy stream once that
 * slot's previous computation is done, makes `compute` wait for the copy,
 * enqueues the estimator for the window on `compute` writing to `outs` (as in
 * ps_execute), and returns the slot index.  The copy of the next window thus
 * overlaps the computation of the current one.  The host buffer must stay
 * untouched until the window's copy has completed, and `outs` must not be read
 * before its computation has (ps_streamer_wait on the slot, or synchronising
 * `compute`).  Windows must be pushed from one host thread, all on the same
 * `compute` stream. */
typedef struct ps_streamer_s* ps_streamer_t;
ps_status ps_streamer_create(ps_plan_t plan, int64_t window_samples, int32_t dtype, int32_t depth,
                             ps_streamer_t* out);
ps_status ps_streamer_push(ps_streamer_t s, const void* h_pinned, const ps_output* outs, ps_stream_t compute,
                           int32_t* slot);
ps_status ps_streamer_wait(ps_streamer_t s, int32_t slot);
ps_status ps_streamer_destroy(ps_streamer_t s);

/* Several windows per push.  ps_streamer_create_multi is ps_streamer_create
 * with staging slots of up to max_windows (1..64) consecutive windows.
 * ps_streamer_push_multi takes n_windows (1..max_windows) consecutive windows
 * from one pinned host buffer (window w, channel c starting at sample
 * (w * n_channels + c) * window_samples) and runs them as ONE ps_execute with
 * one record per window, outs[w] receiving window w; copy/compute overlap,
 * ownership and the rules above are as for ps_streamer_push, per slot.  The
 * group shares every launch and its tail, which keeps the GPU busy when one
 * window is a small problem.  ps_streamer_push is ps_streamer_push_multi with
 * one window.  Errors: PS_E_INVALID_ARG for n_windows outside 1..max_windows or
 * NULL arguments; otherwise as for ps_execute. */
ps_status ps_streamer_create_multi(ps_plan_t plan, int64_t window_samples, int32_t max_windows, int32_t dtype,
                                   int32_t depth, ps_streamer_t* out);
ps_status ps_streamer_push_multi(ps_streamer_t s, const void* h_pinned, int32_t n_windows, const ps_output* outs,
                                 ps_stream_t compute, int32_t* slot);

/* Running accumulation over one long record delivered in pieces, with
 * checkpoint and resume.  Section 4.2 estimates a spectrum and its error bar
 * from the parts (chunks) only through the sums over chunks of each chunk's
 * estimate x and of (Re x)^2 and (Im x)^2, and their count Np; these sums are
 * the whole state of the estimate, so an accumulation can be stopped, saved
 * and continued exactly.  The record's samples arrive as consecutive pushes of
 * any length; frames and chunks are cut from the concatenated sample sequence
 * exactly as ps_execute cuts one record (samples that do not complete a chunk
 * wait in a carry buffer for the next push).
 *
 *   ps_stream_begin(plan, max_push_samples, dtype, out)
 *       allocates (device) the FP64 state, the carry buffer of m N samples per
 *       channel, the work tables and a workspace for pushes of up to
 *       max_push_samples samples per channel; the state starts empty.  Needs a
 *       plan with the batched schedule and without interlaced windows
 *       (PS_E_UNSUPPORTED otherwise).  Freed by ps_stream_destroy.
 *   ps_stream_push(s, d_data, n_samples, channel_stride, stream)
 *       appends n_samples samples per channel (0 <= n_samples <=
 *       max_push_samples; element type `dtype`; channel c at d_data + c *
 *       channel_stride elements) and enqueues on `stream` the estimator for
 *       every chunk the sequence now completes, adding its sums to the state.
 *       d_data must stay valid until the stream has run the push.
 *       PS_E_UNSUPPORTED (nothing enqueued) once the state would hold more
 *       than 2^31 - 1 chunks.
 *   ps_stream_end(s, out, stream)
 *       enqueues the finalize of the state (mean and error bars as ps_execute
 *       gives them, NaN without a complete chunk) into `out`; the state is
 *       kept, so pushes may continue afterwards.
 *   ps_stream_counts(s, n_chunks, n_samples, n_carry)
 *       host counters: chunks accumulated, samples pushed, samples waiting.
 *   ps_stream_export_state(s, h_buf, n_bytes)
 *       waits for the pushes enqueued so far, then writes the state (a header
 *       naming the plan's configuration and the dtype, the counters, the FP64
 *       sums and the carried samples) to host memory.  With h_buf == NULL only
 *       *n_bytes is set (the size); otherwise *n_bytes is the capacity on input
 *       (PS_E_INVALID_ARG if too small) and the size written on output.
 *   ps_stream_import_state(s, h_buf, n_bytes)
 *       replaces the state of `s` by an exported one (synchronous).
 *       PS_E_INVALID_ARG unless it was exported by a stream of the same
 *       configuration (frame length, N_f, m, channels, orders, combinations,
 *       window, dt, precision, estimator, signal type) and dtype.
 * Resuming from an exported state and pushing the remaining samples gives the
 * same outputs, bit for bit, as one uninterrupted stream.  Pushes to one
 * stream must be enqueued from one host thread on the same `stream`. */
typedef struct ps_accum_s* ps_accum_t;
ps_status ps_stream_begin(ps_plan_t plan, int64_t max_push_samples, int32_t dtype, ps_accum_t* out);
ps_status ps_stream_push(ps_accum_t s, const void* d_data, int64_t n_samples, int64_t channel_stride,
                         ps_stream_t stream);
ps_status ps_stream_end(ps_accum_t s, const ps_output* out, ps_stream_t stream);
ps_status ps_stream_counts(ps_accum_t s, int64_t* n_chunks, int64_t* n_samples, int64_t* n_carry);
ps_status ps_stream_export_state(ps_accum_t s, void* h_buf, size_t* n_bytes);
ps_status ps_stream_import_state(ps_accum_t s, const void* h_buf, size_t n_bytes);
ps_status ps_stream_destroy(ps_accum_t s);

/* Per-point comparison of two estimates of the same spectrum, e.g. quasi-
 * spectra computed with different m (Section 8: a spectrum that changes with m
 * beyond its error bars points to non-stationarity): d_out[i] =
 * |a_i - b_i| / sqrt(sa_i^2 + sb_i^2), for the real and the imaginary parts of
 * n_points complex values (arrays [n_points][2] in the layouts of ps_output:
 * spectra and their error-bar pairs).  0/0 gives NaN.  Enqueued on `stream`.
 * A descriptive statistic, not a test with a known distribution when both
 * estimates come from the same data. */
ps_status ps_spectra_zscore(const double* d_a, const double* d_a_err, const double* d_b, const double* d_b_err,
                            int64_t n_points, double* d_out, ps_stream_t stream);

/* The first stage alone (Section 3, eq. a_k without the dt factor): for every
 * frame f < Np*m of every channel, d_coef[c][f][k] = sum_i g_i z_{fN+i}
 * exp(+2 pi j i k/N), k < n_coef, as interleaved FP32 complex.  d_coef must hold
 * n_channels * Np * m * n_coef float pairs. */
ps_status ps_coefficients(ps_plan_t plan, const ps_record* rec, float* d_coef, ps_stream_t stream);

/* Per-stage timing with HIP events recorded on the execution stream.  While
 * enabled, ps_execute records an event pair around every stage launch;
 * ps_profile_read waits for those events and returns, per stage, the summed
 * milliseconds since the previous read: [0] windowed FFT (stage a1), [1] chunk
 * means, [2] S2, [3] S3, [4] S4, [5] finalize; stage_ms[6..] (if n > 6) receive
 * the number of launches of stage 0..5.  Timing adds event records between
 * launches; leave it off outside measurements. */
ps_status ps_profile_enable(ps_plan_t plan, int32_t on);
ps_status ps_profile_read(ps_plan_t plan, double* stage_ms, int32_t n);

/* Launch configuration of the moment stages.  These change how fast
 * ps_execute runs, not
 * what it computes: the spectra agree to the order of FP64 additions (the
 * tiles split across blocks, whose partial sums are added separately, depend
 * on the tile order).
 *   tile_group      the output tiles of a spectrum are walked in
 *                   tile_group x tile_group blocks of tiles (1 = row by row);
 *                   1, 2, 4, 8 (default) or 16.  Larger blocks keep the
 *                   coefficient columns that concurrent blocks read in L2.
 *   s3_frame_batch  frames staged per LDS batch by the S3 kernel: 10, 11 or
 *                   16, or 0 (default) to choose by the rows per chunk
 *                   (m, or m + 1 with PS_EST_C3OPT): exactly their number
 *                   for 11 to 13 rows (one batch), else 10.
 * ps_plan_set_tuning rewrites the plan's tile tables in device memory
 * (synchronously): no execute or graph launch of the plan may be in flight.
 * Graphs captured earlier use the new tile order from their next launch and
 * keep the S3 frame batch they were captured with (the frame batch does not
 * change the S3 sums: frames are added in the same order either way).
 * Errors: PS_E_INVALID_ARG for NULL or values outside the lists above. */
typedef struct ps_tuning {
    int32_t tile_group;
    int32_t s3_frame_batch;
} ps_tuning;
ps_status ps_plan_get_tuning(ps_plan_t plan, ps_tuning* t);
ps_status ps_plan_set_tuning(ps_plan_t plan, const ps_tuning* t);

/* Autotuner: times every candidate configuration (tile_group 1, 4, 8, 16;
 * with S3 requested and m > 10 also the S3 frame batch: the default rule (0),
 * 10 and 16) with one warm-up
 * and `reps` (1..100) timed ps_execute calls on the caller's records,
 * workspace and outputs (arguments as for ps_execute; the outputs end up
 * holding the last run's spectra), measured with HIP events on `stream`, and
 * keeps the fastest in the plan.  Synchronises the stream; the same rule as
 * for ps_plan_set_tuning applies.  `report` (may be NULL) receives the
 * candidates, the mean milliseconds per execute of each and the index of the
 * one kept.  Errors: PS_E_INVALID_ARG for NULL or empty arguments or reps out
 * of range; otherwise as for ps_execute, with the plan's configuration left as
 * it was before the call. */
#define PS_TUNE_MAX 16
typedef struct ps_tune_report {
    int32_t n;
    int32_t best;
    ps_tuning cand[PS_TUNE_MAX];
    double ms[PS_TUNE_MAX];
} ps_tune_report;
ps_status ps_plan_autotune(ps_plan_t plan, const ps_record* recs, int32_t n_rec, void* d_ws, size_t ws_bytes,
                           const ps_output* outs, int32_t reps, ps_stream_t stream, ps_tune_report* report);

/* Host only: the "every orbit" combination list of `order` (2, 3 or 4) for
 * n_channels (1..4) channels, in the order ps_plan_create uses.  With out ==
 * NULL only the count is returned in *n; otherwise *n is the capacity of `out`
 * in combinations on input and the count on output. */
ps_status ps_enumerate_combos(int32_t n_channels, int32_t order, int8_t* out, int32_t* n);

const char* ps_status_string(ps_status s);
const char* ps_last_error(void);
int32_t ps_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* POLYSPEC_H */
