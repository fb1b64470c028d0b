/*
 * xeng.h - C ABI of the MI355X X-engine.
 *
 * The X-engine of an FX correlator (paper Sec. 2 and Sec. 2.2): the voltages
 * of every input have already been channelised by the F stage and transposed
 * so that the samples of one frequency from all inputs sit together (the
 * "corner turn", Sec. 2.1).  For every frequency channel f the engine forms
 * the complex multiply-accumulate of every pair of inputs, auto-correlations
 * included, and integrates it over a chosen duration:
 *
 *     V[f][k(i,j)] = sum_t x_i(t,f) * conj(x_j(t,f)),   0 <= j <= i < N,
 *     k(i,j) = i(i+1)/2 + j     ("fix one input, run over all inputs up to and
 *                                 including itself", Sec. 2.3)
 *
 * Input samples (Sec. 2.1 equaliser, Sec. 2.3 packet payload): one byte per
 * complex sample, real part = 4-bit two's complement in bits 7..4, imaginary
 * part = 4-bit two's complement in bits 3..0 (code 1000b decodes as -8).
 * Voltage blocks are uint8 [T][F][N] (time, channel, input), input fastest.
 *
 * Output: int32 [F][N(N+1)/2][2], (re, im) interleaved, channel-major, in the
 * k(i,j) order above; V_ji = conj(V_ij) gives the upper triangle.  Values are
 * the exact integer sums (no averaging; divide by n_integrated for a mean).
 *
 * All entry points return an xeng status (0 = OK, < 0 = error) unless stated;
 * no entry point throws or aborts.  Device pointers are HIP device memory of
 * the device current when the plan was made.  Every call on one plan must come
 * from one host thread at a time.  With the environment variable XENG_TRACE
 * set (not "0") when a plan is made, the plan logs every kernel launch to
 * stderr.
 */
#ifndef XENG_H
#define XENG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xeng_plan_s xeng_plan_t;

/* One independent array: N inputs, F channels, and the largest number of
 * time samples one xeng_correlate call may pass for it. */
typedef struct {
    int32_t n_inputs;           /* N, 1 .. XENG_MAX_INPUTS              */
    int32_t n_chans;            /* F, >= 1, F * N <= 2^31 - 1           */
    int64_t max_time_per_call;  /* >= 1, <= XENG_MAX_INTEGRATION        */
} xeng_array_desc;

enum {
    XENG_OK        =  0,
    XENG_EINVAL    = -1,  /* bad argument: size, null or misaligned pointer  */
    XENG_ENOMEM    = -2,  /* device or host allocation failed                 */
    XENG_EOVERFLOW = -3,  /* integration would exceed XENG_MAX_INTEGRATION    */
    XENG_EDEVICE   = -4,  /* HIP runtime error; text in xeng_last_error       */
    XENG_ESTATE    = -5   /* plan unusable after an earlier device error      */
};

enum {
    XENG_DUMP_KEEP    = 1u << 0,  /* copy out but keep integrating             */
    XENG_DUMP_TO_HOST = 1u << 1   /* dst are host pointers; call is synchronous */
};

enum {
    XENG_PLAN_BATCH   = 1u << 0   /* batched plan even with 0 or 1 arrays      */
};

/* Largest number of inputs per array the kernels are built for (the paper's
 * largest design, eight boards of 32 inputs, Sec. 2.3). */
#define XENG_MAX_INPUTS 256
/* Largest integration (samples since the last dump) whose sums are
 * guaranteed to fit int32: one sample adds at most 128 in magnitude
 * (all codes -8), and (2^31 - 1) / 128 = 16,777,215. */
#define XENG_MAX_INTEGRATION 16777215LL

/*
 * xeng_plan - create an engine for n_arrays independent arrays.
 *   out        receives the plan (owned by the library; free with xeng_destroy).
 *   arrays     n_arrays descriptors (read during the call only).
 *   n_arrays   >= 1, or 0 with XENG_PLAN_BATCH (arrays attached later).
 *              With one array (and no flag) this is the plain per-dump
 *              engine: one kernel launch per xeng_correlate.  Otherwise the
 *              plan is batched: every xeng_correlate runs the work of all its
 *              arrays as one persistent launch over a work list of (array,
 *              channel group, time chunk) items, recorded into a hipGraph
 *              (Sec. 2: each X node takes a band of channels; Sec. 2.2: one
 *              GPU core per band - here many bands of many arrays share one
 *              GPU).  Results are bit-identical to the plain engine's.
 *   flags      0 or XENG_PLAN_BATCH.
 *   hip_stream hipStream_t to run on, or NULL for a stream the plan owns.
 * The array indices of later calls are slots 0 .. n_arrays-1 (see
 * xeng_attach for more).  Allocates the HBM-resident int32 accumulators
 * (zeroed).  Errors: EINVAL (null out, null arrays with n_arrays > 0, N or F
 * or max_time_per_call out of range, unknown flags), ENOMEM, EDEVICE.
 */
int xeng_plan(xeng_plan_t **out, const xeng_array_desc *arrays, int32_t n_arrays,
              uint32_t flags, void *hip_stream);

/*
 * xeng_correlate - integrate one block of voltages per array (Sec. 2.2 CMAC,
 * Sec. 1/2 integration).  Asynchronous on the plan's stream.
 *   d_voltages  one device pointer per slot (xeng_slots), each uint8
 *               [n_time[a]][F][N], 16-byte aligned; caller-owned, must stay
 *               valid until the stream reaches this work.  May be NULL where
 *               n_time[a] == 0.
 *   n_time      one sample count per slot; 0 skips that array (and must be 0
 *               for a free slot).
 * The block is added to the array's running integration.  A batched plan
 * launches one captured graph per call; the graph keeps the pointers and
 * counts of this call, so the caller may reuse its argument arrays at once.
 * Errors: EINVAL (null/misaligned pointer, n_time < 0 or > max_time_per_call,
 * n_time > 0 for a free slot), EOVERFLOW
 * (samples since the last dump would exceed XENG_MAX_INTEGRATION; nothing is
 * launched and the state is unchanged), EDEVICE, ESTATE.
 */
int xeng_correlate(xeng_plan_t *p, const uint8_t *const *d_voltages, const int64_t *n_time);

/*
 * xeng_dump - hand out the integrated visibilities (Sec. 2.2: the CPU and
 * disk threads take the GPU's output) and start a new integration.
 *   array         slot of the array, or -1 for all slots.
 *   dst           one pointer per dumped slot (1, or xeng_slots for -1; free
 *                 slots are skipped and their pointer ignored), each int32
 *                 [F][N(N+1)/2][2]; device memory, or host memory with
 *                 XENG_DUMP_TO_HOST.  Caller-owned.  8-byte aligned device
 *                 destinations are written by one copy kernel for all dumped
 *                 arrays; others by a copy each.
 *   flags         XENG_DUMP_KEEP: do not reset; XENG_DUMP_TO_HOST: see above.
 *   n_integrated  optional out, one per dumped array: samples in the dump.
 * Without KEEP the integration restarts from zero and the sample count is
 * reset (the accumulator memory is overwritten by the next launch, or
 * cleared first when that launch adds atomically).
 * Stream-ordered after all earlier correlate calls; with TO_HOST it waits for
 * the copy before returning.  Errors: EINVAL, EDEVICE, ESTATE.
 */
int xeng_dump(xeng_plan_t *p, int32_t array, int32_t *const *dst, uint32_t flags,
              int64_t *n_integrated);

/*
 * xeng_correlate_dump - integrate one block per array and dump it in the same
 * call (the usual pattern of a correlator: one dump per integration, Sec. 2.2).
 * Same result as xeng_correlate followed by xeng_dump of the arrays given a
 * destination, but the kernels write the visibilities straight into the
 * destination: an empty integration never touches the accumulator, and one
 * with earlier samples has them copied over first.
 *   d_voltages, n_time  as for xeng_correlate.
 *   d_dst         one pointer per slot: NULL leaves that array integrating
 *                 (as xeng_correlate); otherwise int32 [F][N(N+1)/2][2] device
 *                 memory (checked), 8-byte aligned, caller-owned, receives the
 *                 visibilities including this call's samples, and the
 *                 array's integration restarts.  A slot with n_time 0 and a
 *                 destination is dumped as by xeng_dump.
 *   n_integrated  optional out, one per slot: samples in each dump (written
 *                 for the dumped slots only).
 * Asynchronous on the plan's stream.  Errors: as xeng_correlate, and EINVAL
 * for a destination that is misaligned or not device memory.
 */
int xeng_correlate_dump(xeng_plan_t *p, const uint8_t *const *d_voltages, const int64_t *n_time,
                        int32_t *const *d_dst, int64_t *n_integrated);

/*
 * xeng_attach - add an array to a batched plan between calls (admission of a
 * new sub-array into a running serving loop).
 *   d      its descriptor (read during the call only).
 *   index  receives its slot: the first free slot, else a new one at the end.
 * Allocates and zeroes its accumulator of xeng_accumulator_bytes(N, F) bytes
 * (hipMalloc).  Errors: EINVAL (plain plan, bad descriptor, null pointer),
 * ENOMEM (the accumulator does not fit; the plan is unchanged), EDEVICE, ESTATE.
 */
int xeng_attach(xeng_plan_t *p, const xeng_array_desc *d, int32_t *index);

/*
 * xeng_detach - remove an array from a plan and free its accumulator.  Waits
 * for the plan's stream first (dump the array before detaching it).  The
 * slot is free afterwards: n_time must be 0 for it and dumps skip it.
 * Errors: EINVAL (slot out of range or free), EDEVICE, ESTATE.
 */
int xeng_detach(xeng_plan_t *p, int32_t index);

/* Counters of a plan since it was made (xeng_stats). */
typedef struct {
    int64_t calls;      /* xeng_correlate calls that did work                     */
    int64_t launches;   /* kernel launches (plain, or persistent batch launches)   */
    int64_t samples;    /* time samples integrated, summed over arrays             */
    int64_t cmacs;      /* useful complex MACs: samples x F x N(N+1)/2, summed     */
    int64_t bytes_in;   /* voltage bytes consumed                                  */
    int64_t dumps;      /* arrays dumped                                           */
    int64_t bytes_out;  /* visibility bytes dumped                                 */
} xeng_stats_t;

/* Copy the plan's counters to out.  Errors: EINVAL (null pointers). */
int xeng_stats(const xeng_plan_t *p, xeng_stats_t *out);

/*
 * xeng_load_acc - seed an array's integration from saved visibilities (resume
 * from a checkpoint: the accumulator is the engine's whole state, and a KEEP
 * dump is a snapshot of it).  src is int32 [F][N(N+1)/2][2], device or host
 * memory (caller-owned, read on the plan's stream); n_integrated is the
 * sample count it holds (0 .. XENG_MAX_INTEGRATION).  Later calls add to it.
 * Errors: EINVAL, EDEVICE, ESTATE.
 */
int xeng_load_acc(xeng_plan_t *p, int32_t array, const int32_t *src, int64_t n_integrated);

/* Number of slots of the plan (attached or free); -1 for NULL. */
int32_t xeng_slots(const xeng_plan_t *p);

/* Bytes of one array's accumulator, F * N(N+1)/2 * 2 * 4; -1 on bad sizes. */
int64_t xeng_accumulator_bytes(int32_t n_inputs, int32_t n_chans);

/*
 * xeng_autotune - pick launch shapes by timing them on the caller's data.
 *   d_voltages, n_time  one call's arguments, as for xeng_correlate.
 *   reps                calls timed per candidate (>= 1).
 *   best_ms             optional out: mean time of one call with the choice.
 * Batched plan: the work-item granularity of the persistent launch (about
 * 1, 2, 4 or 8 items per compute unit; items are cut along time), then per
 * array, largest first, whether it runs as items of the persistent launch
 * (16-row tiles) or as a plain launch of its own inside the same graph, with
 * the tile shape and time split that suit it.  Plain plan, per array: the
 * tile shape (16-row tiles of the 16x16x64 ring kernel, 32-row tiles of the
 * 32x32x32 ring kernel, both for N a multiple of 16, or 16-row tiles of the
 * staging kernel) and the number of workgroups per compute unit that the
 * time split aims for.  The choice is kept by the plan for later calls and
 * entered in the process's tuning cache (xeng_tune_cache_save), which new
 * plans of the same GPU architecture, kind, N and power-of-two buckets of F
 * and of max_time_per_call start from.  Every accumulator must be freshly
 * dumped (or never used); the trial sums are discarded and the accumulators
 * are zero on return.  Synchronous.  Errors: EINVAL, EDEVICE, ESTATE.
 */
int xeng_autotune(xeng_plan_t *p, const uint8_t *const *d_voltages, const int64_t *n_time,
                  int32_t reps, float *best_ms);

/*
 * xeng_tune_cache_save / xeng_tune_cache_load / xeng_tune_cache_clear - the
 * process-wide tuning cache of xeng_autotune as a text file (one choice per
 * line: architecture, batched, N, log2 F bucket, log2 T bucket, tile shape,
 * time split, own launch; a batched plan's items per workgroup are kept as a
 * line with N = 0, F bucket 0 and the log2 bucket of its array count in
 * place of the T bucket), so a later process skips the timing.  Loading
 * adds to (and overrides) what the cache holds; plans made afterwards use
 * it.  Errors: EINVAL (null path, file not readable or writable; for load
 * also malformed lines, which are skipped).
 */
int xeng_tune_cache_save(const char *path);
int xeng_tune_cache_load(const char *path);
int xeng_tune_cache_clear(void);

/*
 * xeng_requantize - equaliser / 4-bit requantiser of the F stage (Sec. 2.1),
 * the step that produces the X-engine's input.  Stateless, asynchronous on
 * hip_stream (NULL: the default stream).
 *   d_words   uint64 [n_time][n_chans][n_inputs], device, 8-byte aligned: PFB
 *             output words, 18-bit two's-complement real part (fix_18_17) in
 *             bits 35..18, imaginary part in bits 17..0; higher bits ignored.
 *   d_gains   uint32 [n_chans][n_inputs], device, 4-byte aligned: scale
 *             factors, unsigned fix_18_7 in the low 18 bits (higher ignored).
 *   d_out     uint8 [n_time][n_chans][n_inputs], device: packed 4+4-bit
 *             samples, the X-engine's input (real part in bits 7..4).
 * Each part times its gain (a fix_36_24 product) is rounded half to even at
 * the fix_4_3 LSB and saturated to -7 .. 7 (1.001b .. 0.111b).  Exact.
 * Buffers are caller-owned.  n_time == 0 is a no-op.  Errors: EINVAL (null or
 * misaligned pointer, n_chans or n_inputs < 1, n_time < 0, grid too large),
 * EDEVICE (launch failure).
 */
int xeng_requantize(const uint64_t *d_words, const uint32_t *d_gains, uint8_t *d_out,
                    int64_t n_time, int32_t n_chans, int32_t n_inputs, void *hip_stream);

/*
 * xeng_eq_update - equaliser gains from the X-engine's autocorrelations
 * (Sec. 2.1, Eq. 3: RMS = sqrt(P / 2N), P the integrated auto power over N
 * samples), so that the 4-bit RMS comes to target_rms_x16 / 16 (the paper
 * aims at 2..3).  Stateless, asynchronous on hip_stream.
 *   d_vis          int32 [n_chans][N(N+1)/2][2], device: a dump of the
 *                  requantised data (only the autos Re V_ii are read).
 *   n_integrated   N, the dump's sample count (1 .. XENG_MAX_INTEGRATION).
 *   d_gains_in     uint32 [n_chans][n_inputs], device: the gains used (fix_18_7).
 *   d_gains_out    uint32 [n_chans][n_inputs], device (may equal d_gains_in).
 *   target_rms_x16 1 .. 255.
 * G' = G * t * sqrt(2 N / P), t = target / 16, rounded to the nearest integer
 * (halves up) exactly, clamped to [1, 2^18 - 1]; inputs with P = 0 keep
 * their word.  Errors: EINVAL, EDEVICE.
 */
int xeng_eq_update(const int32_t *d_vis, int64_t n_integrated, const uint32_t *d_gains_in,
                   uint32_t *d_gains_out, int32_t n_chans, int32_t n_inputs, int32_t target_rms_x16,
                   void *hip_stream);

/*
 * xeng_ingest - packet ingest and corner turn on the X side (Sec. 2.3,
 * Sec. 2.1): assemble one integration block from the F engine's packets.
 * Stateless, asynchronous on hip_stream.
 *   d_packets      n_packets packets, device, 8-byte aligned, packet_stride
 *                  bytes apart (a multiple of 8, >= 8 + 8 * n_chans * 32).
 *                  Each: 6-byte big-endian counter MCNT, 1 byte Fid (board),
 *                  1 byte Xid (band), then uint8 [8][n_chans][32] samples
 *                  of the board's 32 inputs ([time, channel, input]).
 *   mcnt0          counter of the first time block (0 .. 2^48 - 1).
 *   n_blocks       time blocks of 8 samples in the output (1 .. 65535).
 *   n_boards       boards (inputs 32 Fid .. 32 Fid + 31), 32 n_boards <=
 *                  XENG_MAX_INPUTS.
 *   n_chans        channels per packet (32 for a 1024-point spectrum on 32
 *                  bands, 16 for 512).
 *   xid            this node's band: packets of other bands are ignored.
 *   d_index        int32 [n_blocks][n_boards], device, out: the packet
 *                  number that filled each (time block, board) tile, or -1
 *                  where none arrived (loss; its samples are zero).
 *   d_out          uint8 [8 n_blocks][n_chans][32 n_boards], device, 8-byte
 *                  aligned, out: the X-engine's input block.
 * Packets outside [mcnt0, mcnt0 + n_blocks), of a board >= n_boards or of
 * another band are ignored; of two packets for one tile the later in the
 * buffer wins.  Errors: EINVAL (sizes, alignment, null pointers), EDEVICE.
 */
int xeng_ingest(const uint8_t *d_packets, int64_t n_packets, int32_t packet_stride, int64_t mcnt0,
                int32_t n_blocks, int32_t n_boards, int32_t n_chans, int32_t xid, int32_t *d_index,
                uint8_t *d_out, void *hip_stream);

/*
 * xeng_channelise - F-stage channeliser (Sec. 2.1, Eq. 1-2): 4-tap polyphase
 * filter bank (Hamming-windowed sinc prototype) and one complex FFT of
 * L = 2 n_chans points per pair of real inputs (2q, 2q + 1), split by Eq. 2.
 * Float32.  Stateless, asynchronous on hip_stream; allocates nothing.
 *   d_adc       int8 [n_inputs][n_samples], device, 8-byte aligned: real
 *               ADC samples, one stream per input (n_samples % 8 == 0).
 *   n_inputs    even, >= 2.
 *   n_chans     F, a power of two from 8 to 1024.
 *   d_out       float [S][F][n_inputs][2], device, 16-byte aligned: complex
 *               spectra in the X side's [time, channel, input] order;
 *               spectrum s uses samples [2Fs, 2F(s + 4)); S from
 *               xeng_channelise_spectra; channel k < F (Nyquist dropped).
 *               May be NULL when there are no spectra.
 *   d_tables    float [xeng_channelise_table_floats(F)], device, 16-byte
 *               aligned: scratch for the filter and twiddle tables, written
 *               by the call (caller-owned; one per concurrent call).
 * Errors: EINVAL (sizes, alignment, null pointers), EDEVICE.
 */
int xeng_channelise(const int8_t *d_adc, int64_t n_samples, int32_t n_inputs, int32_t n_chans,
                    float *d_out, float *d_tables, void *hip_stream);

/*
 * xeng_channelise_noalloc - xeng_channelise for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same computation and arguments without
 * d_tables.  The filter and twiddle tables go to a scratch array inside the
 * library, one per GPU, of 4 * 2048 + 2048 floats (40 KB, enough for the
 * largest spectrum, F = 1024), held until the process ends; the call itself
 * allocates nothing.  Every call on a GPU rewrites that GPU's array before
 * reading it, so calls that overlap on one GPU (on different streams) race
 * and must not be issued.  Errors: as xeng_channelise (EINVAL also for F
 * beyond the scratch size), EDEVICE if the scratch address cannot be
 * obtained.
 */
int xeng_channelise_noalloc(const int8_t *d_adc, int64_t n_samples, int32_t n_inputs, int32_t n_chans,
                            float *d_out, void *hip_stream);

/* Spectra produced from n_samples samples: n_samples / 2F - 3 (>= 0); -1 on bad sizes. */
int64_t xeng_channelise_spectra(int64_t n_samples, int32_t n_chans);

/* Floats of the table scratch for F channels: 4 * 2F + 2F; -1 on bad sizes. */
int64_t xeng_channelise_table_floats(int32_t n_chans);

/* xeng_destroy - wait for the plan's work, free everything it owns.  NULL is a no-op. */
void xeng_destroy(xeng_plan_t *p);

/* Number of baselines N(N+1)/2 including autos; -1 if n < 0. */
int64_t xeng_nbaselines(int32_t n);

/* k(i,j) = i(i+1)/2 + j for 0 <= j <= i; -1 otherwise. */
int64_t xeng_baseline_index(int32_t i, int32_t j);

/* Static text for a status code. */
const char *xeng_strerror(int status);

/* Text of the plan's last error ("" if none); valid until the next call on p. */
const char *xeng_last_error(const xeng_plan_t *p);

/* Samples integrated since the last dump for one array; -1 on bad arguments
 * or a free slot. */
int64_t xeng_integrated(const xeng_plan_t *p, int32_t array);

#ifdef __cplusplus
}
#endif

#endif /* XENG_H */
