/*
 * vbw.h -- C ABI of the MI355X (gfx950) overlap-save variable-bandwidth filter.
 *
 * Operation (Moryakova & Johansson, arXiv 2406.14116):
 *   Sec. II, overlap-save steps 1-5: every channel is cut into N-sample
 *   segments that advance by M samples (`hop`); each segment is transformed by
 *   an N-point DFT, multiplied by the filter DFT coefficients H(k), inverse
 *   transformed (eq. (4): +j exponent, factor 1/N), the first N-M samples are
 *   dropped and the M-sample pieces are concatenated.
 *   Sec. III-B, eqs. (5)-(7): H(k) = H_R(k) exp(-j 2 pi k D / N) with
 *   D = (L-1)/2 = (N-M)/2, and H_R(k) = 1 on the passband bins
 *   [0,k1-1] u [N-k1+1,N-1], V(k-k1) on the transition bins [k1,k2], V(N-k-k1)
 *   on the mirrored transition bins [N-k2,N-k1], and 0 on the stopband bins,
 *   with k2 = k1 + L_V - 1.  The L_V values V(r) are shared by every bandwidth,
 *   so a bandwidth change is an integer k1 and costs no arithmetic
 *   (Sec. III-D, last paragraph).
 *
 * Framing: segment m covers input samples [m*M - (N-M), m*M + M); samples
 * outside [0, len) read as zero (N-M zeros of history before the stream).
 * Output sample m*M + j (j < M) is sample N-M+j of block m's inverse
 * transform; output length equals input length.  Block count per channel is
 * ceil(len / M).
 *
 * Data layout: each channel's input and output is one contiguous device
 * array of `len` complex samples, interleaved (re, im):
 *   VBW_C64   -- two float32 per sample (8 bytes)
 *   VBW_CF16  -- two IEEE binary16 per sample (4 bytes)
 *   VBW_CBF16 -- two bfloat16 per sample (4 bytes)
 *   VBW_R32   -- real input: one float32 per sample (4 bytes), real output.
 *               The impulse response is real (eq. (8)), so the library
 *               filters two consecutive real blocks as the real and imaginary
 *               parts of one complex block.
 * The FFT engine computes in float32.  The matrix-core engine
 * (VBW_ENGINE_GEMM) feeds its products FP16 hi/lo operand pairs and
 * accumulates in float32, after an exact power-of-two scale per block; its
 * error relative to each block's largest value is about the float32
 * engine's, for any finite FP16 or BF16 input (FP16 subnormals to 65504,
 * BF16 over its whole range).  16-bit values are converted on load and
 * rounded to nearest-even on store.  With VBW_F32_OUT the output is written
 * as float32 pairs whatever the input storage.
 *
 * Errors: every entry point returns a vbw_status; negative values are errors.
 * No exception crosses the ABI and nothing aborts.  A call that fails leaves
 * the plan as it was.  Device failures map to VBW_EDEVICE, allocation
 * failures to VBW_ENOMEM.
 *
 * Threading: one plan is used by one host thread at a time; distinct plans are
 * independent.  The device work of the calls on one plan runs in call order:
 * a vbw_filter or vbw_stream_reset on another stream than the plan's previous
 * call first makes that stream wait (on the device, no host synchronisation)
 * for the previous call's work, since it may rewrite the per-call tables and
 * the stream state that work reads.
 */
#ifndef VBW_H
#define VBW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum vbw_status {
    VBW_OK = 0,
    VBW_EINVAL = -1,        /* malformed argument (see each call) */
    VBW_ERANGE = -2,        /* k1 / L_V outside the admissible bin range */
    VBW_ENOMEM = -3,        /* host or device allocation failed */
    VBW_EDEVICE = -4,       /* HIP runtime or kernel launch error */
    VBW_EUNSUPPORTED = -5,  /* valid request this build does not serve */
    VBW_ETOOLARGE = -6      /* vbw_filter_noalloc: tables exceed its static scratch */
} vbw_status;

typedef enum vbw_dtype {
    VBW_C64 = 0,
    VBW_CF16 = 1,
    VBW_CBF16 = 2,
    VBW_R32 = 3       /* real float32 samples in and out (FFT engine) */
} vbw_dtype;

typedef enum vbw_engine {
    VBW_ENGINE_FFT = 0,     /* LDS-staged Stockham FFT, float32 */
    VBW_ENGINE_GEMM = 1     /* N = 256 as 16 x 16 MFMA products, FP16 hi/lo split
                               operands, FP32 accumulation, exact per-block
                               power-of-two scaling (16-bit storage only) */
} vbw_engine;

/* Plan flags. */
#define VBW_NO_PRUNE   (1u << 0)  /* always run the full N-point inverse */
#define VBW_GRAPH      (1u << 1)  /* replay a captured HIP graph in steady state */
#define VBW_F32_OUT    (1u << 2)  /* write float32 output for 16-bit input */
#define VBW_HOST_ONLY  (1u << 3)  /* validate and build host tables only; no device use */
#define VBW_AUTOTUNE   (1u << 4)  /* time the launch variants on the first vbw_filter */
#define VBW_STREAM     (1u << 5)  /* successive vbw_filter calls continue one stream (FFT engine) */

/* One channel.  `reserved` must be 0. */
typedef struct vbw_channel {
    int32_t n;          /* DFT size N: a power of two, 16 <= N <= 4096 */
    int32_t hop;        /* output samples per block M: 1 <= M <= N-1, N-M even */
    int32_t lv;         /* transition samples per edge L_V >= 0 */
    int32_t v_offset;   /* index of V(0) in the plan's V pool */
    int32_t k1;         /* first transition bin in force from block 0 */
    int32_t reserved;
    int64_t len;        /* input and output length in complex samples, >= 0 */
} vbw_channel;

/* Plan description.  The library deep-copies `channels`, `v_pool` and
 * `tune_cache`; the caller may free them when vbw_plan returns.  V values are
 * rounded to float32 once, here.  `reserved` must be 0.  A zero-initialised
 * tail (tune_cache, max_workgroups) means: no tuning file, no cap. */
typedef struct vbw_plan_desc {
    int32_t n_channels;            /* >= 1 */
    int32_t n_v;                   /* entries in v_pool, >= 0 */
    const vbw_channel *channels;   /* host array of n_channels */
    const double *v_pool;          /* host array of n_v finite values */
    int32_t dtype;                 /* vbw_dtype */
    int32_t engine;                /* vbw_engine */
    uint32_t flags;                /* VBW_* flags */
    int32_t max_workgroups;        /* cap on the workgroups of each persistent
                                      launch (0: as many as are resident);
                                      e.g. to leave CUs to concurrent work */
    const char *tune_cache;        /* NULL, or a file in which VBW_AUTOTUNE
                                      keeps its choices (see vbw_filter) */
    int32_t reserved;
} vbw_plan_desc;

typedef struct vbw_plan_s *vbw_plan_t;

/* Create a plan (Sec. II framing, Sec. III-B coefficients).
 * Validates every channel, copies descriptors and V, builds the integer work
 * list and uploads the device tables (float32 twiddles generated in float64
 * and rounded to nearest).  Uses the current HIP device.
 * Errors: VBW_EINVAL for a NULL pointer, a bad N / hop / L_V / v_offset /
 * len, a non-finite V, an unknown dtype/engine/flag or nonzero reserved
 * field; VBW_ERANGE when k1 < 1 or k2 = k1 + L_V - 1 > N/2 - 1 (the one
 * exception is the all-pass L_V = 0, k1 = N/2 + 1); VBW_EUNSUPPORTED for the
 * GEMM engine with float32 storage, any channel with N != 256, or
 * VBW_STREAM; VBW_ENOMEM / VBW_EDEVICE from HIP.  With VBW_STREAM every
 * channel's len must be 0 or a multiple of M that is at least N - M (else
 * VBW_EINVAL): a call then carries whole blocks and at least the history the
 * next call needs.
 * On error *out is set to NULL. */
vbw_status vbw_plan(const vbw_plan_desc *desc, vbw_plan_t *out);

/* Change channel `channel`'s bandwidth from block `from_block` on
 * (on a VBW_STREAM plan blocks are counted from the start of the stream, not
 * of the call)
 * (Sec. III-B: only the integer edge k1 changes; V is reused, nothing is
 * recomputed).  Block m uses the entry with the largest from_block <= m; an
 * entry with an equal from_block is replaced.  O(entries) host work, no device
 * call; the change reaches the device with the next vbw_filter.
 * Errors: VBW_EINVAL (NULL plan, channel out of range, from_block < 0,
 * more than 4096 entries on one channel); VBW_ERANGE (k1 as in vbw_plan). */
vbw_status vbw_set_bandwidth(vbw_plan_t plan, int32_t channel, int32_t k1,
                             int64_t from_block);

/* Fix the plan's launch variant (0 <= variant < vbw_plan_query(plan,
 * VBW_Q_N_VARIANTS)); the autotuner then keeps it.  Variant 0 is the default
 * shape: one persistent launch per DFT size at full residency with pruning
 * as the flags allow; the others change the resident workgroups per CU, the
 * grid (twice the resident count: shorter ranges per workgroup), pruning, the
 * order of the work (chunks dealt to the workgroups in turn instead of one
 * range each), or use one launch of the kernel that dispatches on N (plans
 * that mix N).  All
 * variants compute the same result (Sec. II; only the schedule changes).
 * Errors: VBW_EINVAL (NULL plan, variant out of range); VBW_EUNSUPPORTED for
 * a VBW_HOST_ONLY plan. */
vbw_status vbw_plan_set_variant(vbw_plan_t plan, int32_t variant);

/* Filter every channel (Sec. II steps 1-5) from zero history.
 * x[c] / y[c] are device pointers to channel c's input / output
 * (layout above); the host arrays x and y hold n_channels pointers and are
 * read during the call only.  The device buffers are caller-owned and must
 * stay valid until the work on `stream` completes.  `stream` is a
 * hipStream_t (NULL: the null stream).  Asynchronous: new pointers or a
 * changed schedule are uploaded, stream-ordered, into one of two per-call
 * tables that take turns (one with VBW_GRAPH); the host waits only when the
 * table's previous upload has not left its staging buffer yet.
 * With VBW_STREAM the calls continue one stream per channel (Sec. II: the
 * input is one unbounded sequence cut into blocks): a call's block 0 reads
 * the previous call's last N - M input samples instead of zeros, the band
 * schedule counts blocks from the start of the stream, and the output of a
 * sequence of calls equals that of one call over the concatenated input.  The
 * stream state lives on the device and advances in stream order, so calls may
 * be queued (or replayed from a graph) without host synchronisation.
 * With VBW_AUTOTUNE the first call also times every launch variant on these
 * buffers (blocking; the outputs are the filter's outputs all the same),
 * each N group's launch on its own as well, and keeps the fastest variant,
 * or the combination of each N group's fastest launch, for the plan's
 * lifetime.  When the plan's tune_cache names a file, the choice is appended
 * to it as one "key choice" line (key: device, storage, engine, kernel flags,
 * workgroup cap and the block count per N, rounded to a power of two), and a
 * plan whose key is in the file takes that choice at creation without
 * timing.  With VBW_GRAPH and a non-null
 * stream the launches are captured once into a HIP graph and replayed.
 * Errors: VBW_EINVAL (NULL plan or arrays, NULL pointer for a channel with
 * len > 0, an output range overlapping any other input or output range);
 * VBW_EUNSUPPORTED for a VBW_HOST_ONLY plan; VBW_EDEVICE from HIP. */
vbw_status vbw_filter(vbw_plan_t plan, const void *const *x, void *const *y,
                      void *stream);

/* vbw_filter, with the kernels' own duration: start_event and stop_event
 * (hipEvent_t, created by the caller on the plan's device, timing enabled)
 * take the start time of the call's first filter kernel and the end time of
 * its last, as the GPU records them for the dispatch itself, so that
 * hipEventElapsedTime(start, stop) excludes the queueing and launch latency
 * that events recorded on the stream around the call include.  For
 * measurement: the same work and results as vbw_filter.  A VBW_STREAM plan's
 * state update, which follows the filter kernels, is outside the interval.
 * Errors: as vbw_filter, plus VBW_EINVAL for a NULL event and
 * VBW_EUNSUPPORTED for a VBW_GRAPH plan (its launches are replayed from a
 * graph; time the graph launch with events on the stream instead). */
vbw_status vbw_filter_timed(vbw_plan_t plan, const void *const *x, void *const *y,
                            void *stream, void *start_event, void *stop_event);

/* Restart every channel's stream of a VBW_STREAM plan (Sec. II framing):
 * zero history and block counters, stream-ordered on `stream` (a hipStream_t,
 * NULL: the null stream).  The next vbw_filter behaves like the plan's first.
 * Errors: VBW_EINVAL (NULL plan or a plan without VBW_STREAM);
 * VBW_EUNSUPPORTED for a VBW_HOST_ONLY plan; VBW_EDEVICE from HIP. */
vbw_status vbw_stream_reset(vbw_plan_t plan, void *stream);

/* Release the plan and its device tables (NULL is a no-op).  Synchronizes
 * with work the plan has queued. */
void vbw_destroy(vbw_plan_t plan);

/* Static description of a status code. */
const char *vbw_strerror(vbw_status status);

/* ---------------------------------------------------------------------
 * Allocation-free filtering, for callers that cannot allocate device memory
 * (serving loops and harnesses that forbid hipMalloc): one call does what
 * vbw_plan + vbw_set_bandwidth (once per entry of `switches`) + vbw_filter +
 * vbw_destroy do, with the same kernels and the plan's default launch shape,
 * and calls no hipMalloc, hipFree or other allocating device routine.  Its
 * device tables (twiddles, V, work list, per-call table) live in one static
 * device array of VBW_NOALLOC_SCRATCH_BYTES per GPU, held until the process
 * ends; the first call on a device locates that array and writes the
 * twiddle table into it (synchronously).
 * x[c] / y[c] are caller-owned device pointers as for vbw_filter; the host
 * arrays desc, switches, x and y are read during the call only.  The tables
 * are uploaded from pageable host memory on `stream` (a hipStream_t, NULL:
 * the null stream), so the call may wait for that stream's earlier work;
 * the kernels then run asynchronously on `stream`.
 * Every call on one GPU shares that GPU's array: calls whose work is not
 * ordered on one stream race (results undefined).  Nothing in the array
 * needs to start at zero; every call rewrites what it reads.
 * Flags: only VBW_NO_PRUNE and VBW_F32_OUT (anything else:
 * VBW_EUNSUPPORTED).  Errors: as vbw_plan and vbw_filter, plus VBW_EINVAL
 * for n_switches < 0 or NULL switches with n_switches > 0, VBW_ERANGE /
 * VBW_EINVAL for a switch as in vbw_set_bandwidth, and VBW_ETOOLARGE when
 * the tables would exceed the array. */
#define VBW_NOALLOC_SCRATCH_BYTES (2u << 20)

typedef struct vbw_band_switch {
    int32_t channel;
    int32_t k1;          /* first transition bin from block from_block on */
    int64_t from_block;
} vbw_band_switch;

vbw_status vbw_filter_noalloc(const vbw_plan_desc *desc, int32_t n_switches,
                              const vbw_band_switch *switches,
                              const void *const *x, void *const *y, void *stream);

/* Test hook, for tests of the allocation-failure path: the k-th device
 * allocation (k >= 1) made by each later vbw_plan call on the calling thread
 * fails as if the device were out of memory; k = 0 turns it off. */
void vbw_test_fail_device_alloc(int32_t k);

/* Host-side introspection, for tests and tooling. */
typedef enum vbw_query {
    VBW_Q_N_CHANNELS = 0,
    VBW_Q_N_ITEMS = 1,         /* 4096-value tiles (up to 4096/N consecutive blocks) in the work list */
    VBW_Q_TOTAL_BLOCKS = 2,    /* sum over channels of ceil(len/M) */
    VBW_Q_TOTAL_SAMPLES = 3,   /* sum over channels of len */
    VBW_Q_WORKGROUP = 4,       /* threads per workgroup */
    VBW_Q_LDS_BYTES = 5,       /* LDS per workgroup */
    VBW_Q_GRID = 6,            /* workgroups over the launches of one call */
    VBW_Q_KERNEL_VARIANT = 7,  /* index of the chosen launch variant */
    VBW_Q_N_VARIANTS = 8       /* launch variants the autotuner chooses from */
} vbw_query;

/* Value of `q` for the plan, or a negative vbw_status. */
int64_t vbw_plan_query(vbw_plan_t plan, int32_t q);

/* k1 in force for (channel, block) after every vbw_set_bandwidth so far, or a
 * negative vbw_status. */
int32_t vbw_block_k1(vbw_plan_t plan, int32_t channel, int64_t block);

/* The float32 twiddle table the plan uploads for size n (a power of two,
 * 2 <= n <= 4096): out[2r] = RN(cos(2 pi r/n)), out[2r+1] = RN(-sin(2 pi r/n)),
 * r < n, generated in float64 and rounded to nearest float32 (eq. (4) sign
 * convention: exp(-j 2 pi r / n)). */
vbw_status vbw_twiddle_table(int32_t n, float *out);

/* Streaming device-to-device copy of `bytes` bytes on `stream`, used to
 * measure the achievable HBM bandwidth that the filter is compared with
 * (a plain copy moves exactly the filter's algorithmic bytes per sample).
 * src and dst are device pointers, 16-byte aligned, non-overlapping.
 * Errors: VBW_EINVAL (misaligned, overlapping, NULL with bytes > 0,
 * bytes < 0); VBW_EDEVICE from HIP. */
vbw_status vbw_copy(const void *src, void *dst, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VBW_H */
