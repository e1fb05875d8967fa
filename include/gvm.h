/*
 * gvm.h -- C-ABI of the GPU virtualization manager (GVM) for MI355X.
 *
 * The method (Li, Narayana, El-Ghazawi, "Efficient Resource Sharing Through
 * GPU Virtualization on Accelerated High Performance Computing Systems"):
 * many SPMD host processes share one GPU through a single manager process
 * that owns the only device context (Section 4.2.2, Section 5).  Each
 * process sees its own virtual GPU (VGPU, Section 5), hands its input to the
 * manager through a per-process shared-memory space, and the manager runs
 * every process's copy-in, kernel and copy-out as concurrent device work
 * instead of time-sliced contexts (Section 4.2.1, concurrency types (a)-(c)).
 *
 * Two sides live in one library, libgvm.so:
 *   - the manager ("daemon") side: gvm_init builds every resource and starts
 *     the service thread in the calling process, which then owns the HIP
 *     context of device 0;
 *   - the rank side: gvm_attach / gvm_submit / gvm_wait / gvm_detach, callable
 *     from any process (or thread) on the same host; ranks never touch the
 *     GPU, they talk to the manager through POSIX shared memory only.
 *
 * The routines map onto the API of Section 5 as follows:
 *   REQ()        -> gvm_attach     (acquire the VGPU of a rank)
 *   SND()+STR()  -> gvm_submit     (input into the rank's shared memory, start)
 *   STP()+RCV()  -> gvm_wait       (poll for the result, copy it out)
 *   RLS()        -> gvm_detach     (release the VGPU) / gvm_shutdown
 *
 * Conventions
 *   - Every function returns a gvm_status (0 = GVM_OK, negative = error)
 *     unless stated otherwise; no C++ exception crosses this boundary.
 *     gvm_last_error() gives a text for the calling thread's last error.
 *   - One thread drives one rank at a time (SPMD); different ranks may be
 *     driven by different threads or processes concurrently.
 *   - All element data is IEEE-754 binary32, packed, host byte order.
 *   - Callers own the `in` and `out` buffers; the library owns the shared
 *     memory, the pinned staging, the device memory and the HIP objects.
 */
#ifndef GVM_H
#define GVM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
enum gvm_status {
  GVM_OK = 0,
  GVM_EINVAL = -1,     /* bad argument: rank out of range, n == 0, unknown kernel id, bad config */
  GVM_ENOMEM = -2,     /* request larger than the rank's shared memory space or the HBM budget */
  GVM_EAGAIN = -3,     /* request ring full (non-blocking submit) */
  GVM_ETIMEDOUT = -4,  /* gvm_wait timed out; the request is still pending */
  GVM_EDEAD = -5,      /* the peer (manager or rank process) has died */
  GVM_ESTATE = -6,     /* wrong call order: submit before attach, resident input missing, ... */
  GVM_EDEVICE = -7,    /* HIP runtime error or no usable gfx950 device; see gvm_last_error() */
  GVM_ESYS = -8,       /* operating-system error (shm_open, mmap, futex, ...) */
  GVM_ECANCELED = -9   /* request dropped because its rank detached or died */
};

/* ------------------------------------------------------------ kernel ids
 * Per-rank GPU tasks of the benchmark profiles (Table 3).  For a request of
 * size n the packed binary32 layouts of `in` and `out` are:
 *   GVM_K_VECADD        c = a + b                    in [a(n) | b(n)]            out [c(n)]
 *   GVM_K_BLACKSCHOLES  European call and put        in [S(n) | K(n) | T(n)]     out [call(n) | put(n)]
 *                       (rate r, volatility sigma from gvm_config)
 *   GVM_K_SGEMM         C = A B, n x n row-major     in [A(n*n) | B(n*n)]        out [C(n*n)]
 *   GVM_K_VECMUL        c = a * b (element-wise)     in [a(n) | b(n)]            out [c(n)]
 * and the compute-intensive EP-like kernel (the paper's NPB EP, Table 3 and
 * Section 6), n = number of pairs (1 .. 2^40), 64-bit words:
 *   GVM_K_EP            Gaussian-pair tally          in [k0 | k1] (uint64 key)
 *                       out [sx | sy (binary64) | q[0..9] (uint64)]
 *     pair j of the request takes the words 2j, 2j+1 of the Philox4x64-10
 *     stream of key (k0, k1) (block b = counter (b, 0, 0, 0) gives words
 *     4b .. 4b+3); u = (w >> 11) 2^-53, x = 2u - 1, y likewise; accepted when
 *     0 < t = x*x + y*y <= 1 (binary64, no fused multiply-add); then
 *     X = x sqrt(-2 ln t / t), Y = y sqrt(-2 ln t / t); sx, sy = sums of X, Y;
 *     q[l] = number of accepted pairs with l <= max(|X|, |Y|) < l + 1.
 */
enum gvm_kernel {
  GVM_K_VECADD = 1,
  GVM_K_BLACKSCHOLES = 2,
  GVM_K_SGEMM = 3,
  GVM_K_VECMUL = 4,
  GVM_K_EP = 5
};

/* ------------------------------------------------------------ manager modes */
enum gvm_mode {
  GVM_MODE_BATCH = 0,   /* request barrier of Section 5: wait until every attached rank
                           has a request (or batch_window_us expires), run them together.
                           With early_copy_in the inputs may move before the barrier; the
                           kernels never start before it.  Per-rank chains (PS2) are
                           enqueued a few at a time, finished requests answered between.
                           Large copies move in 32 MiB pieces */
  GVM_MODE_SERVING = 1  /* continuous admission: run requests as soon as device memory
                           (hbm_budget_bytes) and in-flight slots allow; up to two
                           requests of a rank in flight (see gvm_submit).  Large copies
                           move in 8 MiB pieces, the unit a small request waits behind */
};

/* Enqueue policy for a set of requests run together (Section 4.2.1):
 *   PS1      all copy-ins, then all kernels, then all copy-outs (Listing PS-1)
 *   PS2      per rank: copy-in, kernel, copy-out on the rank's stream (Listing PS-2);
 *            the kernel waits for its own input, the copies keep one FIFO per direction
 *   GROUPED  copy-ins per rank, then ONE persistent launch per kernel id that
 *            covers every rank's request, then copy-outs per rank
 *   AUTO     GROUPED when no request of the set moves more than 1 MiB over
 *            PCIe (inputs and results resident, or small copies kept on the
 *            kernel's stream); otherwise PS2, the paper's rule for I/O-intensive
 *            kernels (end of Section 4.2.3), which every kernel here is once
 *            its data crosses PCIe on this GPU */
enum gvm_policy { GVM_POLICY_AUTO = 0, GVM_POLICY_PS1 = 1, GVM_POLICY_PS2 = 2, GVM_POLICY_GROUPED = 3 };

/* Device backend.  HIP is the product path.  LOOPBACK runs the whole host
 * protocol (shared memory, rings, admission, grouping) without a GPU and
 * without computing any kernel: it copies each request's input bytes to its
 * output region unchanged, so that host-logic tests can check routing; it is
 * never chosen implicitly. */
enum gvm_backend { GVM_BACKEND_HIP = 0, GVM_BACKEND_LOOPBACK = 1 };

/* Submit flags (gvm_submit_ex). */
enum gvm_submit_flags {
  GVM_F_IN_RESIDENT = 1u,   /* the input is the one left on the device by this rank's previous
                               request with the same kernel id and n; no copy-in, `in` may be NULL.
                               Serving mode: when the previous request overlapped an earlier
                               one and finished first, its input is gone (GVM_ESTATE) */
  GVM_F_OUT_RESIDENT = 2u,  /* leave the result on the device; no copy-out, `out` may be NULL */
  GVM_F_NONBLOCK = 4u       /* return GVM_EAGAIN instead of waiting when the ring is full */
};

#define GVM_NAME_MAX 48

/* Manager configuration (gvm_init).  Call gvm_config_default first, then
 * override fields.  `size` must be sizeof(gvm_config). */
typedef struct gvm_config {
  uint32_t size;
  uint32_t nranks;              /* number of VGPUs (N_VGPU of Table 2), 1..256 */
  uint64_t shm_bytes_per_rank;  /* per-rank shared memory space (Section 5); bounds in+out of one request */
  uint64_t hbm_budget_bytes;    /* device memory the manager may hold for rank buffers */
  uint64_t staging_bytes;       /* pinned host staging per rank (0 = shm_bytes_per_rank) */
  uint32_t mode;                /* gvm_mode */
  uint32_t policy;              /* gvm_policy */
  uint32_t batch_window_us;     /* batch mode: longest wait for the barrier after the first request */
  uint32_t max_inflight;        /* serving mode: requests on the device at once (0 = two per
                                   rank) */
  uint32_t nstreams;            /* HIP streams for per-rank work (0 = min(nranks, 8)) */
  uint32_t use_graphs;          /* 1: grouped batches are captured once per template (ranks,
                                   kernels, sizes, copy flags, buffers) into a HIP graph and
                                   replayed with one hipGraphLaunch; requests then copy whole,
                                   not in pieces.  GVM_EINVAL together with latency_cus */
  uint32_t backend;             /* gvm_backend */
  uint32_t copy_threads;        /* host threads for shared-memory <-> pinned copies (0 = 4) */
  float bs_rate;                /* Black-Scholes risk-free rate r (default 0.02) */
  float bs_volatility;          /* Black-Scholes volatility sigma (default 0.30) */
  uint32_t batch_timing;        /* 1: time every batch's device phase (first copy-in to last
                                   copy-out) and every copy with device events (gvm_stats_json);
                                   in batch mode a batch is then enqueued as a whole once all of
                                   its inputs are staged, as in the execution model of Section
                                   4.2.3, so that its device phase is one span */
  uint32_t latency_cus;         /* serving mode: spatial partition of the device for QoS
                                   (0 = none).  A multiple of 32 below 256: requests whose
                                   estimated device time is at most 50 us (the latency class)
                                   run their kernels on a compute stream restricted to this
                                   many CUs, all others on a stream restricted to the other
                                   CUs, so that a short request never queues behind a long
                                   one for compute units.  Both partitions hold CUs of every
                                   XCD.  GVM_EINVAL for other values, in batch mode, or on a
                                   device without 256 CUs (gvm_init). */
  uint32_t small_request_bytes; /* serving mode: a request whose input and output total at
                                   most this many bytes is small.  Admission stays first-come
                                   first-served; after it a small request's staging copies
                                   (shared memory <-> pinned) go ahead of every larger
                                   request's queued ones on the copy threads.  The copies to
                                   and from HBM keep one FIFO per direction for every class
                                   (two concurrent streams in one direction cut the link's
                                   duplex rate).  0: one class, first-come first-served
                                   throughout.  Default 8 MiB */
  uint32_t early_copy_in;       /* batch mode: 1 (default) = while a batch runs, a rank whose
                                   request has been answered starts moving its next request's
                                   input (shared memory -> pinned -> HBM) as soon as the request
                                   arrives, once every input of the running batch is on its
                                   way; the request still joins the next request barrier
                                   (Section 5) and its kernel runs with that batch.  0: inputs
                                   move only after the barrier.  No effect with batch_timing
                                   or use_graphs, in serving mode, or for resident inputs */
  char name[GVM_NAME_MAX];      /* shared-memory namespace; "" = "gvm.<uid>" */
} gvm_config;

/* Fill `cfg` with defaults (nranks 8, 64 MiB per rank, budget 16 GiB, batch mode,
 * AUTO policy, window 2000 us, HIP backend, r 0.02, sigma 0.30, small requests up
 * to 8 MiB, early copy-in on). */
void gvm_config_default(gvm_config* cfg);

/* The CU masks the manager uses for gvm_config.latency_cus (extension; no
 * device needed): 8 words each, bit i = CU i of the 256 in HIP's numbering,
 * latency partition and bulk partition, disjoint and covering all CUs, with
 * the same share of every XCD in each.  Host-owned arrays of 8 uint32_t.
 * GVM_EINVAL unless latency_cus is a multiple of 32 in 32..224. */
int gvm_cu_partition_masks(uint32_t latency_cus, uint32_t* latency_mask, uint32_t* bulk_mask);

/* Manager side (Section 5, "GVM run-time process"): create the control
 * segment and one shared-memory space per rank, the single HIP context on
 * device 0, the streams, the device arena (hbm_budget_bytes) and the pinned
 * staging, then start the service thread and return.  One manager per
 * process.  GVM_EDEVICE if no gfx950 device is usable (the HIP backend never
 * falls back to the CPU). */
int gvm_init(const gvm_config* cfg);

/* Rank side, REQ() of Section 5: map the manager's segments of namespace
 * `name` (NULL = $GVM_NAME, else "gvm.<uid>") and claim VGPU `rank`
 * (0 <= rank < nranks).  Waits up to 10 s for the manager to come up.
 * GVM_ESTATE if the rank is already attached by a live process. */
int gvm_attach(int rank);
int gvm_attach_ns(const char* name, int rank);

/* Rank side, SND()+STR() of Section 5: queue one request of `kernel_id` with
 * size n (see the layouts above).  The input is copied into the rank's
 * shared memory before the call returns, unless `in` already points inside
 * the rank's space (gvm_rank_buffer), which is then used in place.  `out`
 * must stay valid until gvm_wait returns for this ticket; if it points
 * inside the rank's space the result is left there.  Returns a ticket >= 0
 * or a negative gvm_status.  Requests of one rank are admitted in submission
 * order.  In batch mode a rank has one request in flight at a time; in
 * serving mode a second plain request (no resident flags) may be admitted
 * while the first is still in flight, so that its copies overlap the first's
 * device work, and the two may finish in either order (wait by ticket or
 * with gvm_wait_any).  A request with resident flags waits until the rank
 * has nothing in flight. */
int64_t gvm_submit(int rank, int kernel_id, const void* in, void* out, uint64_t n);
int64_t gvm_submit_ex(int rank, int kernel_id, const void* in, void* out, uint64_t n, uint32_t flags);

/* Rank side, STP()+RCV() of Section 5: wait until request `ticket` of
 * `rank` has finished (ticket -1: every outstanding request of the rank),
 * copy its result to `out` and return its status.  timeout_ns < 0 waits
 * forever.  GVM_ETIMEDOUT leaves the request pending; GVM_EDEAD if the
 * manager died. */
int gvm_wait(int rank, int64_t ticket, int64_t timeout_ns);

/* As gvm_wait for one ticket (>= 0), and on return also stores the
 * request's timestamps (CLOCK_MONOTONIC ns) in ts[0..4]: submitted by the
 * rank, admitted by the manager, device work enqueued, device work observed
 * complete, result posted.  `ts` may be NULL. */
int gvm_wait_timed(int rank, int64_t ticket, int64_t timeout_ns, uint64_t* ts);

/* Wait for whichever outstanding request of `rank` finishes first; its
 * ticket goes to *ticket_out.  GVM_EINVAL if nothing is outstanding. */
int gvm_wait_any(int rank, int64_t timeout_ns, int64_t* ticket_out);
/* As gvm_wait_any, and stores the request's timestamps in ts[0..4] as
 * gvm_wait_timed does (`ts` may be NULL). */
int gvm_wait_any_timed(int rank, int64_t timeout_ns, int64_t* ticket_out, uint64_t* ts);

/* Rank side, RLS() of Section 5: wait for the rank's outstanding requests,
 * release its VGPU and unmap its segments.  Device buffers of the rank are
 * freed by the manager. */
int gvm_detach(int rank);

/* Release everything the calling process holds: detach its ranks and, if it
 * runs the manager, drain the outstanding work, stop the service thread,
 * free device memory, pinned memory and HIP objects and unlink the shared
 * memory. */
int gvm_shutdown(void);

/* Pointer to `bytes` bytes at the start of `rank`'s shared-memory space
 * (attached rank only), for zero-copy submission; NULL if too large. */
void* gvm_rank_buffer(int rank, uint64_t bytes);

/* Manager statistics (this process's manager) as a JSON object: per-kernel
 * launch count and device time from HIP events, request counts, latencies,
 * admission waits, peak device bytes.  Returns the JSON length, or a
 * negative status; the text is truncated to cap-1 bytes. */
int gvm_stats_json(char* buf, uint64_t cap);
/* Reset the manager's statistics counters (and the request trace). */
int gvm_stats_reset(void);

/* Write the manager's per-request trace to the file `path` as Chrome
 * trace-event JSON (opened by Perfetto and chrome://tracing): one track per
 * rank, and per request four slices from the manager's timestamps --
 * "queued" (submitted -> admitted: ring, request barrier, admission),
 * "copy-in" (admitted -> device work enqueued), "device" (enqueued -> seen
 * complete: copies to and from HBM and the kernel) and "copy-out" (-> result
 * posted), each with the ticket, n and status.  Covers the last 2^20
 * requests answered since gvm_init or gvm_stats_reset.  GVM_ESTATE without a
 * manager in this process, GVM_ESYS if the file cannot be written. */
int gvm_trace_dump(const char* path);

/* Text of the calling thread's last error ("" if none). */
const char* gvm_last_error(void);

/* Plain per-process path without virtualization (the execution cycle of
 * Section 4.1, Eq. 1): in the calling process, initialise the device
 * context, allocate device memory, copy `in` from pageable host memory,
 * run the same kernel code object the manager uses, copy the result back
 * to `out` and free the device memory.  Timings of the stages (seconds) go
 * to `t` (may be NULL): t[0] context init, t[1] allocation, t[2] copy-in,
 * t[3] kernel, t[4] copy-out, t[5] free. */
int gvm_plain_run(int kernel_id, const void* in, void* out, uint64_t n,
                  float bs_rate, float bs_volatility, double* t);

/* Allocation-free variant of gvm_plain_run, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It enqueues the same kernel code objects on
 * caller-owned device buffers and returns without waiting:
 *   d_in    device memory of the current device holding the packed input of
 *           the request (layouts above); 16-byte alignment gives the
 *           vectorised SGEMM loads;
 *   d_out   device memory receiving the packed output;
 *   stream  a hipStream_t of the current device (NULL: the null stream).
 * The caller owns both buffers and synchronises the stream before reading
 * d_out.  It calls no hipMalloc, hipFree or allocating routine.  The EP-like
 * kernel's per-unit partial records (96 bytes per 2^15 pairs) go to a static
 * device array of GVM_NOALLOC_SCRATCH_BYTES per GPU, held until the process
 * ends; an EP request needing more (n > 357,892,096 pairs) returns
 * GVM_ENOMEM before anything is enqueued.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (different streams or threads) race
 * and must be serialised by the caller.  GVM_EINVAL for a bad kernel id,
 * size or NULL buffer; GVM_EDEVICE for a device that is not a gfx950 or a
 * failed launch. */
#define GVM_NOALLOC_SCRATCH_BYTES (1u << 20)
int gvm_plain_run_noalloc(int kernel_id, const void* d_in, void* d_out, uint64_t n,
                          float bs_rate, float bs_volatility, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GVM_H */
