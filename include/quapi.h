/*
 * quapi.h -- C ABI of the MI355X (gfx950) path-propagation library for
 * MACGIC-iQUAPI (mask-assisted coarse-graining of influence coefficients,
 * iterative quasi-adiabatic propagator path integral).
 *
 * The library propagates the augmented reduced density tensor of a quantum
 * system bilinearly coupled to a harmonic bath (Sec. 2, eqs. tot_ham,
 * quapi_red_rho, SysP, inf_fun).  The tensor is a sparse set of paths: each
 * path is the sequence of forward/backward state pairs over the memory window
 * (dk_max points) plus a complex weight.  One time step (Sec. 2.1, Sec. 3.1,
 * Sec. 3.2.1):
 *   1. merge the stored paths that agree on the mask positions (pre-merging on
 *      the reduced mask {mask[i]-1 : i>=1}, or post-merging on the mask);
 *      a group keeps the sum of the member weights and, as representative
 *      history, the member of largest |w|;
 *   2. extend every group by every forward/backward pair: weight times the
 *      short-time propagator element (eq. SysP) times the influence factor of
 *      the new point with the points of the window (eq. inf_fun, lags 0..dk_max);
 *   3. drop children whose |w| is below theta (Sec. 2.1, path filtering);
 *   4. add the survivors to rho(t) (Sec. 3.2.1).
 * All device memory is owned by the library; every step runs as HIP kernels
 * on one stream without host synchronisation.
 *
 * Conventions (all functions):
 *   - return QUAPI_OK (0) or a negative QUAPI_E* code; quapi_strerror() names it;
 *   - a context is used by one host thread at a time; the only state shared
 *     between contexts is, per device, the library stream of contexts that pass
 *     no stream and the event that orders step kernels (both thread-safe);
 *   - complex numbers are quapi_c64 {re, im}; matrices are row-major;
 *   - pair index p = a*M + b for forward state a and backward state b;
 *   - hbar = 1.
 */
#ifndef QUAPI_H
#define QUAPI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } quapi_c64;

#define QUAPI_OK            0
#define QUAPI_EINVAL       -1   /* invalid argument                                   */
#define QUAPI_ENOMEM       -2   /* device allocation failed or group capacity exceeded */
#define QUAPI_EDEVICE      -3   /* HIP runtime error or kernel-reported fault          */
#define QUAPI_ESTATE       -4   /* call not valid in the current state                 */
#define QUAPI_EUNSUPPORTED -5   /* valid input this build does not handle              */

#define QUAPI_PRE   0           /* pre-merging (Sec. 3.1): merge on {mask[i]-1 : i>=1} before extending */
#define QUAPI_POST  1           /* post-merging (Sec. 2.1): merge the children on the mask              */

#define QUAPI_FP64      0       /* amplitudes and influence exponents in FP64                           */
#define QUAPI_FP32_LOG  1       /* precision form: stored amplitudes as FP32 (ln|w|, arg w); each       */
                                /* child's influence exponent (eq. inf_fun) and amplitude formed in     */
                                /* FP32 in that log domain; the merge sums (Sec. 3.1.2), the eta table  */
                                /* and the rho(t) sums stay FP64.  This form has no bucketed store:    */
                                /* DIRECT where it applies, else the hash-table merge.  Results differ  */
                                /* from the FP64 form by the FP32 rounding of each child, and the      */
                                /* filter and representative decisions                                  */
                                /* near their thresholds may differ too                                 */

/* Where the groups live and how they merge (Sec. 3.1.2; quapi_params.merge). */
#define QUAPI_MERGE_AUTO     0  /* DIRECT where it applies, else BUCKETED where it applies, else the      */
                                /* hash-table store merged through partitions (PARTITION)                  */
#define QUAPI_MERGE_DIRECT   1  /* a slot per key of the merge positions 0..L-1 (two-level systems,       */
                                /* 6 <= L <= 12, FP64 or FP32_LOG, lone contexts): the parents that merge  */
                                /* are the occupied slots of an aligned segment of four, every merged      */
                                /* group has a fixed slot; a step is a planner (the occupied segments     */
                                /* listed by group count) and one kernel whose waves never wait on one    */
                                /* another                                                                  */
#define QUAPI_MERGE_BUCKETED 2  /* merge positions 0..L-1: groups sorted by key in buckets of their top   */
                                /* points, merged on chip as runs of neighbours                             */
#define QUAPI_MERGE_HASH     3  /* any merge positions: histories in one or two words, merged through an   */
                                /* open-addressing hash table in device memory                             */
#define QUAPI_MERGE_PARTITION 4 /* the same store and the same groups as HASH, merged without a table:     */
                                /* each expand pass's merged children are appended (one counter increment  */
                                /* each, 32-byte entries) to partitions chosen by the hash of their key,   */
                                /* and a second kernel merges each partition in an LDS table and writes   */
                                /* its groups (no table scan, no second pass for the representative)      */

typedef struct quapi_ctx quapi_ctx;

/* Problem definition, copied by quapi_create (the caller keeps ownership of
 * every pointer and may free it after the call). */
typedef struct {
    int M;                    /* number of system (DVR) states, 2..4 (M > 4: QUAPI_EUNSUPPORTED; M = 4, */
                              /* 16 pairs, runs on the hash-table store only: HASH or PARTITION)       */
    const quapi_c64* H;       /* M*M Hermitian system Hamiltonian H_S (eq. tot_ham), used as given;     */
                              /* rejected if |H_ij - conj(H_ji)| > 1e-12 max(1, max|H|)                  */
    const double* q;          /* M coupling eigenvalues q_i of the DVR states (eq. tot_ham)             */
    double dt;                /* Trotter time step, > 0                                                 */
    int dk_max;               /* memory length K (Sec. 2): a stored path holds K points, lags 0..K-1;   */
                              /* the new point couples to lags 0..K                                     */
    const quapi_c64* eta;     /* 3*(K+1) influence coefficients, three columns of K+1 lags:             */
                              /*  eta[0*(K+1)+d]  both points interior (window dt),                     */
                              /*  eta[1*(K+1)+d]  one point is the initial or final point (window dt/2),*/
                              /*  eta[2*(K+1)+d]  initial x final point (d >= 1);                       */
                              /* eta[1*(K+1)+0] is the end-point self term (eq. inf_fun)                 */
    const int* mask;          /* MACGIC mask (Sec. 2.1): n_mask sorted lags, mask[0]=0, mask[1]=1,      */
                              /* mask[n_mask-1] <= K-1; NULL: every lag 0..K-1.  Merge positions       */
                              /* 0..L-1 (L >= 2, M <= 3) run on the direct-mapped or bucketed store    */
                              /* (see merge); any other set takes the hash-table store and needs the   */
                              /* history in 128 bits, the merge positions in 62 and the other          */
                              /* positions in 64 (M = 2: K <= 63, at most 31 merge and 32 other        */
                              /* positions; M = 3 and 4: half of each)                                 */
    int n_mask;
    double theta;             /* filter: drop a child when |w|^2 < theta^2; 0 disables                  */
    const quapi_c64* rho0;    /* M*M initial reduced density matrix                                     */
    int mode;                 /* QUAPI_PRE or QUAPI_POST                                                */
    int qbits;                /* representative choice compares |w|^2 = re*re + im*im (no fused         */
                              /* multiply-add) with its low qbits mantissa bits cleared; equal values    */
                              /* go to the history that is smaller read from the oldest point.          */
                              /* < 0: default 32, or 40 in the FP32 precision form (whose rounding of    */
                              /* |w|^2, ~1e-6 relative, must stay well below the compared quantum).     */
                              /* Parity with the oracle is tested at the defaults; at qbits 8 and 20 a  */
                              /* few representatives differ from the oracle's (alike on every store)   */
    long long max_groups;     /* stored groups to allocate for, spread evenly over the key buckets     */
                              /* (at least one each; an uneven fill reports ENOMEM first); 0: room   */
                              /* for every key of the merge positions (hash-table store: up to 2^21). */
                              /* The direct-mapped store always holds every key: AUTO takes it only   */
                              /* when max_groups is 0 or at least P^L                                 */
    int max_steps;            /* initial capacity of the rho(t) history; grows on demand; <= 0: 1024    */
    void* stream;             /* hipStream_t to run on (e.g. a torch stream); NULL: the library's      */
                              /* stream of the device, shared by every context that passes NULL.  A     */
                              /* step kernel needs the whole GPU resident, so the library orders the    */
                              /* step kernels of one device across all streams: a step kernel on     */
                              /* another stream than the last one waits for it; other work overlaps  */
    int precision;            /* QUAPI_FP64 (0) or QUAPI_FP32_LOG                                       */
    int merge;                /* QUAPI_MERGE_*: the store (0, AUTO: DIRECT, else BUCKETED, else         */
                              /* PARTITION, the first that applies); a store that does not apply       */
                              /* returns QUAPI_EUNSUPPORTED; HASH and PARTITION take any mask           */
} quapi_params;

/* Per-step counters, available for every step t >= 1 that has completed. */
typedef struct {
    int t;
    long long n_groups;       /* groups extended at step t                                              */
    long long n_children;     /* n_groups * M^2 (path-steps of step t)                                  */
    long long n_survivors;    /* children with |w| >= theta                                             */
    long long n_stored;       /* groups stored after step t (the groups step t+1 extends)               */
    double dropped_abs;       /* sum of |w| over the filtered children                                  */
} quapi_stepstat_t;

/* Layout facts of a context (for accounting and tests). */
typedef struct {
    int M, P, K, L;           /* P = M*M pairs; L = key length in points (merge positions 0..L-1)     */
    int bits_per_point;       /* history bits per point                                                 */
    int record_bytes;         /* bytes of one stored group: 8 key + 8 history tail + 16 weight (32),    */
                              /* 8 history tail + 16 weight (24) on the direct-mapped store, whose slot  */
                              /* is the key, or 8 or 16 history + 16 weight (24 or 32) on the hash-table */
                              /* merge; the FP32 precision form stores an 8-byte weight (16 B records on */
                              /* the direct-mapped store)                                                 */
    long long capacity;       /* maximum number of stored groups (of one instance)                      */
    size_t device_bytes;      /* device memory held by the context                                      */
    int precision;            /* QUAPI_FP64 or QUAPI_FP32_LOG                                           */
    int hash_merge;           /* 1: the hash-table store (HASH or PARTITION), 0: a store sorted by key  */
    int n_instances;          /* instances of a batched context, else 1                                 */
    int store;                /* QUAPI_MERGE_DIRECT, _BUCKETED, _HASH or _PARTITION                      */
} quapi_info_t;

/* Create a context and its initial state t = 0 (one path per nonzero
 * element of rho0, weighted by the initial point's self term).
 * Errors: EINVAL (bad argument), EUNSUPPORTED (M > 4; merge positions 0..L-1
 * with L bits-per-point > 62 bits or a tail over 64 bits; other merge positions
 * with a history over 128 bits, a key over 62 bits or other positions over 64
 * bits; coefficients whose influence phases could reach 1e5 radians in one
 * step, |q_a - q_b| sum_d |Im eta_d| max|q_a + q_b| >= 1e5, beyond the range
 * of the kernels' sine and cosine), ENOMEM, EDEVICE.  *out is NULL on error. */
int quapi_create(const quapi_params* p, quapi_ctx** out);

/* Batched form: n_inst instances of the method (for instance bath parameter
 * points of eq. SD) that share every field of p but the influence
 * coefficients (p->eta is not read) and, optionally, the system Hamiltonian,
 * propagated together: each step is one launch of the step kernel over the
 * groups of all instances.  Instance j's coefficients are
 * eta_batch[3*(K+1)*j .. 3*(K+1)*(j+1)-1], laid out as quapi_params.eta; its
 * Hamiltonian is H_batch[M*M*j ..] when H_batch is not NULL (each checked as
 * p->H is), else p->H.  The caller keeps ownership of both.  Each instance's results
 * (rho(t), counters, groups) are those of a context created with quapi_create
 * on its own coefficients and the same bucket layout.  p->max_groups counts
 * one instance.  The functions without "batch" in their name address
 * instance 0.  Merge positions 0..L-1 (the bucketed store), FP64 only.
 * Errors: as quapi_create; EINVAL (n_inst < 1 or > 1024, eta_batch NULL or not
 * finite, an H_batch matrix not Hermitian), EUNSUPPORTED (the hash-table store
 * or the FP32 form). */
int quapi_create_batch(const quapi_params* p, int n_inst, const quapi_c64* eta_batch, const quapi_c64* H_batch,
                       quapi_ctx** out);

/* Enqueue n_steps time steps on the context's stream; returns without waiting.
 * Errors: EINVAL (n_steps < 0), ESTATE (a previous step failed), ENOMEM
 * (history growth), EDEVICE.  A capacity overflow inside a step is reported by
 * the next synchronising call; the context then stays at the last complete step. */
int quapi_step(quapi_ctx* c, int n_steps);

/* Enqueue n_steps >= 1 time steps, in the step order of Sec. 3.2.1 (merge,
 * extend, filter, rho(t)), as one HIP graph: the launches quapi_step makes,
 * recorded once after a kernel that clears the look-back words, then replayed
 * by later calls that start at the same step with the same buffers (after
 * quapi_reset, for instance).  A call that does not match the recorded run
 * records anew.  Results equal quapi_step's bit for bit.  Launch timing
 * (quapi_profile_*) skips graph steps.  The direct-mapped and bucketed stores
 * (lone or batched).
 * Recording captures the context's stream: nothing else may be enqueued on it
 * meanwhile (e.g. by another thread's context on the shared library stream). 
 * Errors: EINVAL (n_steps < 1), ESTATE (a previous step failed), ENOMEM
 * (history growth), EUNSUPPORTED (the hash-table store), EDEVICE (capture,
 * instantiation or launch failed). */
int quapi_step_graph(quapi_ctx* c, int n_steps);

/* Wait for the enqueued steps; returns the first error a step reported. */
int quapi_sync(quapi_ctx* c);

/* Current time step (number of completed steps; synchronises). */
int quapi_time(quapi_ctx* c, int* t_out);

/* rho(t) for 0 <= t <= current step into caller-owned rho_out[M*M] (synchronises). */
int quapi_rho(quapi_ctx* c, int t, quapi_c64* rho_out);

/* rho(t0 .. t0+n-1) into caller-owned out[n*M*M] (synchronises). */
int quapi_rho_history(quapi_ctx* c, int t0, int n, quapi_c64* out);

/* Counters of steps t0 .. t0+n-1 (t0 >= 1) into caller-owned out[n] (synchronises). */
int quapi_step_stats(quapi_ctx* c, int t0, int n, quapi_stepstat_t* out);

/* The stored groups (the groups the next step extends), in store order (sorted
 * by merge key on the direct-mapped and bucketed stores):
 * hist[i*K + j] = pair index of group i at lag j (0 for lags the paths do not
 * yet hold), w[i] = group amplitude.  Writes min(n, cap) groups; *n_out = n.
 * hist or w may be NULL with cap = 0 to query n (synchronises). */
int quapi_groups(quapi_ctx* c, long long cap, unsigned char* hist, quapi_c64* w,
                 long long* n_out);

/* As quapi_rho_history, quapi_step_stats and quapi_groups, for instance inst
 * (0 <= inst < n_instances) of a batched context.  Errors: EINVAL (inst out of
 * range), as the instance-0 forms otherwise. */
int quapi_batch_rho_history(quapi_ctx* c, int inst, int t0, int n, quapi_c64* out);
int quapi_batch_step_stats(quapi_ctx* c, int inst, int t0, int n, quapi_stepstat_t* out);
int quapi_batch_groups(quapi_ctx* c, int inst, long long cap, unsigned char* hist, quapi_c64* w,
                       long long* n_out);

/* rho(t0 .. t0+n-1) of every instance into caller-owned out[n][n_instances][M*M],
 * in one copy (synchronises).  Errors: as quapi_rho_history. */
int quapi_batch_rho_all(quapi_ctx* c, int t0, int n, quapi_c64* out);

/* Run length of the step kernel's chunk assignment: a workgroup takes `run`
 * consecutive chunks of the group order, then moves `run` times the grid on
 * (1 = round-robin).  In the batched form a longer run changes instance less
 * often (a chunk reloads its instance's coefficients) and finds its look-back
 * predecessor in the same workgroup; a lone context ignores it.  Results do not
 * depend on it.  Errors: EINVAL (run < 1 or > 64). */
int quapi_set_chunk_run(quapi_ctx* c, int run);

/* Time n_steps steps from t = 0 with each run length of 1, 2, 4, 8, 16 (HIP
 * events on the context's stream), keep the fastest, write it to *run_out (may
 * be NULL) and return the context to t = 0.  A lone context keeps 1 without
 * timing.  Errors: EINVAL, ESTATE (a step had failed), and those of quapi_step. */
int quapi_autotune(quapi_ctx* c, int n_steps, int* run_out);

/* Return to t = 0 with the initial state (tables and buffers are kept). */
int quapi_reset(quapi_ctx* c);

int quapi_info(quapi_ctx* c, quapi_info_t* out);

/* The hipStream_t the context runs on. */
void* quapi_stream(quapi_ctx* c);

const char* quapi_strerror(int code);

/* Launch timing, for measurement.  quapi_profile_begin clears the record and
 * makes the next quapi_step calls record HIP events on the context's stream
 * around each of the next max_launches steps: one before the step kernel, one
 * between it and the planner that follows it, one after the planner.  On the
 * hash-table store: one before the expand kernel, one after it, one after the
 * rest of the step.
 * Errors: EINVAL (max_launches < 1), ENOMEM, EDEVICE. */
int quapi_profile_begin(quapi_ctx* c, int max_launches);

/* Durations in milliseconds of the recorded steps, oldest first: step_ms[k] of
 * the step kernel, plan_ms[k] of the planner after it (either array may be NULL);
 * on the hash-table store, of the expand kernel and of the rest of the step.
 * Writes min(cap, n) entries, *n_out = n; synchronises and stops recording.
 * Errors: EINVAL, ESTATE (no recording began), EDEVICE. */
int quapi_profile_end(quapi_ctx* c, int cap, double* step_ms, double* plan_ms, int* n_out);

/* Free the context and its device memory (synchronises first).  NULL is a no-op. */
void quapi_destroy(quapi_ctx* c);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the propagation of
 * quapi_create + quapi_step(n_steps) on the direct-mapped store
 * (QUAPI_MERGE_DIRECT) as one call that allocates nothing.  Every buffer of the
 * run lives in one 96 MiB file-scope device array that each device holds
 * until the process ends; the host tables reach the device as kernel
 * arguments.  Enqueues on p->stream (NULL: the null stream) and returns
 * without waiting; rho_out is a caller-owned DEVICE buffer of
 * (n_steps+1)*M*M quapi_c64, filled with rho(0..n_steps) when the stream
 * reaches the end of the run.  The results equal those of a context created
 * with merge = QUAPI_MERGE_DIRECT.  Calls that overlap on one device share the
 * array and race: order them (one stream, or events).
 * Takes M = 2, FP64, dk_max <= 40, merge positions 0..L-1 with 6 <= L <= 10,
 * p->merge AUTO or DIRECT; p->max_groups and p->max_steps are not read.
 * Errors: EINVAL (bad argument, as quapi_create), EUNSUPPORTED (a problem
 * outside that range), ENOMEM (the run needs more than the 96 MiB array:
 * about 70 B per slot of 4^L plus 48 B per step), EDEVICE. */
int quapi_run_static(const quapi_params* p, int n_steps, quapi_c64* rho_out);

/* ---------------------------------------------------------------- host utilities */

/* Spectral density of eq. SD as an Ohmic part plus Brownian-oscillator peaks:
 *   J(w) = (pi/2) ohmic_alpha w exp(-w/ohmic_wc)
 *        + sum_k 2 lam_k gam_k w0_k^2 w / ((w0_k^2 - w^2)^2 + gam_k^2 w^2),
 * peaks[3k..3k+2] = (w0_k, gam_k, lam_k) with lam_k = (1/pi) int J_k(w)/w dw. */
typedef struct {
    double ohmic_alpha, ohmic_wc;
    int n_peaks;
    const double* peaks;
} quapi_bath;

/* eta columns (layout of quapi_params.eta) for the bath at inverse temperature
 * beta, step dt and memory dk_max: integrals of the bath response function
 * over the Trotter windows of the two points (interior: dt; initial/final
 * point: dt/2), from g(t) = int_0^t int_0^t' alpha.  Host only, no GPU needed.
 * Errors: EINVAL. */
int quapi_eta(const quapi_bath* bath, double beta, double dt, int dk_max, quapi_c64* eta_out);

/* U = exp(-i H dt) (M*M, row-major) as the library computes it, by a Jacobi
 * eigendecomposition.  Host only.  Errors: EINVAL (M out of 1..8, non-Hermitian H). */
int quapi_propagator(int M, const quapi_c64* H, double dt, quapi_c64* U_out);

#ifdef __cplusplus
}
#endif

#endif /* QUAPI_H */
