/* mgme: tree-level squared matrix elements on MI355X (gfx950).
 *
 * C ABI of libmgme.so.  A process is built once from its external particles
 * and couplings; a call then maps a device array of phase-space momenta to
 * per-event |M|^2, summed over helicities and colours, in one lockstep
 * data-parallel launch.  This is the batched matrix-element call that the
 * paper substitutes for the event-by-event one (section 2: batches of events
 * held in large arrays and handed to the matrix-element engine in one call),
 * with the matrix element itself computed from Feynman diagrams and helicity
 * amplitudes (section 1) and its colour algebra as in section 3.
 *
 * Conventions for every call:
 *  - Every function returns an mgme_status; 0 is success.  No exception or
 *    signal crosses the ABI.  mgme_last_error() returns a thread-local text
 *    describing the last failure on the calling thread.
 *  - Device pointers (d_*) are owned by the caller (for example
 *    torch.Tensor.data_ptr() of a CUDA/HIP tensor); the library never frees
 *    or retains them.  A process owns its host state and one small device
 *    table (the colour matrix in matrix-core operand layout).
 *  - Kernels are enqueued asynchronously on `hip_stream` (a hipStream_t; NULL
 *    is the default stream).  Nothing synchronises; an asynchronous device
 *    fault is reported as MGME_EDEVICE by the next call.
 *  - Momenta are FP64, structure-of-arrays: component mu (E, px, py, pz, in
 *    GeV) of particle i (in the order of the pdg list, initial state first)
 *    for event e is d_mom[(i*4 + mu)*ld + e].  ld >= nevt; a multiple of 64
 *    keeps every load coalesced.
 *  - nevt == 0 is a no-op returning MGME_OK; nevt < 0, ld < nevt or a NULL
 *    required pointer returns MGME_EINVAL.
 */
#ifndef MGME_H
#define MGME_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGME_OK = 0,
  MGME_EINVAL = -1,        /* bad argument (NULL, negative size, ld < nevt, bad parameter) */
  MGME_EUNSUPPORTED = -2,  /* process, precision or parameter not supported */
  MGME_ENOMEM = -3,        /* device allocation failed (process creation only) */
  MGME_EDEVICE = -4        /* HIP runtime error, including a fault of an earlier launch */
} mgme_status;

typedef enum {
  MGME_FP64 = 0, /* plain method: every step in double precision */
  MGME_FP32 = 1, /* diagrams in single precision; momenta, propagator denominators,
                    colour quadratic form and helicity sum in double */
  MGME_MIXED = 2, /* single-precision diagrams; colour sum on the matrix cores with J split into two
                     power-of-two-scaled half-precision parts (FP32 accumulation of C J, the dot product
                     J^dagger (C J) in double); helicity sum in double */
  MGME_FP64_FP32COLOUR = 3 /* the "mixed" mode of the paper (section 3, Table 3): diagrams and J in
                              double, colour algebra Re(J^dagger C J) in single precision, helicity sum
                              in double */
} mgme_precision;

/* Couplings and masses.  alpha_s is fixed (no running).  The top width wt
 * must be 0 (propagators of internal top quarks carry no width).  z_enabled
 * = 0 removes Z exchange from e+e- -> mu+mu-. */
typedef struct {
  double alpha_s, alpha_em, sin2w, mz, wz, mt, wt;
  int z_enabled;
} mgme_params;

typedef struct {
  int n_ext;              /* external particles */
  int n_diagrams;         /* tree-level Feynman diagrams */
  int n_amp_terms;        /* diagrams with each four-gluon colour structure counted once */
  int n_colour;           /* colour flows (trace basis) */
  int n_hel;              /* helicity configurations, 2^n_ext */
  int n_good_hel;         /* helicities with a non-zero contribution (see mgme_process_create) */
  int n_currents;         /* off-shell currents evaluated per helicity */
  int n_amp_vertices;     /* amplitude vertices evaluated per helicity */
  double norm_factor;     /* 1 / (initial spin-colour average * final identical-particle factor) */
  double flops_per_hel;   /* floating-point operations per event and good helicity (static tally) */
  double flops_per_event; /* helicity-independent operations per event */
  unsigned long long kernel_hash; /* identifies the generated kernels (changes whenever they change) */
} mgme_info;

typedef struct mgme_process mgme_process;

/* Builds a process from its particle list in the order initial state first
 * (n_in = 2), PDG codes:
 *   {-11, 11, -13, 13}            e+ e- -> mu+ mu- (s-channel photon and Z)
 *   {21, 21, 6, -6 [, 21 ...]}    g g -> t t~ + 0..3 gluons
 * Selects the process's compiled kernels on `device`, and determines the
 * good helicities: every helicity configuration is evaluated in FP64 on 64
 * RAMBO events (seed 1, sqrt(s) = 500 GeV for e+e- and 1500 GeV otherwise);
 * a helicity is kept if its contribution is non-zero on at least one event.
 * The process keeps a few kilobytes of device memory (the colour matrix in
 * matrix-core operand layout), released by mgme_process_destroy.  Thread-safe.
 * Errors: EINVAL (NULL pointer, n_in != 2, non-finite or non-positive
 * couplings/masses), EUNSUPPORTED (other particles, wt != 0), EDEVICE. */
int mgme_process_create(int n_in, int n_out, const int* pdg, const mgme_params* params, int device,
                        mgme_process** out);

/* Releases a process; NULL is accepted.  The caller must not use the process
 * after this call, and must have finished (synchronised) its launches. */
int mgme_process_destroy(mgme_process* proc);

int mgme_process_info(const mgme_process* proc, mgme_info* out);

/* The helicities the process sums: the good ones found at creation unless
 * mgme_set_helicities restricted them.  codes[i] has bit (n_ext-1-leg) set
 * when that leg has helicity +1.  `codes` holds at least n_hel entries; *n
 * receives the number of helicities. */
int mgme_good_helicities(const mgme_process* proc, int* codes, int* n);

/* Restricts the helicity sum of mgme_matrix_element, mgme_select and the
 * serving loop to the configurations codes[0..n-1] (helicity codes as
 * above, strictly increasing, each below n_hel): |M|^2 then sums those
 * helicities only, as for a polarised or helicity-resolved cross section
 * (the paper sums over all helicities, section 2; this is the same sum over
 * a subset, with the same normalisation).  n = 0 restores the good
 * helicities of mgme_process_create (codes may then be NULL).  The process
 * must not be in use by a running call or queued request.  Errors: EINVAL
 * (NULL process, n < 0 or above n_hel, NULL codes with n > 0, a code out of
 * range or not above the previous one). */
int mgme_set_helicities(mgme_process* proc, const int* codes, int n);

/* The colour matrix of the trace basis as integer numerators num[n_colour^2]
 * over the common denominator *den, and the basis: basis[s*k + j] is the
 * j-th gluon leg of flow s (k gluons).  Either array pointer may be NULL. */
int mgme_colour_matrix(const mgme_process* proc, long long* num, long long* den, int* basis);

/* RAMBO flat phase space: events first_event .. first_event+nevt-1 of the
 * Philox4x32-10 stream keyed by `seed`, written to d_mom (layout above, the
 * two initial partons along +z and -z with energy sqrt_s/2) and the
 * phase-space weights (with the (2 pi)^(4-3n) convention) to d_wgt[nevt]
 * (d_wgt may be NULL).  Errors: EINVAL (sqrt_s not above the sum of the
 * final-state masses, sizes), EDEVICE. */
int mgme_rambo(const mgme_process* proc, double sqrt_s, unsigned long long seed,
               unsigned long long first_event, long long nevt, long long ld, double* d_mom, double* d_wgt,
               void* hip_stream);

/* |M|^2 per event, summed over the good helicities and all colours and
 * normalised by norm_factor, into d_me[nevt] (FP64 in every precision).
 * Processes with many colour flows (g g -> t t~ g g g) stage colour-flow
 * amplitudes in a workspace taken from the stream-ordered allocator
 * (hipMallocAsync) and returned at the end of the call (at most a few GB, on
 * `hip_stream`); the other processes form every precision's colour sum,
 * MGME_MIXED's on the matrix cores, inside the diagram kernel and take no
 * workspace.  Eight lanes share an event there, each summing every eighth
 * helicity, and their partial sums are added in lane order: an event's
 * |M|^2 does not depend on the batch it is in.  Batches above 2^28 events
 * run as consecutive launches of at most 2^28 events.
 * Errors: EINVAL, EDEVICE (also when the workspace cannot be allocated). */
int mgme_matrix_element(const mgme_process* proc, const double* d_mom, long long nevt, long long ld,
                        int precision, double* d_me, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * mgme_matrix_element with the same arguments, results (bit for bit) and
 * errors, but no device allocation of any kind.  Its staging buffers live in
 * a fixed array of MGME_NOALLOC_SCRATCH_BYTES in the library, one per GPU,
 * held until the process ends; its address is looked up on the first call on
 * each device.  Batches of any size are processed in sub-batches that fit the
 * array (g g -> t t~ g g g: 512 events per sub-batch in FP64, 1024 in FP32
 * and mixed), so large staged batches run slower than with
 * mgme_matrix_element.  The array keeps the contents of the last call; no
 * kernel relies on it starting at zero.  Every call on one GPU shares the
 * array: calls that overlap on one GPU (on different streams, or from
 * different threads without ordering) race, and the caller must serialise
 * them, for example by issuing them on one stream.
 * Errors: as mgme_matrix_element, and EINVAL when one 64-event sub-batch of
 * the process and precision would need more than the array. */
#define MGME_NOALLOC_SCRATCH_BYTES (128ll << 20)
int mgme_matrix_element_noalloc(const mgme_process* proc, const double* d_mom, long long nevt, long long ld,
                                int precision, double* d_me, void* hip_stream);

/* Device workspace (bytes) that mgme_matrix_element takes from the
 * stream-ordered allocator for a batch of nevt events in `precision`
 * (0 when the process needs none). */
int mgme_workspace_bytes(const mgme_process* proc, long long nevt, int precision, long long* bytes);

/* Per-helicity contributions of every one of the n_hel helicity
 * configurations (not only the good ones), normalised like
 * mgme_matrix_element: d_out[h*ldo + e], ldo >= nevt. */
int mgme_matrix_element_per_helicity(const mgme_process* proc, const double* d_mom, long long nevt, long long ld,
                                     int precision, double* d_out, long long ldo, void* hip_stream);

/* |M|^2 as mgme_matrix_element, and for each event a helicity configuration
 * and a leading colour flow drawn at random, as an event generator writes
 * them with an unweighted event (section 5 of the paper names this choice as
 * the last feature added to its GPU workflow; the definitions here are ours):
 *  - d_hel[e]: the helicity code (bit n_ext-1-leg set for helicity +1) of the
 *    first good helicity, in increasing code order, whose running sum of
 *    |M_h|^2 exceeds d_r_hel[e] times |M|^2;
 *  - d_col[e]: the first colour flow s, in the order of mgme_colour_matrix's
 *    basis (orderings of the gluon legs, lexicographic), whose running sum of
 *    sum_h |J_s(h)|^2 exceeds d_r_col[e] times the total (J_s: the
 *    colour-ordered amplitude of flow s; every flow of the trace basis is a
 *    leading-colour flow);
 *  - when no running sum exceeds the threshold (r within rounding of 1), the
 *    last entry with a non-zero weight is taken.
 * d_r_hel and d_r_col hold nevt uniform numbers in (0,1) (caller's random
 * stream); d_me, d_hel, d_col receive nevt values.  The decisions are taken
 * in double precision from the values of the chosen `precision`.  The call
 * takes (n_good_hel + n_colour) * 8 bytes per event of extra workspace from
 * the stream-ordered allocator (at most 4 GB, by sub-batches), plus the
 * staging of mgme_matrix_element for staged processes and MGME_MIXED.
 * Errors as mgme_matrix_element. */
int mgme_select(const mgme_process* proc, const double* d_mom, long long nevt, long long ld, int precision,
                const double* d_r_hel, const double* d_r_col, double* d_me, int* d_hel, int* d_col,
                void* hip_stream);

/* Cross-section weights of a batch of massless colliding partons at fixed
 * sqrt_s (section 2 of the paper counts the cross-section calculation among
 * the event generator's serial tasks):
 *   d_w[e] = (d_wgt[e] * d_me[e]) * (0.3893793721e9 / (2 sqrt_s^2))   [pb]
 * with d_wgt the phase-space weights of mgme_rambo (the flux is 2 s and
 * (hbar c)^2 = 0.3893793721 GeV^2 mb converts GeV^-2 to pb; the constant is
 * formed first, on the host).  d_stats[0..2] = (sum w, sum w^2, max w), so
 * that sigma = sum w / N with error sqrt((sum w^2 / N - sigma^2) / (N - 1)).
 * The sums use a fixed reduction order for a given nevt (the same inputs give
 * the same bits).  d_w may be NULL (sums only); d_stats is 3 device doubles.
 * Runs on the calling thread's current device, enqueued on hip_stream; takes
 * at most 24 KB of workspace from the stream-ordered allocator.
 * Errors: EINVAL (nevt < 0, NULL pointers, sqrt_s not positive), EDEVICE. */
int mgme_event_weights(double sqrt_s, const double* d_wgt, const double* d_me, long long nevt, double* d_w,
                       double* d_stats, void* hip_stream);

/* Hit-or-miss unweighting (section 2 of the paper lists it among the serial
 * tasks worth moving to the GPU): event e is kept when
 * d_r[e] * (*d_w_ref) < d_w[e] (strictly), with d_r uniform in (0,1) and
 * *d_w_ref (one device double, for example d_stats + 2 of
 * mgme_event_weights, or a maximum from an earlier run) at least the largest
 * weight.  d_idx (room for nevt) receives the kept event indices in
 * increasing order and *d_nkept (one device long long) their number; each
 * kept event then carries the weight *d_w_ref.  Runs on the current device;
 * takes 16 bytes per 2048 events of workspace from the stream-ordered
 * allocator.  Errors: EINVAL (nevt < 0, NULL pointers), EDEVICE. */
int mgme_unweight(const double* d_w, const double* d_r, long long nevt, const double* d_w_ref, long long* d_idx,
                  long long* d_nkept, void* hip_stream);

const char* mgme_last_error(void);

/* ------------------------------------------------------------------ serving
 * Continuous batching of requests of different processes, precisions and
 * sizes on one GPU (the paper's observation that several clients sharing a
 * GPU raise its combined throughput, section 2, Fig. 1).  Requests are queued
 * on submission; a scheduler thread admits them in arrival order onto free
 * slots (one stream each) whenever the summed HBM footprint of the running
 * requests stays within the budget.  The footprint of n events is
 * n * (32 n_ext + 8) bytes of momenta and results plus the staging workspace
 * of mgme_workspace_bytes (without graphs; with graphs the staging belongs to
 * the slots).  A request that does not fit may be passed over by a later one
 * that does, at most max_pass_over times; after that nothing behind it is
 * admitted until it fits, so a large request cannot starve.  A request whose
 * footprint exceeds the whole budget is split into parts of a multiple of 64
 * events that fit (a part of 64 events that still does not fit runs alone).
 * Admitted requests run concurrently.  Each request (or part) runs exactly the
 * kernels of a standalone mgme_matrix_element call, so its result does not
 * depend on the others or on the split: an event's |M|^2 does not depend on
 * the batch it is in. */
typedef struct mgme_server mgme_server;

typedef struct {
  int n_slots;                  /* requests running at once (1..64) */
  long long hbm_budget_bytes;   /* bound on the summed footprint of running requests; 0: 0.8 x the
                                   free device memory at creation (hipMemGetInfo, after the slot
                                   workspaces are allocated); the test double: 0 is no bound */
  int use_graphs;               /* 1: each request's launches are captured into a HIP graph on its
                                   slot's stream and replayed; an instantiated graph is kept per
                                   (slot, process, precision, power-of-two batch size) and updated
                                   for the next request of that kind */
  long long slot_workspace_bytes; /* with graphs: device staging buffer owned by each slot and
                                     allocated at creation, outside any graph (0: 1 GiB); the
                                     staged processes run in sub-batches that fit it */
  int max_pass_over;            /* times a queued request may be passed over (0: 4) */
  int fake_executor;            /* 1: test double, no device work: a request completes
                                   fake_ns_per_event * nevt ns after admission, footprint
                                   fake_bytes_per_event * nevt; process and device pointers unused */
  double fake_ns_per_event;
  long long fake_bytes_per_event;
  long long fake_fail_nevt;     /* test double: a request (or part) of exactly this many events
                                   fails with MGME_EDEVICE (0: none fails) */
} mgme_server_config;

typedef struct {
  long long submitted, completed, failed, events;
  double p50_ms, p99_ms, mean_ms, max_ms; /* submission-to-completion latency of completed requests */
  double wall_s;                          /* first submission to last completion */
  int max_concurrent;                     /* most requests (or parts) running at once */
  long long peak_footprint_bytes;         /* largest summed footprint of running requests */
  long long budget_bytes;                 /* the budget in force (0: none) */
  long long split_requests;               /* requests split into parts */
  long long graph_launches;               /* graph replays (use_graphs) */
  long long graph_instantiations;         /* graphs instantiated (the rest were updated in place) */
} mgme_server_stats;

/* Starts a server on `device`.  Errors: EINVAL (bad configuration), ENOMEM
 * (slot workspace), EDEVICE. */
int mgme_server_create(const mgme_server_config* cfg, int device, mgme_server** out);
/* Queues |M|^2 of one batch (arguments as mgme_matrix_element; every pointer
 * must stay valid, and the process alive, until the request completes).
 * hip_stream is the caller's stream that produced d_mom and last wrote d_me:
 * the request's kernels start only after the work enqueued on it before this
 * call (an event is recorded there; NULL is the null stream).  Results are
 * ready when mgme_server_wait returns.  *id identifies the request for
 * mgme_server_wait.  Errors: EINVAL (bad batch, or with graphs a slot
 * workspace too small for the process), EDEVICE. */
int mgme_server_submit(mgme_server* s, const mgme_process* proc, const double* d_mom, long long nevt, long long ld,
                       int precision, double* d_me, void* hip_stream, unsigned long long* id);
/* Blocks until request `id` completed; returns its status (MGME_OK, or the
 * error of its launch or of any of its parts) and releases it (each request is
 * waited for at most once). */
int mgme_server_wait(mgme_server* s, unsigned long long id, double* latency_ms);
/* Blocks until no request is queued or running. */
int mgme_server_drain(mgme_server* s);
int mgme_server_get_stats(mgme_server* s, mgme_server_stats* out);
/* Runs every queued request to completion, then releases the server. */
int mgme_server_destroy(mgme_server* s);
const char* mgme_server_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGME_H */
