/*
 * atfd.h - C ABI of libatfd, asynchrony-tolerant (AT) finite differences on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: K. Aditya & D. A. Donzis, "High-order asynchrony-tolerant finite
 * difference schemes for partial differential equations", arXiv 1702.00496.
 *
 * A periodic 1-, 2- or 3-D box is split into simulated processing elements
 * (PEs). Every PE face receives its neighbour's edge values through a ring of
 * past time levels and sees them with a random delay k in [0, L-1] (Sec. 2),
 * drawn per step and per face from a counter-based generator (Sec. 5.1).
 * Points whose stencil crosses a face combine T successive delayed levels with
 * weights c_m(k) so that the delay error cancels to the scheme's order
 * (Sec. 3.4 Example 3 eq. cd4-at; Tables atschemes-left/right); all other
 * points take the standard central difference (Sec. 2 eq. general_deriv).
 * The right-hand side is advection-diffusion or viscous Burgers (Sec. 5 eq.
 * general) and is advanced with Euler, AB2, AB3 (Sec. 4.1 eqs. time_disc,
 * time_ab2) or Heun RK2.
 *
 * Conventions for every call:
 *  - Device pointers ("_dev") point to HIP device memory owned by the caller.
 *    The library never allocates or frees device memory: all its state lives
 *    in a caller-provided workspace whose size the *_workspace_size calls
 *    report. Host pointers are read during the call only.
 *  - Fields are dense C-order arrays [nz][ny][nx] (x fastest) of the bulk
 *    precision: double for AT_F64, float for AT_F32_F64B. Grid nodes are
 *    x_i = i * length / n (per axis).
 *  - Work is queued on the HIP stream given at creation; calls that return
 *    numbers to the host synchronise that stream.
 *  - Errors are reported only through the status code; at_last_error()
 *    returns a text for the most recent failure of a context (or, with NULL,
 *    of the calling thread). Nothing throws across this interface.
 *  - A context is used by one host thread at a time.
 */
#ifndef ATFD_H
#define ATFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AT_OK = 0,
  AT_EINVAL = 1,     /* invalid argument or unsupported combination            */
  AT_ENOMEM = 2,     /* workspace too small                                    */
  AT_EHIP = 3,       /* a HIP runtime call failed                              */
  AT_EUNSTABLE = 4,  /* a norm evaluation met a non-finite value (blow-up)     */
  AT_ESTATE = 5      /* call out of order (e.g. at_step before at_set_state)   */
} at_status;

/* Model equation (Sec. 5 eq. general). */
enum { AT_ADVDIFF = 0,   /* u_t + c . grad u = alpha lap u                     */
       AT_BURGERS = 1 }; /* u_t + u (sum_d u_{x_d}) = alpha lap u (scalar)     */

/* Time integrator (Sec. 4.1). AB2 starts with one Euler step, AB3 with Euler
 * then AB2. RK2 is Heun's method; its predictor u* is a field of its own
 * with its own ring of past levels, so its stage derivative is also AT. */
enum { AT_EULER = 0, AT_AB2 = 1, AT_AB3 = 2, AT_RK2 = 3 };

/* Arithmetic. AT_F32_F64B: fields, history and rings stored in float, the
 * bulk stencil in float, the AT combination of delayed levels and all error
 * norms in double. */
enum { AT_F64 = 0, AT_F32_F64B = 1 };

/* Delay model. RNG: one draw per step, PE and face from the counter-based
 * generator below. ZERO: every delay is 0 (the scheme then equals the
 * synchronous one). HOST: delays from a caller table. SYNC: the synchronous
 * reference scheme that reads neighbours' current values directly (no ring
 * traffic; the comparison arm "standard scheme"). */
enum { AT_DELAY_RNG = 0, AT_DELAY_ZERO = 1, AT_DELAY_HOST = 2, AT_SYNC = 3 };

/* AT family at the points next to a PE face (Tables atschemes-left/right).
 * TIME: the time-expanded schemes, a combination of T delayed levels of the
 * central difference (rows (1,2,2)b, (2,2,2)b, (1,4,2), (2,4,2), (2,6,2) and
 * their order-6 first-derivative sibling); with k = 0 they are the CD.
 * SPACE_212, SPACE_222: the space-expanded single-level schemes of the
 * second-order CD (Sec. 5.1 Cases 2 and 3): one delayed level n-k of 2 or 3
 * buffer points; first derivative (1,2,2)a, second derivative (2,1,2) or
 * (2,2,2)a. They are not the CD at k = 0, and a face whose delay is 0 keeps
 * the CD (they act at communication-delayed buffer points). The printed
 * left-boundary (1,2,2)a carries a sign slip (its coefficients do not sum to
 * zero); the library uses the mirror image of the right-boundary row, which
 * is what the order conditions (Sec. 3.1 eq. cond) give.
 * NONUNIFORM_212: the non-uniform-delay class (Sec. 3.4 Example 1): the two
 * buffer points next to a face carry their own delays, k1 (nearest, the
 * face's draw) and k2 (a second draw, see the generator below). First
 * derivative eq. ex1-0, ((k2 - 4k1), 3k1, -k2, k1) / (2 (3k1 - k2)) at
 * (i-1, i, i+1 @ n-k1, i+2 @ n-k2); second derivative the same footprint
 * solved from eq. cond at the accuracy of the (2,1,2) row:
 * ((2k1 - k2), (2k2 - 3k1), -k2, k1) / (3k1 - k2). Both reduce to (1,2,2)a
 * and (2,1,2) when k1 = k2. On the singular set 3k1 = k2 (k1 >= 1) the
 * nearest point takes the next older level k1 + 1 (the paper prescribes
 * altering a delay there); with k1 = k2 = 0 the point keeps the CD2. Left
 * faces use the mirror image. Order 2, T = 0 or 1, no host delay tables. */
enum { AT_SCHEME_TIME = 0, AT_SCHEME_SPACE_212 = 1, AT_SCHEME_SPACE_222 = 2, AT_SCHEME_NONUNIFORM_212 = 3 };

typedef struct at_problem {
  int32_t ndim;        /* 1, 2 or 3                                              */
  int32_t pe[3];       /* PEs per axis (x, y, z); unused axes 1                  */
  int64_t n[3];        /* points per axis; n[d] % pe[d] == 0; unused axes 1      */
  double length;       /* periodic box edge (same on every axis), e.g. 2*pi     */
  double c[3];         /* advection velocity (AT_ADVDIFF)                        */
  double alpha;        /* diffusivity (AT_ADVDIFF) or viscosity (AT_BURGERS)     */
  double dt;           /* time step                                              */
  int32_t equation;    /* AT_ADVDIFF | AT_BURGERS                                */
  int32_t order;       /* spatial order a: 2, 4 or 6; half-width s = a/2         */
  int32_t integrator;  /* AT_EULER | AT_AB2 | AT_AB3 | AT_RK2                    */
  int32_t precision;   /* AT_F64 | AT_F32_F64B                                   */
} at_problem;

/*
 * Delay generator (the paper leaves it unspecified, Sec. 5.1): with
 *   G = 0x9E3779B97F4A7C15 and mix() the SplitMix64 finaliser
 *   (Steele, Lea & Flood, OOPSLA 2014),
 *   face = p * 2 * ndim + 2 * axis + side   (p = px + PX*(py + PY*pz),
 *                                            side 0 = low neighbour),
 *   u53  = mix(seed + ((n << 32 | face) + 1) * G) >> 11,
 *   k~   = first j with u53 < THR[j],  THR[j] = floor(2^53 * W_j / W_{L-1})
 *          with W_j the running sum of the integer bin weights,
 *   k    = min(k~, max(0, n - T + 1))   (no level before t = 0 is touched).
 * Every buffer point of one face uses the same k (uniform-delay class),
 * except under AT_SCHEME_NONUNIFORM_212, whose second buffer point draws its
 * own k with face + P * 2 * ndim in place of face (P = number of PEs).
 */
typedef struct at_delay {
  int32_t L;                 /* maximum delay levels, k in [0, L-1]; 1..8       */
  int32_t T;                 /* time levels in the AT combination; 0 = order/2+1;
                                1 = standard scheme fed with delayed halos     */
  int32_t mode;              /* AT_DELAY_RNG | AT_DELAY_ZERO | AT_DELAY_HOST | AT_SYNC */
  int32_t scheme;            /* AT_SCHEME_TIME | AT_SCHEME_SPACE_212 | AT_SCHEME_SPACE_222
                                | AT_SCHEME_NONUNIFORM_212; the single-level
                                schemes need order 2, T = 0 or 1, PE edges
                                >= 2 (212) or >= 3 (222), and are not covered
                                by at_adjoint                                 */
  uint64_t seed;             /* generator key                                   */
  const uint32_t* weights;   /* host, L integer bin weights (p_j ~ weights[j]);
                                NULL = uniform                                  */
  const int8_t* host_delays; /* host, AT_DELAY_HOST: [host_nsteps][P][ndim][2],
                                each in [0, L-1]; copied at creation            */
  int64_t host_nsteps;
} at_delay;

typedef struct at_ctx at_ctx;
typedef struct at_ens at_ens;

/* Library version string. */
const char* at_version(void);

/* Bytes of device workspace at_create needs for this problem (256-B aligned
 * sub-buffers: the solution (one buffer updated in place, or two used by
 * step parity for the synchronous arm and for 3-D problems of fewer than
 * 1024 PEs without a 32 x 32 PE cross-section, or with the non-uniform
 * scheme, that do not use RK2; problems the 32 x 32 path takes keep their
 * fields PE after PE internally, which at_set_state and at_get_state
 * translate),
 * the integrator history, the RK2 predictor, the face rings of L+T slots,
 * delay tables, counters and reduction scratch). */
at_status at_workspace_size(const at_problem* prob, const at_delay* delay, size_t* bytes);

/* Create a context on `ws_dev` (>= at_workspace_size bytes, 256-B aligned)
 * queuing work on `hip_stream` (a hipStream_t; NULL = default stream): the
 * problem of Sec. 5 eq. general (advection-diffusion or viscous Burgers,
 * periodic box) split into PEs as in Sec. 2, with the delay model of
 * Sec. 5.1 (one delay per PE face and step, drawn from the generator above,
 * zero, or a host table). Derives the central-difference taps and the level
 * weights c_m(k) of the AT combination (Sec. 3.4 Example 3, eq. cd4-at).
 * Validates: ndim 1..3; divisibility; PE edge >= 2s on used axes; order in
 * {2,4,6}; 1 <= L <= 8; 1 <= T <= 4; host delays < L; a PE tile whose
 * sweep workgroup needs more than the 160 KB of LDS of a compute unit (the
 * generic 3-D sweep splits large cross-sections into y-halves where it may
 * split a PE, which lowers the need) (AT_EINVAL); AT_ENOMEM when ws_bytes
 * is too small. The library keeps `ws_dev` and the
 * stream; the caller keeps ownership of both and of every host array. */
at_status at_create(const at_problem* prob, const at_delay* delay, void* ws_dev,
                    size_t ws_bytes, void* hip_stream, at_ctx** out);

/* Set u^0 (the initial condition of Sec. 5.1 eq. IC or any field; bulk
 * precision, device, [nz][ny][nx] x fastest, copied) and reset the step
 * counter to 0. Every ring slot is filled with the edge strips of u^0 (no
 * level exists before t = 0; the start-up clamp of the delays keeps their
 * weights at zero). AT_EINVAL for a null pointer. */
at_status at_set_state(at_ctx* ctx, const void* u0_dev);

/* Advance nsteps time steps (queued on the context's stream, asynchronous):
 * per step the delay draw (Sec. 5.1), the AT combination of the delayed ring
 * levels at the points of I_B and the standard central difference elsewhere
 * (Sec. 2 eqs. general_deriv, general_deriv_async; Sec. 3.4 eq. cd4-at), the
 * right-hand side of Sec. 5 eq. general and the time update of Sec. 4.1
 * (eqs. time_disc, time_ab2; AB3; Heun), then the publish of the new edge
 * strips into the ring slot of level n+1. AT_ESTATE before at_set_state,
 * AT_EINVAL when a host delay table is too short, AT_EHIP on launch failure. */
at_status at_step(at_ctx* ctx, int64_t nsteps);

/* Capture chunks of `chunk` steps into a HIP graph and replay it inside
 * at_step (0 disables). All per-step quantities are read from a device
 * counter, so one graph serves every chunk. */
at_status at_set_graph(at_ctx* ctx, int32_t chunk);

/* Tuning of the sweep schedule of the 3-D kernel for 32 x 32 PE cross-
 * sections: `depth` = D, the z-planes of reads kept in flight per thread
 * (1, 2 or 4) with 4 points per thread and 256 threads per PE, or 8 + D with
 * 2 points per thread and 512 threads per PE, or 16 + D with 4 points per
 * thread and the z sweep direction alternating from launch to launch (each
 * launch starts on the planes the previous one touched last, which the
 * Infinity Cache still holds); 0 = the library default. For the generic
 * 3-D sweep (other PE shapes), 32 + c with c in {1, 2, 4, 8, 16} splits
 * every PE's planes into c z-chunks of one workgroup each (clamped to the
 * PE depth; only where the sweep may split a PE: two solution buffers or
 * Heun) instead of the cost-model split. Every
 * variant computes bit-identical results; only speed differs. Other shapes
 * ignore it. Problems of the 32 x 32 path accept only the variants that
 * path runs for them (D must divide the PE depth; the space-expanded schemes
 * take 1 and 2): AT_EINVAL otherwise. The default is 2, or 1 where two
 * planes in flight do not divide the PE depth. */
at_status at_set_tuning(at_ctx* ctx, int32_t depth);
at_status at_get_tuning(const at_ctx* ctx, int32_t* depth);

/* Autotune: time `nsteps` steps for every candidate schedule, keep the
 * fastest and return it in *best_depth (ms per step of each candidate in
 * ms_out[AT_TUNE_CANDIDATES] for variants 1, 2, 4, 9, 10, 12, 17, 18, 20, 33, 34,
 * 36, 40, 48, -1 where a variant does not apply; the z-chunk variants apply
 * only to problems the 32 x 32 path does not take; may be NULL). The field
 * and all history are
 * saved to `scratch_dev` (>= at_checkpoint_size bytes) first and restored
 * afterwards, so the simulation is unchanged. Synchronises the stream. */
enum { AT_TUNE_CANDIDATES = 14 };
at_status at_autotune(at_ctx* ctx, void* scratch_dev, size_t scratch_bytes, int32_t nsteps,
                      int32_t* best_depth, double* ms_out);

/* Copy the current field u^n (bulk precision, [nz][ny][nx], x fastest) to
 * the caller's device buffer `u_dev` (Sec. 2: the solution at time level n).
 * AT_ESTATE before at_set_state. Queued on the context's stream. */
at_status at_get_state(at_ctx* ctx, void* u_dev);

/* Current step number n, i.e. t = n dt (host-side mirror; no
 * synchronisation). */
at_status at_get_step(const at_ctx* ctx, int64_t* n);

/* Delays k (after the start-up clamp) of steps n0 .. n0+count-1, computed on
 * the device with the same routine the step kernel uses:
 * host_out[count][P][ndim][2] (int8). Synchronises the stream. */
at_status at_get_delays(at_ctx* ctx, int64_t n0, int64_t count, int8_t* host_out);

/* AT_SCHEME_NONUNIFORM_212 only (Sec. 3.4 Example 1): delays of the second
 * buffer point of every face (the generator draw with face + P * 2 * ndim,
 * after the start-up clamp, before the singular-set shift of k1), laid out as
 * at_get_delays, whose table holds k1. AT_EINVAL for other schemes.
 * Synchronises the stream. */
at_status at_get_point_delays(at_ctx* ctx, int64_t n0, int64_t count, int8_t* host_out);

/* Error norms of the current field (Sec. 4 averages; Sec. 5.1 error E = u -
 * u_a), accumulated in double with a fixed reduction order. Reference: the
 * decaying advected Fourier series of Sec. 5.1 eq. ana_sol with nmodes > 0
 * (kappa host [nmodes][3], amp, phase host [nmodes]; evaluated at t = n dt as
 * sum A exp(-alpha |kappa|^2 t) sin(kappa . (x - c t) + phase)), or, with
 * nmodes == 0, the double field `ref_dev` [nz][ny][nx].
 * out (host, 9 doubles): mean|E|, rms E, max|E| over all points; mean|E|,
 * rms E over I_B (points within s of a PE face); mean|E|, rms E over I_I;
 * |I_B|; |I_I|. Returns AT_EUNSTABLE if any value is not finite.
 * Synchronises the stream. At most 16 modes. */
at_status at_norms(at_ctx* ctx, int32_t nmodes, const int32_t* kappa, const double* amp,
                   const double* phase, const double* ref_dev, double* out);

/* Allocation-free variant of at_norms, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): same arguments, results and errors, but the
 * per-workgroup partial sums and the result live in a static device array of
 * the library (1024 x 8 + 16 doubles, one per GPU, held until the process
 * ends) instead of the context's workspace. Calls no allocating routine.
 * Must be called with the context's device current (AT_EINVAL otherwise).
 * Calls that overlap on one GPU share that array and race: serialise them. */
at_status at_norms_noalloc(at_ctx* ctx, int32_t nmodes, const int32_t* kappa, const double* amp,
                           const double* phase, const double* ref_dev, double* out);

/* Checkpoint: bytes needed, save to / restore from `ckpt_dev`. The state is
 * the field, the integrator history, every ring slot and the step counter; a
 * restored run continues bit for bit. */
at_status at_checkpoint_size(const at_ctx* ctx, size_t* bytes);
at_status at_save(at_ctx* ctx, void* ckpt_dev);
at_status at_load(at_ctx* ctx, const void* ckpt_dev);

/* Release the context (device memory stays with the caller). */
at_status at_destroy(at_ctx* ctx);

/* Text of the last failure of `ctx`, or of the calling thread for NULL. */
const char* at_last_error(const at_ctx* ctx);

/* ------------------------------------------------------------------------
 * Discrete adjoint of the AT step (advection-diffusion or viscous Burgers;
 * Euler, AB2 or Heun RK2; every delay mode of the time-expanded schemes; AB3
 * and the space-expanded schemes are not covered: AT_EINVAL). This is not
 * in the paper: it is the exact transpose of the linearised discrete map that
 * at_step applies, so that gradients of a function J(u^N) of the field after
 * N steps can be taken with respect to the initial field and the diffusivity
 * (viscosity).
 *
 * at_adjoint runs the N forward steps from the state set at step 0, saving a
 * checkpoint every `every` steps, then sweeps backwards: each segment is
 * recomputed from its checkpoint, its levels kept, and the transposed steps
 * are applied from lambda^N = seed (dJ/du^N, bulk precision, device) down to
 * lambda^0 = dJ/du^0, which is written to grad_u0_dev. Contributions to older
 * levels through the AT halos go to an adjoint ring of the forward ring's
 * shape (the delayed levels' transpose); RK2 keeps a second one for the
 * predictor's levels. Burgers linearises around the recomputed forward
 * levels of the segment. *grad_alpha receives
 * dJ/dalpha = sum_n <dJ/df^n, d f^n / d alpha>, accumulated in double in a
 * fixed order. The context is left at step N with the forward field.
 * Scratch (device, 256-B aligned) of at_adjoint_scratch_size bytes holds the
 * checkpoints, the levels of one segment (two when a segment's levels and
 * ring copies take at most 4 GB: segment s-1 is then recomputed on a second
 * stream of the library, at default priority, while segment s is reversed),
 * three adjoint fields and the adjoint ring. Synchronises the stream.
 * AT_ESTATE unless the context is at step 0.
 */
at_status at_adjoint_scratch_size(at_ctx* ctx, int64_t nsteps, int32_t every, size_t* bytes);
at_status at_adjoint(at_ctx* ctx, int64_t nsteps, int32_t every, const void* seed_dev, void* scratch_dev,
                     size_t scratch_bytes, void* grad_u0_dev, double* grad_alpha);

/* ------------------------------------------------------------------------
 * Delay ensembles: many independent 1-D advection-diffusion problems, each
 * with its own grid, PE count, scheme, L and generator key, advanced together
 * in one persistent launch. Their errors give the statistics over delay
 * realisations and grid spacings that the paper's error analysis averages
 * over (Sec. 4 ensemble averages; Sec. 5.1 realisations of the delays).
 * Member fields are packed one after another, member i starting at
 * sum_{j<i} n_j, in the bulk precision.
 */
typedef struct at_ens_member {
  int64_t n;                 /* points of this periodic 1-D problem              */
  int32_t pe;                /* PEs; n % pe == 0 and n / pe >= 2s                */
  int32_t order;             /* 2, 4 or 6                                        */
  int32_t integrator;        /* AT_EULER | AT_AB2                                */
  int32_t L;                 /* 1..8                                             */
  int32_t T;                 /* 0 = order/2+1; 1..4                              */
  int32_t mode;              /* AT_DELAY_RNG | AT_DELAY_ZERO | AT_SYNC           */
  double length;             /* box length                                       */
  double c;                  /* advection speed                                  */
  double alpha;              /* diffusivity                                      */
  double dt;                 /* time step                                        */
  uint64_t seed;             /* generator key of this member (as at_delay.seed)  */
  const uint32_t* weights;   /* host, L integer bin weights; NULL = uniform      */
} at_ens_member;

/* Workspace bytes for `count` members (descriptors, schedule, two packed
 * field buffers, the packed AB2 history, every member's ring of L+T slots,
 * counters, norm results). */
at_status at_ens_workspace_size(int32_t count, const at_ens_member* members, int32_t precision,
                                size_t* bytes);

/* Create an ensemble on `ws_dev` (>= at_ens_workspace_size bytes, 256-B
 * aligned), queuing work on `hip_stream`. `precision` is AT_F64 or
 * AT_F32_F64B. Members are spread over workgroups by a longest-first balance
 * of their work; a member never spans two workgroups. Every member is
 * validated like at_create validates a problem. Synchronises the stream. */
at_status at_ens_create(int32_t count, const at_ens_member* members, int32_t precision, void* ws_dev,
                        size_t ws_bytes, void* hip_stream, at_ens** out);

/* Set u^0 of every member (packed, device, bulk precision), fill every ring
 * slot with its edge strips and reset the step counter to 0. */
at_status at_ens_set_state(at_ens* ens, const void* u0_dev);

/* Advance every member nsteps steps in ONE persistent launch: a workgroup
 * loops over the steps of its members with a workgroup barrier between
 * steps. The launch is captured into a HIP graph the first time a given
 * nsteps is run and the graph is replayed afterwards (the start step is read
 * from a device counter). */
at_status at_ens_run(at_ens* ens, int64_t nsteps);

/* Schedule: workgroups per compute unit (1, 2 or 4) and threads per
 * workgroup (256, 512 or 1024); 0 keeps the current value. Results are
 * bit-identical for every choice. */
at_status at_ens_set_tuning(at_ens* ens, int32_t groups_per_cu, int32_t threads);

/* The workgroup schedule of the persistent launch (host arrays): `*nbins`
 * workgroups; workgroup j runs the members order[bin_start[j]] ..
 * order[bin_start[j+1] - 1] (bin_start: nbins + 1 entries, order: one entry
 * per member; either may be NULL to query *nbins first). A workgroup holds
 * the descriptors of at most AT_ENS_BATCH members at a time: a larger bin
 * runs every step for its first AT_ENS_BATCH members, then for the next
 * ones (members are independent problems). */
enum { AT_ENS_BATCH = 24 };
at_status at_ens_get_schedule(const at_ens* ens, int32_t* nbins, int32_t* bin_start, int32_t* order);

/* Bytes of device scratch at_ens_autotune needs to keep the current state
 * (both field buffers, the AB2 history, the rings and the step counter). */
at_status at_ens_state_size(const at_ens* ens, size_t* bytes);

/* Autotune the schedule of the persistent launch (a12: launch shape search,
 * not a part of the method): time nsteps steps for every candidate
 * (workgroups per CU in {1, 2, 4}) x (threads in {256, 512, 1024}), candidate
 * c = 3 * (index of groups) + (index of threads), each from the current state
 * (saved to `scratch_dev`, >= at_ens_state_size bytes, and restored after
 * every candidate), keep the fastest and leave the ensemble at the state and
 * step it had. ms[AT_ENS_TUNE_CANDIDATES] (host, may be NULL) receives each
 * candidate's milliseconds per step. Every candidate gives bit-identical
 * results. AT_ESTATE before at_ens_set_state. Synchronises the stream. */
enum { AT_ENS_TUNE_CANDIDATES = 9 };
at_status at_ens_autotune(at_ens* ens, void* scratch_dev, size_t scratch_bytes, int64_t nsteps,
                          int32_t* best_groups, int32_t* best_threads, double* ms);

/* Current schedule choice (workgroups per CU, threads per workgroup). */
at_status at_ens_get_tuning(const at_ens* ens, int32_t* groups_per_cu, int32_t* threads);

/* Copy the packed current fields to `u_dev`. */
at_status at_ens_get_state(at_ens* ens, void* u_dev);

/* Current step number n (host-side mirror; no synchronisation). */
at_status at_ens_get_step(const at_ens* ens, int64_t* n);

/* Per-member error norms in double with a fixed reduction order:
 * out[count][3] = mean|E|, rms E, max|E|. Reference: the exact decaying
 * advected Fourier series of Sec. 5.1 eq. ana_sol (nmodes > 0: kappa and amp
 * [nmodes] shared by all members, phase [count][nmodes] per member, evaluated
 * at t = n dt of each member), or, with nmodes == 0, the packed double field
 * `ref_dev`. Returns AT_EUNSTABLE if any value is not finite. Synchronises the
 * stream. At most 16 modes. */
at_status at_ens_norms(at_ens* ens, int32_t nmodes, const int32_t* kappa, const double* amp,
                       const double* phase, const double* ref_dev, double* out);

/* Ensemble statistics of the per-member RMS error against the grid spacing
 * (Sec. 4 ensemble averages of the error over delay realisations; Sec. 5.1
 * error E = u - u_a). Members are grouped by spatial order (group 0, 1, 2 for
 * orders 2, 4, 6) and, within a group, by dx = length / n into `nbins`
 * (1..AT_ENS_MAX_DX_BINS) bins with host edges dx_edges[0] < ... <
 * dx_edges[nbins]; bin j holds edges[j] <= dx < edges[j+1], members outside
 * every bin are not counted. Host output out[(g * nbins + j) * 4 + q]: q = 0
 * member count, 1 mean dx, 2 mean of the members' RMS errors, 3 their
 * unbiased variance (denominator count - 1; 0 when count < 2). Reference as
 * for at_ens_norms; the per-member errors and the statistics are computed on
 * the device in double with a fixed summation order. Returns AT_EUNSTABLE if
 * any value is not finite, AT_EINVAL for bad bins. Synchronises the stream. */
enum { AT_ENS_MAX_DX_BINS = 64 };
at_status at_ens_error_stats(at_ens* ens, int32_t nmodes, const int32_t* kappa, const double* amp,
                             const double* phase, const double* ref_dev, int32_t nbins, const double* dx_edges,
                             double* out);

/* Release the ensemble (device memory stays with the caller). */
at_status at_ens_destroy(at_ens* ens);

/* Text of the last failure of `ens`, or of the calling thread for NULL. */
const char* at_ens_last_error(const at_ens* ens);

/* ------------------------------------------------------------------------
 * Scheme derivation (host only, exact arithmetic; no device work, no
 * context, callable without a GPU).
 *
 * A stencil is n pairs (j[i], l[i]): the scheme uses u_{i+j}^{n-l} (Sec. 3.2
 * eq. general_deriv_at2). The order conditions of Sec. 3.1 eq. cond are
 * imposed for every Taylor term u^{(p,q)} with p + r q < d + a (dt ~ dx^r),
 * and the system is classified by the rank test of the Sec. 3.1 derivation
 * recipe. Coefficients are exact reduced fractions num[i] / den[i] (den > 0)
 * of the dimensionless scheme: d^d u/dx^d ~ sum_i c_i u_{i+j[i]}^{n-l[i]} / dx^d.
 */
enum { AT_DERIVE_UNIQUE = 0,    /* rank(A) = rank(A|b) = n: one scheme          */
       AT_DERIVE_NONE = 1,      /* rank(A) < rank(A|b): the stencil has none    */
       AT_DERIVE_INFINITE = 2   /* rank(A) = rank(A|b) < n: a family            */
};

typedef struct at_derivation {
  int32_t status;      /* AT_DERIVE_*                                           */
  int32_t order;       /* accuracy a whose conditions were imposed             */
  int32_t n_cond;      /* equations (terms with p + r q < d + a)               */
  int32_t n_unknown;   /* stencil entries                                      */
  int32_t rank_a;      /* rank(A)                                              */
  int32_t rank_ab;     /* rank(A|b)                                            */
} at_derivation;

/* Derive the scheme of derivative order d (1..4) and accuracy a (1..12) for
 * dt ~ dx^r (r 1..4) on the stencil (j[n], l[n]) (host arrays, 1 <= n <= 48,
 * |j| <= 32, 0 <= l <= 64, no repeated pair). Writes num[n], den[n] and
 * *info. UNIQUE: the scheme. INFINITE: one member of the family (the free
 * unknowns set to zero). NONE: all zero. AT_EINVAL for out-of-range
 * arguments or when exact 128-bit arithmetic would overflow (never rounds). */
at_status at_derive_scheme(int32_t d, int32_t a, int32_t r, int32_t n, const int32_t* j, const int32_t* l,
                           int64_t* num, int64_t* den, at_derivation* info);

/* Search for the smallest AT scheme of a fixed interior layout (step 2 of the
 * Sec. 3.1 recipe, done systematically): interior points j = -s_min..0 at
 * level n (j = 0 only if with_centre), buffer points j = 1..s_max each at the
 * T successive levels n-k .. n-k-T+1 (the uniform-delay layout of Sec. 3.2 eq.
 * cond-async2 for T = 1, the time-expanded one for T > 1). s_max grows from 1
 * to max_extent; a stencil whose system has a family of solutions takes
 * further conditions (a + 1, a + 2, ...) while the family persists and, if
 * that leaves no scheme, is reduced by one buffer entry (oldest level of the
 * farthest point first) (both routes of recipe step 3); the first unique
 * scheme with a nonzero buffer coefficient is returned
 * (*n_out entries of j_out, l_out, num, den, at most `cap`; info->order is the
 * accuracy reached). side = -1 mirrors it to a buffer on the left
 * (j -> -j, coefficients times (-1)^d). *n_out = 0 and info->status =
 * AT_DERIVE_NONE when none exists up to max_extent (1..32). */
at_status at_search_scheme(int32_t d, int32_t a, int32_t r, int32_t s_min, int32_t with_centre, int32_t k,
                           int32_t T, int32_t side, int32_t max_extent, int32_t cap, int32_t* n_out,
                           int32_t* j_out, int32_t* l_out, int64_t* num, int64_t* den, at_derivation* info);

#ifdef __cplusplus
}
#endif

#endif /* ATFD_H */
