/*
 * pimdb -- bosonic path-integral MD exchange potential and forces on MI355X.
 *
 * C ABI of libpimdb.so.  The library evaluates, on one AMD gfx950 GPU, the
 * bosonic ring-polymer potential V^[1,N] of Feldman & Hirshberg, "Quadratic
 * Scaling Bosonic Path Integral Molecular Dynamics", and its force on every
 * bead, for one system or for a batch of independent systems of uneven size.
 *
 * Definitions (paper, Sec. "Background: cubic scaling bosonic PIMD" and
 * Sec. "Reducing the potential/force to O(N^2 + PN)"):
 *   - N particles of mass m, P beads each, d = 3; bead j of particle l is r_l^j.
 *   - k = (1/2) m omega_P^2.  omega_P is taken as given (the paper's choice
 *     is sqrt(P)/(beta hbar)).
 *   - E_int(l) = k sum_{j=1}^{P-1} |r_l^{j+1} - r_l^j|^2 (interior springs).
 *   - E^[u,v] = energy of the ring formed by particles u..v: interior springs,
 *     links from bead P of l to bead 1 of l+1, and the closing spring from
 *     bead P of v to bead 1 of u.
 *   - exp(-beta V^[1,v]) = (1/v) sum_{k=1}^{v} exp(-beta(V^[1,v-k] + E^[v-k+1,v])),
 *     V^[1,0] = 0  (the forward recurrence; V^[1,N] is "the energy").
 *   - forces = -grad V^[1,N] on all N*P beads: interior beads get the ordinary
 *     ring-polymer force; beads 1 and P get the connection-probability-weighted
 *     forces of Sec. "Force on exterior beads", with the probabilities of
 *     Sec. "Connection probabilities" and Methods.
 *   - Only the spring (kinetic) part is computed.  The interaction potential
 *     U-bar of the paper is not included; an optional harmonic trap
 *     (pimdb_set_trap) adds U-bar = (1/P) sum_j sum_l (1/2) m w^2 |r_l^j|^2.
 *
 * Data layout (all device pointers, FP64):
 *   - Positions and forces are bead-major structure-of-arrays of shape
 *     (P, 3, N): element (j, c, l) lives at index (j*3 + c)*N + l, with
 *     0-based bead j (j = 0 is the paper's bead 1, j = P-1 is bead P),
 *     component c and particle l.
 *   - A batch of S systems is packed back to back: system s starts at element
 *     offset pimdb_system_offset(h, s) = sum_{s'<s} 3 P_s' N_s'.
 *   - Energies: one double per system.
 *
 * Ownership and execution:
 *   - The caller owns every device buffer (positions, forces, energies,
 *     workspace, adjoint state).  The library owns its handle and two small
 *     device tables (system descriptors and the launch schedule) that it
 *     allocates in pimdb_set_system / pimdb_set_batch and frees in
 *     pimdb_destroy or on the next set call.
 *   - Evaluation calls are asynchronous on the handle's stream, allocate
 *     nothing, never synchronise the host and read no device value on the
 *     host, so they may be captured into a HIP graph.  pimdb_status and
 *     pimdb_debug_get are synchronous.
 *   - Output buffers are overwritten, never accumulated.  Inputs and outputs
 *     must not alias.  Calls on one handle must not overlap in time on
 *     different streams (they share the workspace).
 *
 * Errors: every int-returning call returns PIMDB_OK (0) or a negative code;
 * no exception crosses the ABI.  Errors found on the device (non-finite
 * inputs or results, exponent range) cannot be returned by asynchronous
 * calls; they set bits in a device status word read by pimdb_status.
 */
#ifndef PIMDB_H
#define PIMDB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define PIMDB_OK 0
#define PIMDB_EINVAL (-1)     /* bad argument: N < 1, P < 2, non-positive or non-finite beta/m/omega_P, L < 0, null pointer */
#define PIMDB_ENOSYS (-2)     /* no system or batch has been set on the handle */
#define PIMDB_EWORKSPACE (-3) /* no workspace bound, or the bound one is too small */
#define PIMDB_EDEVICE (-4)    /* HIP runtime error (no device, launch failure); see pimdb_last_error */
#define PIMDB_ENONFINITE (-5) /* returned by pimdb_status when the device status word is non-zero */
#define PIMDB_ERANGE (-6)     /* size outside the supported range (N above PIMDB_MAX_N, batch too large) */

/* ---- precision modes (pimdb_set_precision) ---- */
#define PIMDB_FP64 0  /* every step in IEEE double */
#define PIMDB_MIXED 1 /* endpoint-spring lengths |r_v^P - r_u^1|^2 in FP32 with compensated
                         summation (displacements formed in FP64); recursions, probabilities
                         and forces in FP64 */
#define PIMDB_FP64_DIRECT 2 /* FP64 with every pair displacement formed directly.  PIMDB_FP64 expands
                               |a - b|^2 around bead 1 of particle 0 for open systems (faster); its
                               rounding grows with the system's extent, and past the bound where
                               it still assures 1e-10 it sets PIMDB_STATUS_PRECISION.  This mode
                               has no such bound (about 25% slower). */

/* ---- algorithms (pimdb_set_algorithm) ---- */
#define PIMDB_ALG_FAST 0     /* the quadratic algorithm (Alg. 1, "Fast PIMD-B"); default */
#define PIMDB_ALG_ORIGINAL 1 /* the original cubic algorithm (appendix "Algorithm Pseudocode", the
                                original method; Background): a comparison path, FP64 only */
/* shift of the forward recurrence's exponential sums under PIMDB_ALG_ORIGINAL
 * (appendix "Numerical Stability"; any shift is exact in exact arithmetic) */
#define PIMDB_SHIFT_MIN 0      /* the smallest exponent of each sum (largest term 1); default */
#define PIMDB_SHIFT_TWO_TERM 1 /* the smaller of E^[1,v] and V^[1,v-1] + E^[v,v]: overflows
                                  (PIMDB_STATUS_NONFINITE_OUTPUT) once another term lies more than
                                  about 709/beta below both */

/* ---- device status bits (pimdb_status) ---- */
#define PIMDB_STATUS_NONFINITE_INPUT 1  /* a position was NaN or infinite */
#define PIMDB_STATUS_NONFINITE_OUTPUT 2 /* an energy or force came out NaN or infinite */
#define PIMDB_STATUS_RANGE 4            /* out of range, results invalid: a spring exponent
                                           beta*k*|d|^2*log2(e) above 2^28, or a recursion value
                                           whose binary exponent passed +-2^29 (the chain's
                                           cumulative spring exponents, e.g. particles with
                                           consecutive labels thousands of length units apart) */
#define PIMDB_STATUS_TIMEOUT 16         /* a workgroup of a split recursion waited more than 2 s
                                           for another (results invalid) */
#define PIMDB_STATUS_PRECISION 8        /* PIMDB_FP64 on an open system whose extent passes the
                                           expansion's rounding bound: beta*k*log2(e)*max|r - r_0^1|^2
                                           above 2^23 (about 600 length units at beta k = 16).
                                           Results are finite but may miss 1e-10 relative; use
                                           PIMDB_FP64_DIRECT */

/* ---- what pimdb_debug_get exports ---- */
#define PIMDB_DEBUG_PROBABILITIES 1 /* dense N x N per system, [l-1][l'-1] = Pr[l -> l'] */
#define PIMDB_DEBUG_CYCLE_ENERGIES 2 /* dense N x N per system, [u-1][v-1] = E^[u,v] for u <= v, 0 below */
#define PIMDB_DEBUG_FORWARD 3        /* N+1 per system: V^[1,v], v = 0..N */
#define PIMDB_DEBUG_BACKWARD 4       /* N+2 per system: index u holds V^[u,N] for u = 1..N+1; index 0 is 0 */

#define PIMDB_MAX_N 4096
#define PIMDB_MAX_BATCH 65536
/* size of the device-resident scratch of pimdb_exchange_forces_static (16 MiB) */
#define PIMDB_STATIC_SCRATCH_BYTES 16777216

typedef struct pimdb_ctx *pimdb_t;

/* ------------------------------------------------------------ handle */

/* Create a handle on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t passed as void*; NULL = the null stream).  The caller's
 * current device is restored on return.  The handle starts with no system,
 * FP64 precision, open boundaries and no trap.  *out is set to NULL on
 * failure.  Returns PIMDB_EINVAL for a null out or a device index out of
 * range, PIMDB_EDEVICE when no device can be used.  Also sets up, once per
 * device, the scratch of pimdb_exchange_forces_static. */
int pimdb_create(pimdb_t *out, int device, void *stream);

/* Free the handle and the tables it owns (waits for its stream first).
 * NULL is accepted. */
int pimdb_destroy(pimdb_t h);

/* Change the stream on which later calls are enqueued (follows the caller's
 * current stream, e.g. during graph capture).  Never fails for a valid h. */
int pimdb_set_stream(pimdb_t h, void *stream);

/* ------------------------------------------------------ system set-up */

/* One system of N >= 1 particles with P >= 2 beads, inverse temperature
 * beta > 0, particle mass m > 0 and ring-polymer frequency omega_P > 0
 * (Background: the bead springs of frequency omega_P with prefactor
 * (1/2) m omega_P^2; P >= 2 because the exterior-bead forces of Theory,
 * "Force on exterior beads", need distinct beads 1 and P).  Equivalent to
 * pimdb_set_batch with S = 1.  PIMDB_EINVAL for arguments outside those
 * ranges, PIMDB_ERANGE for N > PIMDB_MAX_N.  Unbinds the workspace: query
 * pimdb_workspace_bytes and bind again before evaluating. */
int pimdb_set_system(pimdb_t h, int64_t N, int32_t P, double beta, double m, double omega_P);

/* A batch of S independent systems (host arrays of length S; each entry as
 * in pimdb_set_system).  One evaluation call processes the whole batch in
 * two kernel launches (springs and recursions of every system, then
 * exterior forces and energies); the first launch puts the largest systems
 * first.  PIMDB_EINVAL / PIMDB_ERANGE as pimdb_set_system, and PIMDB_ERANGE
 * for S > PIMDB_MAX_BATCH.  Unbinds the workspace.  On error the handle is
 * left with no system set. */
int pimdb_set_batch(pimdb_t h, int32_t S, const int64_t *N, const int32_t *P, const double *beta,
                    const double *m, const double *omega_P);

/* Cubic periodic box of side L applied to every spring displacement as the
 * minimum image d - L*rint(d/L), round half to even (Methods, "Simulation
 * details", states periodic boundaries; the per-spring minimum image is this
 * library's reading).  L = 0 (default): open boundaries.  PIMDB_EINVAL for
 * L < 0 or non-finite L. */
int pimdb_set_box(pimdb_t h, double L);

/* Harmonic external trap of angular frequency w >= 0 (0 = none, default):
 * energies include the scaled potential U-bar = (1/P) sum_j sum_l
 * (1/2) m w^2 |r_l^j|^2 of the Background section and forces include
 * -(m w^2 / P) r_l^j on every bead.  PIMDB_EINVAL for w < 0 or non-finite. */
int pimdb_set_trap(pimdb_t h, double w);

/* PIMDB_FP64 (default), PIMDB_MIXED or PIMDB_FP64_DIRECT; PIMDB_EINVAL
 * otherwise.  Takes effect at the next evaluation call. */
int pimdb_set_precision(pimdb_t h, int mode);

/* Scaled pair interaction (Theory, the bosonic partition function, where
 * each imaginary-time slice's interaction enters scaled by 1/P):
 *   U-bar = (1/P) sum_{j=1}^{P} sum_{a<b} U(|r_a^j - r_b^j|),
 * with the caller's Gaussian U(r) = g exp(-r^2 / (2 sigma^2)) (the form of
 * a Gaussian repulsion; g and sigma are the caller's, no parameter of the
 * paper's systems is assumed), minimum image in a periodic box.  Once set
 * (g != 0), every evaluation that writes forces or energies adds
 * -grad U-bar and U-bar to them: pimdb_exchange_forces, _energy, _batched,
 * _static, _energy_save, _adjoint (its gradient), pimdb_md_step and
 * pimdb_distinguishable_forces, under either algorithm.  O(P N^2) pair
 * terms per system, in FP64 whatever the precision mode.  g = 0 (default)
 * removes it.  With a system set this rebuilds the tables and unbinds the
 * workspace like pimdb_set_batch (the workspace grows by one double per
 * pair workgroup).  PIMDB_EINVAL for non-finite g, or sigma <= 0 or
 * non-finite with g != 0. */
int pimdb_set_pair_gaussian(pimdb_t h, double g, double sigma);

/* The pair interaction alone: forces = -grad U-bar (P,3,N layout, may be
 * NULL) and energies = U-bar (may be NULL), overwritten.  Asynchronous like
 * the evaluations.  PIMDB_EINVAL when no pair interaction is set or both
 * outputs are NULL. */
int pimdb_pair_forces(pimdb_t h, const double *pos, double *forces, double *energy);

/* Select the algorithm of pimdb_exchange_forces, pimdb_exchange_energy and
 * pimdb_md_step.  PIMDB_ALG_ORIGINAL evaluates the original method of the
 * appendix "Algorithm Pseudocode" (Background, "cubic scaling bosonic
 * PIMD"): cycle energies from their defining sum, the forward recurrence
 * with the chosen shift, and the forces from the derivative of that
 * recurrence evaluated for every bead coordinate, O(P N^3) time and
 * O(P N^2) workspace doubles per system (about 0.8 GB at N = 1024, P = 32);
 * it always computes in FP64 (the precision mode is ignored), honours the
 * box and the trap, and gives the same potential and forces as
 * PIMDB_ALG_FAST to rounding.  shift must be PIMDB_SHIFT_MIN with
 * PIMDB_ALG_FAST.  With a system set, this rebuilds the tables and unbinds
 * the workspace like pimdb_set_batch.  Under PIMDB_ALG_ORIGINAL the batched,
 * static-scratch, energy-save and adjoint entries return PIMDB_EINVAL, and
 * pimdb_debug_get still exports the quadratic algorithm's tables.
 * PIMDB_EINVAL for unknown values. */
int pimdb_set_algorithm(pimdb_t h, int algorithm, int shift);
/* The current algorithm and shift. */
int pimdb_get_algorithm(pimdb_t h, int *algorithm, int *shift);

/* Launch shape override: threads per workgroup (64, 128, 256, 512 or 1024)
 * and particles owned per thread in the recursions (1, 2, 4 or 8; 4 and 8 need
 * threads <= 512).  Both 0 restores the built-in choice.  PIMDB_EINVAL if the
 * pair cannot hold the largest system (threads * per_thread < N_max).  With
 * a system set, this rebuilds the tables and unbinds the workspace like
 * pimdb_set_batch; graphs captured before keep working (the replaced tables
 * stay allocated until pimdb_destroy) as long as their workspace does. */
int pimdb_set_tuning(pimdb_t h, int threads, int per_thread);

/* Timing mode (enable = 1; 0 turns it off): every later evaluation that is
 * not being captured into a graph records HIP events on the handle's stream
 * before and after the exchange launch and after the finalize launch.
 * Creates the events on first use.  For measurement, not for graphs. */
int pimdb_set_timing(pimdb_t h, int enable);

/* Durations in ms of the two launches of the last timed evaluation
 * (waits for it): the fused exchange launch (springs and recursions) and
 * the finalize launch (exterior forces and energies).  PIMDB_ENOSYS if no
 * evaluation has been timed since timing was enabled. */
int pimdb_last_timing(pimdb_t h, float *exchange_ms, float *finalize_ms);

/* Split recursions: spread each system's forward and backward recursion
 * over 1 + nhelp workgroups on different CUs, so that small batches use the
 * device (the serial chain of steps stays in one workgroup; helper
 * workgroups add the terms of published blocks to the accumulators they own
 * and deliver them to the chain; the accumulators follow the terms of the
 * recurrences of Background and Theory, "Connection probabilities").
 * blocks_per_helper: -1 automatic (default: split when the batch has fewer
 * recursion workgroups than a quarter of the CUs), 0 never, g >= 1 at most g
 * blocks of 64 accumulators per helper.  Systems of N <= 128 are never split
 * (N <= 192 when every workgroup of the launch has a CU of its own).
 * Results equal those of the whole recursions up to rounding.  PIMDB_EINVAL
 * if the plan would not fit the workgroups the device holds at once.  With a
 * system set, rebuilds the tables and unbinds the workspace. */
int pimdb_set_split(pimdb_t h, int blocks_per_helper);

/* Blocks per helper of the current tables (0: no system split), the number
 * of helper workgroups a forces call launches, and (cu_per_workgroup, may be
 * NULL) 1 if a split launch gives every workgroup a CU of its own (small
 * plans), 0 if two share a CU. */
int pimdb_get_split(pimdb_t h, int *blocks_per_helper, int *helpers, int *cu_per_workgroup);

/* Current launch shape (after the automatic choice). */
int pimdb_get_tuning(pimdb_t h, int *threads, int *per_thread);

/* Element offset of system s in packed position/force arrays; -1 if s is out
 * of range or no system is set. */
int64_t pimdb_system_offset(pimdb_t h, int32_t s);

/* Total elements (sum 3 P_s N_s) of a packed position array; 0 if unset. */
int64_t pimdb_total_elements(pimdb_t h);

/* Device scratch bytes the evaluation calls need for the current batch
 * (about 80 N bytes per system; nothing O(N^2) is ever stored). */
size_t pimdb_workspace_bytes(pimdb_t h);

/* Bind caller-owned device memory (at least pimdb_workspace_bytes, 256-byte
 * aligned) as scratch.  The library clears its status word with a kernel
 * on the handle's stream.  The memory must stay allocated while bound.
 * PIMDB_EINVAL for a null or misaligned pointer, PIMDB_EWORKSPACE if too
 * small. */
int pimdb_bind_workspace(pimdb_t h, void *dev_ptr, size_t bytes);

/* --------------------------------------------------------- evaluation
 * Common to the evaluation calls: device pointers in the layout above;
 * asynchronous on the handle's stream; PIMDB_ENOSYS without a system,
 * PIMDB_EWORKSPACE without a large enough bound workspace, PIMDB_EINVAL for
 * null or aliasing pointers, PIMDB_EDEVICE if a launch fails.  Non-finite
 * or out-of-range data are reported through pimdb_status. */

/* V^[1,N] of every system -> energy[s]: the interior spring energies and the
 * forward recurrence exp(-beta V^[1,v]) = (1/v) sum_{k=1}^{v}
 * exp(-beta (V^[1,v-k] + E^[v-k+1,v])), V^[1,0] = 0 (Background, the
 * recurrence that defines the potential), with the cycle energies E^[u,v]
 * of Theory, "Reducing the potential to O(N^2 + PN)".  energy: S doubles. */
int pimdb_exchange_energy(pimdb_t h, const double *pos, double *energy);

/* Energies (energy may be NULL) and forces -grad V^[1,N] (plus trap terms if
 * set) on all beads of all systems: interior beads by Theory, "Force on
 * interior beads"; beads 1 and P by the probability-weighted sums of Theory,
 * "Force on exterior beads", with the backward potentials V^[u,N] of Theory,
 * "Connection probabilities", the direct-link probability given there and
 * the cycle-closing probabilities of Methods, "Expressions for connection
 * probabilities" (the whole of Alg. 1 in the appendix).  forces: same
 * layout as pos, overwritten.  One kernel launch runs the interior springs
 * and both recursions of every system concurrently, a second one the
 * exterior-bead forces and energies. */
int pimdb_exchange_forces(pimdb_t h, const double *pos, double *forces, double *energy);

/* pimdb_exchange_forces for systems packed at caller-chosen places:
 * offsets_dev is a device array of S int64 element offsets, system s
 * occupying 3 P_s N_s elements (bead-major (P, 3, N)) from offsets_dev[s] in
 * both pos_packed and forces_packed; energies: S doubles.  The offsets are
 * read on the device and honoured as given: the caller guarantees that every
 * system lies inside its buffers and that systems do not overlap in
 * forces_packed.  A negative offset skips that system and sets
 * PIMDB_STATUS_RANGE.  Same passages as pimdb_exchange_forces. */
int pimdb_exchange_forces_batched(pimdb_t h, const double *pos_packed, const int64_t *offsets_dev,
                                  double *forces_packed, double *energies);

/* pimdb_exchange_forces without a caller workspace, for callers that cannot
 * allocate (code under HIP graph capture that must not call hipMalloc, tight
 * serving loops, harnesses that forbid allocation).  Same results, layout and
 * asynchrony as pimdb_exchange_forces; its scratch is a library-owned device
 * array of PIMDB_STATIC_SCRATCH_BYTES (one per device, held until the process
 * ends), so no workspace needs to be bound and nothing is allocated.
 * Returns PIMDB_ERANGE when the batch needs more scratch than that
 * (pimdb_workspace_bytes > PIMDB_STATIC_SCRATCH_BYTES), PIMDB_EDEVICE if the
 * scratch could not be set up at pimdb_create.  Every call on one device
 * shares that device's scratch (it keeps the last call's contents): calls
 * that overlap in time on one device, from any handle or stream, race.
 * pimdb_status after such a call reads the scratch's status word. */
int pimdb_exchange_forces_static(pimdb_t h, const double *pos, double *forces, double *energy);

/* Bytes of the adjoint state written by pimdb_exchange_energy_save. */
size_t pimdb_state_bytes(pimdb_t h);

/* Forward half for reverse-mode differentiation: energies -> energy[s] (as
 * pimdb_exchange_energy), and the forward potentials V^[1,v] plus the
 * forward-weighted endpoint displacements -> state (caller-owned device
 * buffer of pimdb_state_bytes), which the reverse half needs for the
 * exterior-bead forces. */
int pimdb_exchange_energy_save(pimdb_t h, const double *pos, double *energy, void *state);

/* Reverse half (the adjoint): grad_pos = grad_energy[s] * dV_s/dpos for every
 * system s, from the positions and a state written by
 * pimdb_exchange_energy_save on the same positions.  grad_energy is a device
 * array of S doubles.  It runs the backward recursion (Theory, "Connection
 * probabilities"), the connection probabilities and the interior and
 * exterior bead forces of Theory, "Reducing the force to O(N^2 + PN)",
 * scaled by -grad_energy[s]. */
int pimdb_exchange_adjoint(pimdb_t h, const double *pos, const void *state, const double *grad_energy,
                           double *grad_pos);

/* Velocity-Verlet step for every bead of every system (bead mass m_s; the
 * time step of the paper's runs is in Methods, "Simulation details"):
 *   vel += dt/(2 m) forces; pos += dt vel; forces, energy <- pimdb_exchange_forces(pos);
 *   vel += dt/(2 m) forces.
 * forces must hold the forces of the incoming positions.  Asynchronous and
 * graph-capturable like pimdb_exchange_forces.  energy may be NULL.
 * PIMDB_EINVAL for null pointers or a non-finite dt. */
int pimdb_md_step(pimdb_t h, double *pos, double *vel, double *forces, double *energy, double dt);

/* Forces and energies of distinguishable particles (each particle its own
 * closed ring; no exchange), the ordinary PIMD that the paper's "Benchmarks &
 * Applications" compares bosonic PIMD with; same layout and trap/box
 * settings. */
int pimdb_distinguishable_forces(pimdb_t h, const double *pos, double *forces, double *energy);

/* ------------------------------------------------------------ exports */

/* Synchronous export of intermediates for system s (see PIMDB_DEBUG_*) into
 * device memory dst, recomputed from pos: cycle energies E^[u,v] (Theory,
 * "Reducing the potential"), V^[1,v] (Background recurrence), V^[u,N] and
 * Pr[l -> l'] (Theory, "Connection probabilities"; Methods, "Expressions for
 * connection probabilities").  For tests and analysis; allocates nothing
 * but synchronises the stream.  PIMDB_EINVAL for s out of range or an
 * unknown `what`. */
int pimdb_debug_get(pimdb_t h, const double *pos, int32_t s, int what, double *dst);

/* Endpoint springs s(v,u) = k |r_v^P - r_u^1|^2 of system s (the closing
 * spring of the cycle energy E^[u,v], Theory, "Reducing the potential"),
 * packed lower triangle row by row (row v = 1..N holds u = 1..v; entry (v,u)
 * at index v(v-1)/2 + u-1), FP64 (as_float = 0) or FP32 (as_float = 1,
 * compensated), into device memory dst.  Asynchronous.  This is the
 * pairwise part the exchange kernels evaluate in registers without storing
 * it. */
int pimdb_endpoint_springs(pimdb_t h, const double *pos, int32_t s, int as_float, void *dst);

/* Synchronise the stream, read and clear the device status word of the
 * workspace the last evaluation used.  *flags (may be NULL) receives the
 * PIMDB_STATUS_* bits.  Returns PIMDB_ENONFINITE if any bit was set,
 * PIMDB_OK otherwise, PIMDB_EWORKSPACE if no workspace was ever used. */
int pimdb_status(pimdb_t h, int32_t *flags);

/* Static text for a return code. */
const char *pimdb_strerror(int code);

/* Text of the last error recorded on the handle (HIP error string or the
 * argument that was rejected); "" if none.  Valid until the next call. */
const char *pimdb_last_error(pimdb_t h);

#ifdef __cplusplus
}
#endif

#endif /* PIMDB_H */
