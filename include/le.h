/*
 * le.h -- C ABI of the MI355X Lees-Edwards shear-flow MD hot path.
 *
 * Method: Xu, Vance, Tretyakov, Stuehn, Brinkmann, "Implementation and
 * Parallel Optimization of the Lees-Edwards Boundary Condition in
 * ESPResSo++", arXiv 2109.11083.  One call advances a sheared periodic box
 * of N particles: Lees-Edwards cell build (Section 2.3, Fig. decomp),
 * LJ/WCA pair forces (Eqs. lj, lj-shift) and Kremer-Grest FENE bonds
 * (Eq. fene) with an optional cosine angle term (Eq. angle), velocity
 * Verlet with the boundary crossing of Eq. pos_new, a Langevin force on the
 * peculiar velocity (Eqs. vi, langevin) or the paper's alternatives (DPD,
 * Eqs. dissipative, random, omega; friction on the lab velocity) driven by
 * counter-based Philox4x32-10 noise, and the Irving-Kirkwood stress that
 * yields the viscosity (Eqs. tensor, viscosity), with profiles and mean
 * squared displacements (Figs. profile, msd).
 *
 * Axes: x is the flow direction, y the gradient direction (the paper's z),
 * z the vorticity direction.  The periodic image directly above the box
 * (y + L_y) is displaced by +Delta along x, Delta = shear_rate * L_y * t
 * reduced into [0, L_x); a particle leaving through y = L_y re-enters at
 * y - L_y with x - Delta and lab velocity u_x - shear_rate * L_y.
 *
 * Units are reduced (epsilon = sigma = m = k_B = 1 in the paper's runs).
 *
 * Memory and ownership
 *   - Every array argument is a DEVICE pointer unless stated otherwise.
 *   - Particle arrays at the ABI are float64 structure-of-arrays [3][n]
 *     (all x, then all y, then all z), indexed by particle tag 0..n-1.
 *   - The caller owns all device memory, including ONE workspace buffer of at
 *     least le_workspace_bytes() bytes, which must stay allocated and
 *     untouched until le_destroy().  The library never calls hipMalloc or
 *     hipFree; it allocates only its small host-side handle.
 *   - Inputs given to le_init() are copied; the caller may free them after.
 *
 * Streams and synchronisation
 *   - All work is enqueued on the hipStream_t passed to le_init() and is
 *     asynchronous, except le_build_cells() (it returns a pair count to the
 *     host), le_get_state() and le_sync(), which wait for the stream.
 *
 * Errors
 *   - Invalid arguments, geometry and workspace size are reported
 *     synchronously by the call that receives them.
 *   - Errors found on the device (a FENE bond stretched to r >= R0, a
 *     non-finite coordinate, a neighbour-list or cell overflow) are latched
 *     in a status word inside the workspace.  Every later kernel of that
 *     simulation becomes a no-op, and the next synchronising call returns
 *     the status.  le_step() returns a latched status once a synchronising
 *     call has seen it.  Only le_destroy() and a new le_init() clear it.
 *   - No call throws; le_strerror() maps a status to a static string.
 *
 * Calls on one le_sim are not thread-safe; distinct le_sim handles are
 * independent (they may share a stream).
 */
#ifndef LE_H
#define LE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct le_sim le_sim;
typedef struct le_graph le_graph;
typedef int32_t le_status;

#define LE_OK 0
#define LE_E_ARG (-1)       /* bad argument (null pointer, n < 2, dt <= 0, ...)    */
#define LE_E_GEOMETRY (-2)  /* box too small: L_a <= 2 r_list or < 3 cells on an axis */
#define LE_E_WORKSPACE (-3) /* workspace smaller than le_workspace_bytes()          */
#define LE_E_BOND (-4)      /* FENE bond reached r >= R0 (Eq. fene: V = +infinity)  */
#define LE_E_NONFINITE (-5) /* NaN or Inf in positions or velocities                */
#define LE_E_CAPACITY (-6)  /* neighbour list or cell occupancy over capacity       */
#define LE_E_HIP (-7)       /* a HIP runtime call failed                            */
#define LE_E_STATE (-8)     /* call not valid in the current state                  */

#define LE_PAIR_LJ 0  /* 4 eps[(s/r)^12 - (s/r)^6], force truncated at rc (Eq. lj) */
#define LE_PAIR_WCA 1 /* the same force with rc = 2^(1/6) s (Eq. lj-shift)         */

#define LE_FP64 0  /* every operation in float64                                    */
#define LE_MIXED 1 /* pair-force arithmetic in float32 after a float64 cutoff test;
                      positions, offset, bonds, sums and integrator in float64      */

/* Thermostats (Section 2.2).  theta is uniform on (-1/2, 1/2) from Philox4x32-10. */
#define LE_THERMO_LANGEVIN 0 /* Eq. langevin on the peculiar velocity c = u - gamma_dot (y - L_y/2) e_x:
                                F_i += -gamma m c_i + sqrt(24 gamma m kT / dt) theta_i          */
#define LE_THERMO_DPD 1      /* Eqs. dissipative, random, omega, pairwise for r < dpd_rc with
                                e = r_ij / r, v_ij = u_i - u_j minus the streaming velocity of
                                j's image (s_y gamma_dot L_y e_x), w = 1 - r / dpd_rc:
                                F_i += [-gamma w^2 (e . v_ij) + sqrt(24 gamma kT / dt) w theta_ij] e,
                                F_j -= the same; theta_ij shared by the pair.  Conserves momentum.
                                Requires the global-memory pair layout (tune 0 or 2).           */
#define LE_THERMO_LANGEVIN_LAB 2 /* Eq. langevin with the friction on the lab velocity u (the
                                paper's xi_abs, Section 3.1): F_i += -gamma m u_i + noise       */

/* Velocity storage (Section 2.2, Eq. vi).  The velocity arrays given to
 * le_init and returned by le_get_state are the stored velocities.          */
#define LE_VEL_LAB 0      /* u is the lab velocity; a particle crossing a sheared face has its
                             u_x changed by -/+ gamma_dot L_y; x moves with u              */
#define LE_VEL_PECULIAR 1 /* u is the peculiar velocity c of Eq. vi (continuous across the
                             faces); x moves with c_x + gamma_dot (y - L_y/2), the streaming
                             velocity of its height.  Drops the -gamma_dot c_y coupling of the
                             lab form (a different dynamics, as integrated in ESPResSo++).
                             Requires LE_THERMO_LANGEVIN (friction on c).                  */

/* Parameters of one simulation (Sections 2.1, 2.2, 2.4).  All 8-byte fields
 * come first so that the layout has no padding. */
typedef struct le_params {
  int64_t n;           /* number of particles (2 .. 16,777,214)                    */
  double box[3];       /* L_x, L_y, L_z                                             */
  double shear_rate;   /* gamma_dot of Eq. shear-rate (any sign; 0 = equilibrium)   */
  double dt;           /* time step (> 0)                                           */
  double kT;           /* thermostat temperature (>= 0)                             */
  double gamma;        /* Langevin friction xi of Eq. langevin (>= 0; 0 = NVE)      */
  double mass;         /* particle mass (> 0)                                       */
  double eps, sigma;   /* pair parameters                                           */
  double rc;           /* pair cutoff; pairs interact iff r < rc                    */
  double skin;         /* Verlet skin (>= 0); 0 rebuilds and wraps every step       */
  double fene_k;       /* FENE spring constant k                                    */
  double fene_r0;      /* FENE maximal bond length R0                               */
  double dpd_rc;       /* cutoff r_c of the DPD weight omega (Eq. omega); 0 = rc;
                          must not exceed rc (the pair list covers rc only)      */
  double force_cap;    /* > 0: every LJ/WCA pair force is capped in magnitude,
                          |F_ij| <= force_cap (direction kept; bonds and angles
                          uncapped).  For the warm-up of overlapping starts (a
                          random-walk melt) before the equilibration that precedes
                          shear (Section 2.4); 0 = the plain force law.  Requires
                          LE_FP64, not LE_THERMO_DPD; uses the global pair layout. */
  double angle_k;      /* cosine angle term of the chains (Eq. angle), read as
                          V = angle_k (1 + cos theta) per consecutive bead triple,
                          theta the angle at the middle bead (minimum at 180
                          degrees; the paper's KG melts use 1.5); 0 = none, >= 0   */
  int64_t n_chains;    /* linear chains: tag = chain*chain_len + k; 0 = no bonds    */
  uint64_t seed;       /* Philox key of the thermostat noise                        */
  int32_t chain_len;   /* beads per chain (0 = no bonds)                            */
  int32_t pair;        /* LE_PAIR_LJ or LE_PAIR_WCA                                 */
  int32_t precision;   /* LE_FP64 or LE_MIXED                                       */
  int32_t cells[3];    /* cell grid; 0 = floor(L_a / (rc + skin)); each must be >= 3 */
  int32_t max_neighbors; /* neighbour-list capacity per particle (two sub-lists of half
                            each; the first also takes the second's partial last block
                            of up to 7 entries); 0 = from density */
  int32_t tune;        /* pair-kernel layout: 0 = chosen from density, 1 = partners staged
                          in an LDS halo per tile, 2 = partners read from global memory;
                          the physics is the same (sums may differ in the last bits) */
  int32_t thermostat;  /* LE_THERMO_*: how gamma and kT act (Section 2.2)                */
  int32_t velocity;    /* LE_VEL_*: what the stored (and exchanged) velocities are       */
} le_params;

/* Device bytes needed for a simulation with these parameters.  Pure host
 * function; validates the parameters (same errors as le_init). */
le_status le_workspace_bytes(const le_params* p, size_t* bytes);

/* Create a simulation from the state (x0, u0) at step index step0.
 * x0, u0: device float64 [3][n] by tag; positions may lie outside the box
 * (they are wrapped with the offset of step0, Eq. pos_new), u0 are lab-frame
 * velocities.  f0: NULL, or the device float64 [3][n] total force of step
 * step0 as returned by le_get_state (exact restart); when NULL the force of
 * step0 (conservative + thermostat with the noise of step0, evaluated at u0) is
 * computed here.  workspace: device buffer of ws_bytes >=
 * le_workspace_bytes(p).  hip_stream: a hipStream_t (NULL = the null
 * stream).  *out receives the handle. */
le_status le_init(const le_params* p, const double* x0, const double* u0, const double* f0,
                  void* workspace, size_t ws_bytes, void* hip_stream, int64_t step0, le_sim** out);

/* Rebuild now: apply the boundary crossing and periodic wrap to the current
 * state, re-bin the particles into cells (Section 2.3: ids
 * (iz*ny + iy)*nx + ix, order ascending (cell, tag)), recompute the
 * Lees-Edwards cell stencil (neighbour rows across the gradient faces offset
 * by Delta, Fig. decomp) and the neighbour lists of radius rc + skin.
 * Optional device outputs (NULL to skip):
 *   cell_of[n]  int32 cell id of each tag;
 *   order[n]    int32 tag at each cell-sorted slot;
 *   pairs       int64 [pairs_cap][2]: every unordered pair (tag_i < tag_j)
 *               with r < rc + skin, in unspecified order; *n_pairs (host)
 *               receives the total count even when it exceeds pairs_cap.
 * Synchronous when n_pairs is given. */
le_status le_build_cells(le_sim* s, int32_t* cell_of, int32_t* order, int64_t* pairs,
                         int64_t pairs_cap, int64_t* n_pairs);

/* Conservative forces of the current state (Eqs. lj/lj-shift + fene).
 * f_out: device float64 [3][n] by tag (may be NULL); virial6: device
 * float64[6] receiving W_ab = sum over pairs i<j of d_a F_ij,b in the order
 * xx, yy, zz, xy, xz, yz (may be NULL).  Does not change the state. */
le_status le_forces(le_sim* s, double* f_out, double* virial6);

/* Advance nsteps velocity-Verlet steps (Section 2.2).  When sample_every > 0,
 * the stress tensor (see le_stress) of every sample_every-th new state is
 * written to stress_ring[(k mod ring_cap)][6], k = 0, 1, ... counted within
 * this call; stress_ring is a device float64 buffer of ring_cap*6 values. */
le_status le_step(le_sim* s, int64_t nsteps, int32_t sample_every, double* stress_ring,
                  int64_t ring_cap);

/* Batched stepping (the same velocity-Verlet steps as le_step, Section 2.2,
 * for many independent simulations at once): advances every simulation of
 * sims[0..nsims) by nsteps.  Each kernel of a step is launched once for all
 * members of one kernel configuration (precision, pair layout, bonds,
 * thermostat kind), its grid covering the blocks of every member, so the
 * launch count per step does not grow with nsims; members may differ in N,
 * box, shear rate, skin, seed and every other parameter.  Each member's
 * arithmetic is exactly that of le_step on it alone, so its results are
 * bitwise the same alone and in any batch.
 *   All members must share one stream (the one given to their le_init);
 *   a null, repeated or foreign-stream entry is LE_E_ARG.
 *   sample_every > 0: the stress tensor of every sample_every-th new state of
 *   member k goes to stress_rings[k][(j mod ring_cap)][6], j counted within
 *   this call (stress_rings: host array of nsims device pointers).
 *   A member with a latched error (seen by a synchronising call) is skipped;
 *   one that latches during the call stops on the device, the others go on.
 *   Per-member errors are reported by le_sync on that member.  Asynchronous. */
le_status le_step_batch(le_sim* const* sims, int32_t nsims, int64_t nsteps, int32_t sample_every,
                        double* const* stress_rings, int64_t ring_cap);

/* Stress of the current state (Eq. tensor): sigma_ab = -(1/V)[sum_i m c_a c_b
 * + sum_{i<j} d_a F_ij,b] with peculiar velocities c (Eq. vi) and
 * conservative forces only; order xx, yy, zz, xy, xz, yz.  The viscosity of
 * Eq. viscosity is <sigma_xy> / shear_rate.  sigma6: device float64[6]. */
le_status le_stress(le_sim* s, double* sigma6);

/* Observables of the current state (Fig. profile; Section 3): per bin of
 * nbins equal bins along the gradient axis y, the particle count, the summed
 * lab flow velocity u_x and the summed peculiar kinetic term m c^2 (Eq. vi;
 * the temperature profile is sum_mc2 / (3 count)), each particle counted at
 * its image inside the box with the velocity of that image; then the kinetic
 * temperature sum_i m c_i^2 / (3n-3) and the centre-of-mass lab velocity of
 * the in-box images.
 * out: device float64[3*nbins + 4] = count[nbins], sum_ux[nbins],
 * sum_mc2[nbins], kT, com[3].
 * 1 <= nbins <= LE_MAX_BINS.  Sums are taken in a fixed order (reproducible).
 * Does not change the state. */
#define LE_MAX_BINS 256
le_status le_observables(le_sim* s, int32_t nbins, double* out);

/* Unwrapped gradient and vorticity coordinates (for the mean squared
 * displacement of Fig. msd): yz_out, device float64 [2][n] by tag, receives
 * y + k_y L_y and z + k_z L_z, where k counts the periodic wraps the library
 * has applied to the particle since le_init (the coordinates given to
 * le_init are the origin, so a run restarted from le_get_state counts from
 * the wrapped state).  The flow coordinate has no unwrapped form under the
 * sheared boundary and is not reported.  Does not change the state. */
le_status le_unwrapped(le_sim* s, double* yz_out);

/* Mean squared displacement along y and z relative to ref_yz (device float64
 * [2][n] by tag, from an earlier le_unwrapped of the same simulation):
 * out2 (device float64[2]) = mean over particles of (y - y_ref)^2 and of
 * (z - z_ref)^2 with unwrapped y, z.  Fixed summation order. */
le_status le_msd(le_sim* s, const double* ref_yz, double* out2);

/* Copy the current state out in tag order: positions x, lab velocities u and
 * the total force f of the current step (device float64 [3][n] each; any may
 * be NULL), and its step index (*step, host, may be NULL).  Pending boundary
 * crossings are applied first (a rebuild, which changes no physical
 * quantity), so the positions lie in the box; le_init(x, u, f, step) then
 * continues the run exactly.  Waits for the stream and returns any latched
 * device error. */
le_status le_get_state(le_sim* s, double* x, double* u, double* f, int64_t* step);

/* A HIP graph of le_step(s, nsteps, sample_every, stress_ring, ring_cap),
 * captured once on the simulation's stream so that a chunk of steps costs
 * one launch on the host.  nsteps must be even (each step alternates the
 * device control copy, so an even chunk ends on the copy it started from).
 * Every launch advances nsteps steps exactly as that le_step call would and
 * writes its stress samples to the same ring rows.  Phase timing is off
 * inside the graph.  The graph is owned by the caller (le_graph_destroy) and
 * must not outlive the simulation.  LE_E_STATE if the simulation runs on the
 * legacy default stream (null), which cannot be captured. */
le_status le_graph_create(le_sim* s, int64_t nsteps, int32_t sample_every, double* stress_ring,
                          int64_t ring_cap, le_graph** out);

/* A HIP graph of le_step_batch(sims, nsims, nsteps, sample_every,
 * stress_rings, ring_cap), captured once on the members' common stream (one
 * host launch per chunk of steps for the whole batch).  nsteps must be even;
 * replays advance every member as that call would.  The graph is owned by
 * the caller (le_graph_destroy) and must not outlive any member.  LE_E_STATE
 * on the legacy default stream or when every member has a latched error. */
le_status le_batch_graph_create(le_sim* const* sims, int32_t nsims, int64_t nsteps, int32_t sample_every,
                                double* const* stress_rings, int64_t ring_cap, le_graph** out);

/* Enqueue one replay on the simulation's stream.  Eager calls may be mixed
 * with replays (e.g. le_get_state, odd le_step counts): the device control
 * state is first moved to the copy the graph reads when needed. */
le_status le_graph_launch(le_graph* g);

le_status le_graph_destroy(le_graph* g);

/* Enqueue a copy of the simulation's latched status (0 or an LE_E_* code) to
 * the device int32 *status_out, ordered after the work enqueued so far;
 * does not wait (a caller that tracks its stream with events reads it once
 * the event has completed). */
le_status le_status_out(le_sim* s, int32_t* status_out);

/* Wait for all enqueued work of the simulation; returns any latched error. */
le_status le_sync(le_sim* s);

/* Telemetry (host outputs, synchronous): neighbour-list rebuilds since
 * le_init and the largest neighbour count seen at the last rebuild. */
le_status le_stats(le_sim* s, int64_t* rebuilds, int32_t* max_neighbors);

/* Phase timing: le_step records a pair of HIP events on the simulation's
 * stream around each launch group of an enabled phase and accumulates the
 * elapsed device time per phase: 0 the fused force kernel (pair + bond
 * forces, thermostat and integrator) of plain steps, 1 the rebuild chain
 * (crossing/wrap, sort, stencil, neighbour lists; empty launches on steps
 * without a rebuild), 2 the first half-kick of a call, 3 sampled steps (the
 * force kernel with the virial, then the stress reduction).  enabled is a bit
 * mask over the phases (bit k: phase k; 0 switches timing off, 0xF times
 * all); bits 8..23 hold a stride s (0 means 1): only every s-th plain-step
 * force launch is timed, so the events barely perturb the run.  Enabling
 * resets the totals.  Creating events is the only host-side resource it
 * takes. */
le_status le_timing_enable(le_sim* s, int32_t enabled);

/* Totals since the last enable (waits for the stream): ms[4] elapsed device
 * milliseconds and launches[4] launch-group counts per phase (host arrays). */
le_status le_timing_read(le_sim* s, double* ms, int64_t* launches);

/* Release the handle.  The workspace is the caller's and is not touched. */
le_status le_destroy(le_sim* s);

/* Static description of a status code. */
const char* le_strerror(le_status st);

/* No-allocation variant of le_forces, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the conservative forces and pair virial of one
 * configuration, computed exactly as le_init(p, x, u, NULL, ..., step) followed
 * by le_forces() would (same kernels, same results), but with every
 * intermediate (sorted copies, cells, neighbour lists, block partials) in a
 * library-owned device array of 64 MiB per GPU instead of a caller workspace.
 * No handle is created and nothing is allocated, on the host or the device.
 *   p: as for le_init; le_workspace_bytes(p) must not exceed 64 MiB, else
 *      LE_E_WORKSPACE (about 30,000 LJ particles at density 0.84, rc 2.5).
 *   x: device float64 [3][n] by tag (wrapped with the offset of `step`).
 *   f_out: device float64 [3][n] by tag, or NULL; virial6: device float64[6]
 *      (W_ab as for le_forces), or NULL; at least one must be given.
 *   status_out: device int32, or NULL: receives 0 or the LE_E_* code latched
 *      on the device (bond, capacity, non-finite); when nonzero the outputs
 *      are not written.
 * Enqueued on hip_stream (a stream of the current device) and asynchronous.
 * Every call on a GPU uses that GPU's one array: calls that overlap on one
 * device (other streams, other host threads) race and give wrong results. */
le_status le_forces_static(const le_params* p, const double* x, double* f_out, double* virial6,
                           int32_t* status_out, int64_t step, void* hip_stream);

/* Lees-Edwards offsets Delta_k for k = step0 .. step0+count-1 as the device
 * computes them (Eq. pos_new; fmod of shear_rate*L_y*(k*dt) by L_x, folded
 * into [0, L_x)).  out: device float64[count].  Enqueued on hip_stream. */
le_status le_offsets(double shear_rate, double Lx, double Ly, double dt, int64_t step0,
                     int64_t count, double* out, void* hip_stream);

/* Philox4x32-10 blocks as the thermostat draws them: for each k, counter
 * ctr[4k..4k+3] and key key[2k..2k+1] (device uint32) give out[4k..4k+3]
 * (device uint32).  The Langevin thermostat of step s uses counter (s lo,
 * s hi, tag, 0) and key (seed lo, seed hi); word a maps to (r_a + 1/2) 2^-32
 * - 1/2.  The DPD pair noise of step s uses counter (s lo, s hi, smaller tag,
 * larger tag), key (seed lo, seed hi xor 0x44504421) and word 0. */
le_status le_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                    void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LE_H */
