/*
 * tmd.h - C ABI of the MI355X (gfx950) Lennard-Jones molecular-dynamics hot
 * path described in tinyMD (arXiv 2009.07400).
 *
 * The library advances a periodic cubic box of point particles under the
 * Lennard-Jones 12-6 pair force (Sec. 3.2, Eq. 2) using cell lists and a full
 * Verlet neighbor list built at cutoff + skin (Sec. 3.2, Fig. 1; full lists as
 * in the evaluation setup of Sec. 6), the force sum over each atom's list
 * (the compute_potential example of Sec. 4.2), and velocity-Verlet
 * integration of Newton's law (Sec. 3.2, Eq. 1) with the list rebuilt on a
 * fixed schedule (every 20 steps in Sec. 6).
 *
 * Conventions shared by every entry point
 *   - Floating point is IEEE double (FP64) throughout, as in the paper's runs.
 *   - Arrays exchanged with the caller are device pointers in structure-of-
 *     arrays form (x[N], y[N], z[N]) indexed by ORIGINAL atom id, whatever
 *     order the library keeps internally.
 *   - Streams: `tmd_stream` is a hipStream_t (NULL = legacy default stream).
 *     Every call that takes a stream only enqueues work on it and returns;
 *     pointers passed to such a call must stay valid until that work is done.
 *   - Memory: the library never allocates device memory.  The caller asks
 *     tmd_workspace_size(), allocates that many bytes (256-byte aligned) and
 *     binds them; all device state lives there.  The library never frees
 *     caller memory.
 *   - Errors: argument and call-order errors are returned synchronously.
 *     Conditions detected on the device (list overflow, non-finite state) set
 *     a device error word; tmd_sync() (and any later call that synchronises)
 *     returns them.  Once set, the word stays set until tmd_set_state().
 *   - No entry point is thread-safe on the same tmd_system.
 */
#ifndef TMD_H
#define TMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TMD_OK = 0,
    TMD_EINVAL = -1,        /* bad argument: NULL handle, N <= 0, non-finite or non-positive parameter */
    TMD_EBOX = -2,          /* cutoff + skin >= L/2: the minimum image is not unique */
    TMD_ESTATE = -3,        /* wrong call order (no workspace bound, no state set, ...) */
    TMD_ENBR_OVERFLOW = -4, /* an atom had more than max_neighbors list entries (deferred) */
    TMD_ENONFINITE = -5,    /* a position or force became NaN/Inf, e.g. coincident atoms (deferred) */
    TMD_EWORKSPACE = -6,    /* workspace too small or misaligned */
    TMD_EHIP = -7           /* a HIP runtime call failed; tmd_last_error() has the HIP message */
} tmd_status;

/* Force models (Sec. 3.2). */
enum {
    TMD_MODEL_LJ = 0,             /* Lennard-Jones 12-6 pair force, Eq. 2 */
    TMD_MODEL_SPRING_DASHPOT = 1  /* Spring-Dashpot contact of spheres, Eq. 3 */
};

/* Physical and algorithmic parameters.  epsilon is the depth of the LJ well,
 * sigma the distance at which the pair potential is zero (Sec. 3.2, Eq. 2);
 * cutoff and skin give the force cutoff and the list radius cutoff + skin
 * (Fig. 1 caption; 2.5 and 0.3 in Sec. 6); rebuild_every is the reneighboring
 * interval (20 in Sec. 6); max_neighbors the list capacity per atom.
 * model selects the force: TMD_MODEL_LJ (default), or
 * TMD_MODEL_SPRING_DASHPOT (Sec. 3.2, Eq. 3) for spheres of diameter sigma
 * with spring constant `stiffness` (K) and dissipation constant `damping`
 * (gamma): F_ij = [K (sigma - r) - gamma (u . v_ij)] u while r < sigma, u =
 * x_ij / r, v_ij = v_i - v_j; it needs cutoff >= sigma (the list radius is
 * cutoff + skin) and ignores epsilon.  In velocity Verlet its damping takes
 * the half-step velocities v_{k+1/2} at the force of step k + 1 (the
 * initial force takes the initial velocities). */
typedef struct {
    double epsilon;
    double sigma;
    double mass;
    double cutoff;
    double skin;
    double dt;
    int32_t rebuild_every;
    int32_t max_neighbors;
    double stiffness;  /* Spring-Dashpot K >= 0 */
    double damping;    /* Spring-Dashpot gamma >= 0 */
    int32_t model;     /* TMD_MODEL_* */
    int32_t reserved;  /* 0 */
} tmd_params;

typedef struct tmd_system tmd_system; /* opaque, library-owned host object */
typedef void *tmd_stream;             /* hipStream_t */

/* Read-only facts about a created system (host values). */
typedef struct {
    int64_t n_atoms;         /* all boxes together */
    int64_t n_padded;        /* row stride of the neighbor-major list */
    int32_t cells_per_axis;  /* floor(L / (cutoff + skin)) of box 0 */
    int32_t max_neighbors;
    int64_t n_cells;         /* cells of all boxes */
    size_t workspace_bytes;
    int64_t step;            /* time-step counter of the current state */
    int32_t n_boxes;
    int32_t n_blocks;        /* blocks of cells, one workgroup each */
    int32_t block_threads;   /* threads per force workgroup */
    int32_t lds_atoms;       /* atoms of a block neighborhood staged in LDS */
    int32_t block_edge;      /* cells per block edge (2 or 3) */
    int32_t block_parts;     /* workgroups per block (1, 2 or 4) */
    int32_t lanes_per_atom;  /* lanes sharing one atom's force sum (1, 2 or 4) */
    int32_t build_threads;   /* threads per list-build (and adjoint) workgroup */
    int32_t build_lanes;     /* lanes per atom in the list build (1 or 2) */
    int32_t graph_captures;  /* rebuild intervals captured as graphs (tmd_set_graphs) */
    int64_t graph_launches;  /* rebuild intervals run as graph launches */
    int32_t half_list;       /* 1: half lists inside blocks (tmd_set_half_list) */
    int32_t layout;          /* position layout (TMD_LAYOUT_*, tmd_set_layout) */
} tmd_info;

/* Kernel classes reported by tmd_get_timing(). */
enum {
    TMD_T_FORCE = 0, /* force sum (fused with the kicks and the drift when integrating) */
    TMD_T_NEIGHBOR,  /* neighbor-list build */
    TMD_T_BINNING,   /* cell count, scan, scatter, in-cell ordering and permutation */
    TMD_T_DRIFT,     /* stand-alone kick + drift (first step of an integrate call) */
    TMD_T_THERMO,    /* deterministic reductions of energy, virial and kinetic energy */
    TMD_T_COPY,      /* state load/unload between original and internal order */
    TMD_T_ADJOINT,   /* reverse kernel of the adjoint (Hessian-vector product, drift adjoint) */
    TMD_T_COUNT
};

/* Create a system of n_atoms atoms in a periodic cube of side box_length.
 * Host only; touches no GPU.  Returns TMD_EINVAL for a NULL pointer, n_atoms
 * <= 0 or > 7e8, a non-finite or non-positive epsilon, sigma, mass, cutoff,
 * dt, box_length, a negative skin, rebuild_every < 1 or max_neighbors outside
 * [1, 4096], an unknown model, and for the Spring-Dashpot model a negative or
 * non-finite stiffness or damping or cutoff < sigma; TMD_EBOX when cutoff +
 * skin >= box_length / 2.  On success *out owns a handle to release with
 * tmd_destroy(). */
tmd_status tmd_create(const tmd_params *params, int64_t n_atoms, double box_length, tmd_system **out);

/* Create one system holding n_boxes independent periodic cubes (replicas)
 * that every later call advances together, in the same kernel launches.
 * Box k has n_atoms[k] atoms, side box_lengths[k] and parameters params[k];
 * its atoms occupy the slots [sum_{m<k} n_atoms[m], ...) of every per-atom
 * array the caller exchanges (concatenated original order).  All boxes must
 * share rebuild_every and max_neighbors (TMD_EINVAL otherwise) and hold at
 * most 7e8 atoms together; every other check of tmd_create() applies per
 * box.  Outputs that are per system in
 * tmd_create() become per box (see tmd_compute_forces, tmd_integrate).
 * With n_boxes == 1 this is tmd_create(). */
tmd_status tmd_create_batch(int32_t n_boxes, const int64_t *n_atoms, const double *box_lengths,
                            const tmd_params *params, tmd_system **out);

/* Bytes of device workspace the system needs (host only). */
tmd_status tmd_workspace_size(const tmd_system *sys, size_t *bytes);

/* Bind caller-allocated device memory of at least tmd_workspace_size() bytes,
 * 256-byte aligned.  Borrowed until tmd_destroy() or the next bind; binding
 * discards any state.  TMD_EWORKSPACE if too small or misaligned. */
tmd_status tmd_bind_workspace(tmd_system *sys, void *dev_ptr, size_t bytes);

/* Load positions pos[3] (x, y, z) and velocities vel[3], each a device array
 * of n_atoms doubles in original atom order, and the step counter.  Positions
 * are wrapped once into [0, L) (Sec. 3.2, periodic boundaries).  Clears the
 * device error word and marks the neighbor list and forces stale.  The input
 * arrays are read on `stream` and may be reused once that work completes. */
tmd_status tmd_set_state(tmd_system *sys, const double *const pos[3], const double *const vel[3], int64_t step,
                         tmd_stream stream);

/* Distribute atoms over cells and build the full Verlet list of every atom:
 * all j != i in the 27 neighboring cells (deduplicated when fewer than three
 * cells per axis) with |x_ij|^2 < (cutoff + skin)^2 (Sec. 3.2, Fig. 1).  The
 * library reorders atoms by cell (count / scan / scatter, in-cell order by
 * original id) and stores the list neighbor-major (Sec. 4.2: the n-th
 * neighbors of consecutive atoms are contiguous).  Overflow of max_neighbors
 * is reported by tmd_sync() as TMD_ENBR_OVERFLOW. */
tmd_status tmd_build_neighbors(tmd_system *sys, tmd_stream stream);

/* Forces at the current positions from the current list:
 *   F_i = sum_{j in list(i), |x_ij|^2 < cutoff^2} f(s) x_ij,
 *   f(s) = 48 eps (sigma^6/s^3) (sigma^6/s^3 - 1/2) / s   (Sec. 3.2 Eq. 2; Sec. 4.2 listing)
 * f[3] (nullable) receives F in original order (device, n_atoms doubles each).
 * energy_virial (nullable, device, 2 doubles per box, box-major) receives
 *   U = 1/2 sum_i sum_j 4 eps [(sigma^6/s^3)^2 - sigma^6/s^3]  (unshifted) and
 *   W = 1/2 sum_i sum_j s f(s), summed in a fixed order (bitwise reproducible).
 * TMD_ESTATE if no list has been built since the last tmd_set_state(). */
tmd_status tmd_compute_forces(tmd_system *sys, double *const f[3], double *energy_virial, tmd_stream stream);

/* Advance n_steps velocity-Verlet steps (Sec. 3.2, Eq. 1):
 *   v += dt/(2m) F;  x += dt v;  wrap x into [0, L);
 *   if step % rebuild_every == 0: rebuild cells and list;
 *   F = F(x);  v += dt/(2m) F
 * where `step` is the absolute step counter (so the schedule survives split
 * calls).  Builds the list first if none is valid.  With thermo_every > 0,
 * thermo (device, nullable) receives, for every step k (1-based within the
 * call) that is a multiple of thermo_every, one row of 5 doubles
 * (KE, T, U, W, E) per box: thermo[((k / thermo_every - 1) * n_boxes + box) * 5
 * + q]; T = 2 KE / (3N - 3) with N the box's atoms (0 for N = 1), E = KE + U.
 * n_steps == 0 is a no-op. */
tmd_status tmd_integrate(tmd_system *sys, int32_t n_steps, int32_t thermo_every, double *thermo,
                         tmd_stream stream);

/* Copy the current state out in original atom order (pos[3], vel[3] device
 * arrays of n_atoms doubles; either may be NULL) and the step counter (host,
 * nullable). */
tmd_status tmd_get_state(const tmd_system *sys, double *const pos[3], double *const vel[3], int64_t *step,
                         tmd_stream stream);

/* Export the current list in original ids: counts[N] (device int32) and
 * ids[N * max_neighbors] (device int32, row i holds atom i's neighbors sorted
 * ascending, unused slots -1).  capacity is the length of ids in elements.
 * ids may be NULL to export the counts only (capacity is then ignored).
 * TMD_EINVAL if counts is NULL or capacity < N * max_neighbors; TMD_ESTATE
 * without a list. */
tmd_status tmd_get_neighbors(const tmd_system *sys, int32_t *counts, int32_t *ids, int64_t capacity,
                             tmd_stream stream);

/* Wait for the stream and return the deferred device status (TMD_OK,
 * TMD_ENBR_OVERFLOW, TMD_ENONFINITE, or TMD_EINVAL for a coordinate passed to
 * tmd_set_state() outside [-L, 2L)), or TMD_EHIP. */
tmd_status tmd_sync(tmd_system *sys, tmd_stream stream);

/* Host-side facts about the system. */
tmd_status tmd_get_info(const tmd_system *sys, tmd_info *info);

/* Work schedule of the block kernels.  No value changes the lists; only
 * lanes_per_atom changes positions, velocities or forces (in their last
 * bits: the force on an atom is then summed as interleaved parts), and
 * energy, virial and kinetic sums may differ in their last bits (their
 * summation order follows the workgroups).
 * block_edge: cells per edge of the blocks of cells that one workgroup owns
 * and whose neighborhood it stages in LDS, 2 or 3 (0 keeps the current
 * value; a new edge resets threads and lds_atoms to that edge's defaults).
 * block_parts: workgroups sharing one block, 1, 2 or 4, each taking a
 * contiguous share of the block's atoms and staging the whole neighborhood
 * (more workgroups for small systems; 0 keeps the current value; a new value
 * resets threads to its default).  lanes_per_atom: 1, 2 or 4 lanes of a
 * wavefront per atom in the force kernel, lane p taking the list's groups of
 * eight entries p, p + lanes_per_atom, ... (more parallelism for small
 * systems; 0 keeps the current value; a new value resets threads to its
 * default).  threads: threads per force workgroup, a multiple of 64 in
 * [64, 1024] (0 keeps the current value).  build_threads: threads per
 * workgroup of the kernels that take one lane per atom (the list build,
 * the adjoint's Hessian-vector product and tmd_get_neighbors), same range
 * (0 keeps the current value; a new edge, block_parts or build_lanes
 * resets it to its default).  build_lanes: 1 or 2 lanes per atom in the
 * list build, the two lanes testing alternate candidates (0 keeps the
 * current value); both write the same list.  lds_atoms: how many atoms of a block's neighborhood may be staged
 * in LDS, a multiple of 64 in [64, 4096] (0 keeps the current value; lowered
 * at the next state upload if the device's per-workgroup LDS cannot hold
 * twice that many 24-byte slots); blocks whose neighborhood holds more atoms
 * gather from global memory instead.  A new edge or capacity marks the list
 * stale (the next integrate rebuilds it; compute_forces needs
 * tmd_build_neighbors first).  TMD_EINVAL for other values. */
tmd_status tmd_set_schedule(tmd_system *sys, int32_t threads, int32_t lds_atoms, int32_t block_edge,
                            int32_t block_parts, int32_t lanes_per_atom, int32_t build_threads,
                            int32_t build_lanes);

/* Memory layouts of the device position buffers (the particle data
 * layouts of Sec. 4.2, which the paper specialises its kernels for). */
enum {
    TMD_LAYOUT_SOA = 0,   /* column-major: every atom's x, then every y, then every z */
    TMD_LAYOUT_AOS = 1,   /* row-major: x, y, z of each atom side by side */
    TMD_LAYOUT_AOSOA = 2  /* clustered: per 64 atoms (one wavefront) their 64 x, 64 y, 64 z */
};

/* Store the positions in `layout` (TMD_LAYOUT_*): binning, list build, force
 * and drift kernels then read and write them that way; the state seen
 * through tmd_set_state()/tmd_get_state() (original order, three arrays)
 * and every result are unchanged.  The current positions, if a state is
 * set, are converted on `stream`.  TMD_EINVAL for another value, and for a
 * layout other than TMD_LAYOUT_SOA with the Spring-Dashpot model; the
 * adjoint (tmd_adjoint_forward) needs TMD_LAYOUT_SOA (TMD_EINVAL
 * otherwise), and a change of layout between tmd_adjoint_forward and
 * tmd_adjoint_backward makes the backward pass return TMD_ESTATE.  The
 * list stays valid. */
tmd_status tmd_set_layout(tmd_system *sys, int32_t layout, tmd_stream stream);

/* Half neighbor lists with Newton's third law (Sec. 3.2: each pair stored
 * once, its force applied to both atoms; the half_nb variant of Sec. 4.2),
 * applied inside each block of cells: a pair of two atoms of one block is
 * listed once, by the atom staged first, and the force kernel adds the
 * partner's reaction to a sum in the workgroup's LDS; a pair whose atoms lie
 * in different blocks is listed by both atoms, each block computing only its
 * own atoms' forces (no workgroup writes another's atoms, no global
 * atomics).  Blocks whose neighborhood does not fit in LDS, holds a cell
 * twice (boxes of fewer than block edge + 2 cells per axis) or whose own
 * cells span more LDS slots than the reaction sums hold keep full lists.
 * tmd_get_neighbors then returns each atom's half list (in original ids,
 * rows sorted), the same physics as the full list.  The LDS sums are
 * atomic adds, so forces may differ from run to run in their last bits.
 * half: 1 on, 0 off (the default).  Lennard-Jones only, with one workgroup
 * per block and one lane per atom (tmd_set_schedule refuses block_parts or
 * lanes_per_atom above 1 while it is on); not with the adjoint
 * (tmd_adjoint_forward returns TMD_EINVAL).  A change splits each
 * workgroup's LDS anew between the neighborhood copy and the reaction sums,
 * which resets threads and lds_atoms to the block edge's defaults, and
 * marks the list stale.  TMD_EINVAL for other values or combinations.  Host
 * only. */
tmd_status tmd_set_half_list(tmd_system *sys, int32_t half);

/* Pick the schedule (block edge 2 or 3, full or half lists - the latter
 * for Lennard-Jones, with one workgroup per block and one lane per atom -,
 * workgroups per block 1, 2 or 4, lanes per atom 1, 2 or 4, threads per
 * force and per build workgroup, lanes per atom of the build 1 or 2)
 * with the shortest time per step for the current positions - one launch
 * of the step kernel (force sum, kicks and drift) plus 1/rebuild_every of a
 * list build: for each edge, list kind and workgroups per block, times `repeats`
 * builds per (build lanes, build threads) and `repeats` step-kernel launches per
 * (lanes, threads) candidate, threads from one lane group per mean block
 * atom (in whole wavefronts) up to two wavefronts more, on `stream` with HIP
 * events
 * (synchronises; the launches work on spare copies of the state).  Tune
 * on a state like the one the run will see: every wavefront runs to the
 * longest list among its atoms, so a perfect lattice, where all lists have
 * the same length, favours fewer lanes per atom than a liquid does.  Positions and velocities are not changed, but the list is
 * rebuilt at the current positions, as by tmd_build_neighbors(); call it
 * right after tmd_set_state() or at a rebuild step to keep the fixed
 * rebuild schedule.  Last, at the chosen schedule, the position layout
 * (tmd_set_layout) whose list build plus step kernel time is shortest
 * (Lennard-Jones).  flags: 0, or TMD_TUNE_ADJOINT to keep to full lists
 * and TMD_LAYOUT_SOA, which tmd_adjoint_forward() needs; TMD_EINVAL for
 * other bits. */
tmd_status tmd_autotune(tmd_system *sys, int32_t repeats, int32_t flags, tmd_stream stream);

/* Flags of tmd_autotune(). */
enum {
    TMD_TUNE_ADJOINT = 1 /* only schedules the adjoint runs with: full lists, TMD_LAYOUT_SOA */
};

/* Replace epsilon and sigma of every box (host arrays of n_boxes values, each
 * finite and positive); the copy to the device is enqueued on `stream`.  The
 * list is kept; forces are recomputed at the next step.  Lennard-Jones
 * systems only (TMD_EINVAL otherwise). */
tmd_status tmd_set_lj_params(tmd_system *sys, const double *epsilon, const double *sigma, tmd_stream stream);

/* --- Gradients through the discrete trajectory (reverse mode) ------------
 * The map from (x_0, v_0, epsilon, sigma) to the state after n_steps
 * velocity-Verlet steps, differentiated exactly with every neighbor list and
 * every cutoff indicator [s < cutoff^2] held as in the forward run (the
 * derivative almost everywhere; the force is discontinuous at the cutoff).
 * Going backward with h = dt / (2m), each force evaluation F(x_k) adds
 *   lam_x += c J(x_k) lam_v,   grad_theta += c lam_v . dF(x_k)/dtheta,
 * c = h at k = 0 and k = n_steps and 2h in between (the two half kicks at
 * x_k), J = dF/dx the LJ Hessian block matrix applied to lam_v as a
 * Hessian-vector product, and each drift adds lam_v += dt lam_x. */

/* Bytes of adjoint workspace for an n_steps run: (x, v) checkpoints at each
 * rebuild, the positions of every step (24 bytes per atom and step), each
 * rebuild interval's neighbor list with its atom order and tables (about
 * 40 + 16 * ceil(max_neighbors / 4 + 1) bytes per atom and interval),
 * cotangents. */
tmd_status tmd_adjoint_workspace_size(const tmd_system *sys, int32_t n_steps, size_t *bytes);

/* Integrate n_steps like tmd_integrate() (bit-identical trajectory) while
 * recording checkpoints and every step's positions in `ws`
 * (device, 256-byte aligned, at least tmd_adjoint_workspace_size bytes,
 * borrowed until the backward pass).  The step counter must be a multiple of
 * rebuild_every (TMD_ESTATE otherwise); the run starts from a list built at
 * the current positions.  Lennard-Jones systems only (TMD_EINVAL for the
 * Spring-Dashpot model). */
tmd_status tmd_adjoint_forward(tmd_system *sys, int32_t n_steps, void *ws, size_t bytes, tmd_stream stream);

/* Given the cotangents of the final state lam_x[3] (required) and lam_v[3]
 * (nullable = zero), device arrays in original order, write
 * grad_x0[3] = dL/dx_0, grad_v0[3] = dL/dv_0 (nullable), and per box
 * grad_eps[n_boxes], grad_sigma[n_boxes] (device, nullable).  Needs the run
 * recorded by tmd_adjoint_forward() in the same workspace with no
 * state-changing call in between (TMD_ESTATE otherwise).  Takes each
 * interval's list, atom order and positions from the workspace (as the
 * recorded run built them), and leaves the system in the run's final
 * state. */
tmd_status tmd_adjoint_backward(tmd_system *sys, void *ws, size_t bytes, const double *const lam_x[3],
                                const double *const lam_v[3], double *const grad_x0[3], double *const grad_v0[3],
                                double *grad_eps, double *grad_sigma, tmd_stream stream);

/* Per-kernel-class timing with HIP events recorded on the launch stream
 * (only while enabled): around every kernel, except that the back-to-back
 * force launches of tmd_integrate between two list rebuilds share one pair of
 * events (their average then holds no event overhead).  tmd_get_timing()
 * synchronises, then returns accumulated milliseconds and launch counts for
 * the TMD_T_* classes (arrays of at least TMD_T_COUNT entries) and resets the
 * accumulators. */
tmd_status tmd_set_timing(tmd_system *sys, int32_t enable);
tmd_status tmd_get_timing(tmd_system *sys, double *ms, int64_t *launches);

/* Graph mode for tmd_integrate (off by default).  While enabled, and while
 * thermo_every == 0 and timing is off, tmd_integrate() runs every whole
 * rebuild interval that starts after a step number divisible by
 * rebuild_every and ends before its last step as one HIP graph launch on
 * `stream`: rebuild_every - 1 fused steps, the binning and list build, and
 * the fused step after them.  The first such interval is captured on a
 * stream the library creates and owns; as the interval flips which copy of
 * the double-buffered state is current, runs alternate between two graphs.
 * A graph is keyed by everything it bakes in (schedule, workspace pointers,
 * current copies, interval) and recaptured when any of it changes.  Results
 * are bit-identical to graph mode off.  Disabling releases the graphs;
 * tmd_destroy() releases them and the capture stream.  The graphs hold no
 * memsets and no host work. */
tmd_status tmd_set_graphs(tmd_system *sys, int32_t enable);

/* --- One call that allocates nothing ------------------------------------
 * For callers that cannot allocate device memory or bind a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Equivalent to tmd_create + tmd_bind_workspace +
 * tmd_set_state (zero velocities) + tmd_build_neighbors +
 * tmd_compute_forces + tmd_sync's status, at the default schedule, with
 * bitwise the same forces, energy and virial, but every intermediate
 * (cells, sorted state, neighbor list, block partials, error word) lives in
 * one library-owned device array of TMD_STATIC_SCRATCH_BYTES per GPU.
 * params, n_atoms, box_length: as tmd_create (same synchronous errors).
 * pos[3]: device arrays of n_atoms doubles (original order), read on stream.
 * f[3] (nullable, any component nullable): device arrays receiving F.
 * energy_virial (nullable, device, 2 doubles): U and W as tmd_compute_forces.
 * device_status (nullable, device, 2 int32): [0] the status tmd_sync would
 * return for the device-detected conditions (TMD_OK, TMD_ENBR_OVERFLOW,
 * TMD_ENONFINITE, TMD_EINVAL for a coordinate outside [-L, 2L)), [1] the
 * largest list length requested on overflow; written on stream.
 * Returns TMD_EWORKSPACE, before touching the GPU, when the system's
 * workspace (tmd_workspace_size of the same system at one block edge)
 * exceeds TMD_STATIC_SCRATCH_BYTES: about 90,000 atoms at max_neighbors =
 * 128 and liquid density.  The first call on a device looks up that
 * device's copy of the array and sets kernel attributes (no allocation);
 * make it outside any stream capture.  Calls on the same GPU share its one
 * array: calls that overlap (other streams, other threads) race and must be
 * serialised by the caller; a later call overwrites the earlier one's
 * intermediates (outputs are the caller's and are not touched again). */
#define TMD_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
tmd_status tmd_compute_forces_static(const tmd_params *params, int64_t n_atoms, double box_length,
                                     const double *const pos[3], double *const f[3], double *energy_virial,
                                     int32_t *device_status, tmd_stream stream);

/* Static description of a status code. */
const char *tmd_status_string(tmd_status status);

/* Detail of the last error on this system (never NULL). */
const char *tmd_last_error(const tmd_system *sys);

/* Release the handle (does not free the workspace).  NULL is a no-op. */
void tmd_destroy(tmd_system *sys);

#ifdef __cplusplus
}
#endif

#endif /* TMD_H */
