/*
 * mpx.h -- C ABI of libmpx, the gfx950 (MI355X) implementation of the
 * explicit time step of Maxwell's equations on a 3-D Yee grid coupled cell
 * by cell to the Landau-Lifshitz-Gilbert update of the magnetisation.
 *
 * The coupled problem is the one stated in arXiv:2510.22221, Methods,
 * "Numerical Model": Ampere's law with conduction (eq. Ampere) discretised
 * semi-implicitly in sigma, Faraday's law with B = mu0 (H + M) integrated as
 * eq. (iterate_H), and the Gilbert-form LLG (eq. LLG) advanced with the
 * trapezoidal rule of eqs. (llg_tra4)-(llg_tra6) and normalised to the local
 * saturation magnetisation.  H and M advance in two half steps around each
 * full E step (the dt/4 and dt/(2 mu0) factors of those equations).
 *
 * Conventions shared by every call
 *   - Every function returns mpx_status; nothing throws across the ABI.
 *   - Units are SI: m, s, V/m, A/m, S/m.  |gamma| in rad/(s T).
 *   - Cell (i,j,k) spans [i dx,(i+1) dx] x [j dy,(j+1) dy] x [k dz,(k+1) dz].
 *     Host arrays are x-fastest: element (i,j,k) of an array with natural
 *     dims (n0,n1,n2) is at i + n0 (j + n1 k).
 *   - Natural Yee dims of a field component (mpx_query_field): E_c has N_c
 *     entries along c and N_a + 1 along the other axes a; H_c has N_c + 1
 *     along c and N_a along the others; a periodic axis drops the "+1".
 *   - Host buffers passed in are copied during the call; the caller keeps
 *     ownership.  Device memory the library allocates is released by
 *     mpx_destroy.
 *   - A HIP error makes the handle fail with MPX_E_DEVICE from then on
 *     (sticky); only mpx_destroy and mpx_last_error still work.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef MPX_H
#define MPX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPX_ABI_VERSION 4u

typedef struct mpx_sim mpx_sim;

typedef enum {
    MPX_OK = 0,
    MPX_E_INVALID = 1,     /* bad argument; no side effect */
    MPX_E_STATE = 2,       /* call out of order (e.g. step before materials) */
    MPX_E_NOMEM = 3,       /* device or host allocation failed */
    MPX_E_DEVICE = 4,      /* HIP runtime error (sticky) */
    MPX_E_UNSUPPORTED = 5, /* valid request this library does not implement */
    MPX_E_RANGE = 6,       /* destination too small */
    MPX_E_NONFINITE = 7    /* the non-finite watchdog fired */
} mpx_status;

typedef enum { MPX_F64 = 0, MPX_F32 = 1 } mpx_precision;

typedef enum { MPX_BC_PEC = 0, MPX_BC_PML = 1, MPX_BC_PERIODIC = 2 } mpx_bc;

typedef enum {
    MPX_EX = 0, MPX_EY = 1, MPX_EZ = 2,
    MPX_HX = 3, MPX_HY = 4, MPX_HZ = 5,
    /* the full magnetisation vector at the x-, y- and z-face sites:
     * 3 components, component-major, each over that face family's natural
     * dims; zero at non-magnetic sites.  Always float64. */
    MPX_M_XFACE = 6, MPX_M_YFACE = 7, MPX_M_ZFACE = 8,
    /* the same minus the initial state M0 = Ms_site u (read only) */
    MPX_DM_XFACE = 9, MPX_DM_YFACE = 10, MPX_DM_ZFACE = 11
} mpx_field;

typedef enum {
    MPX_PROBE_FIELD = 0,       /* one E or H component at one site, 1 value */
    MPX_PROBE_MEAN_M = 1,      /* film-averaged M, 3 values per sample */
    MPX_PROBE_FILM_ENERGY = 2, /* EM energy inside the film's cells, 1 value */
    MPX_PROBE_EM_ENERGY = 3    /* discrete EM energy of the whole grid, 1 value */
} mpx_probe_kind;

/* Grid.  dt <= 0 selects dt = courant / (c sqrt(dx^-2 + dy^-2 + dz^-2))
 * (the Courant-limited step of Results, setup section: CFL factor 0.9).
 * bc[] is -x,+x,-y,+y,-z,+z; a periodic axis must be periodic on both faces.
 * PML faces are convolutional PML slabs of pml_cells[] cells backed by a PEC
 * wall, graded sigma = sigma_max rho^order with
 * sigma_max = pml_sigma_factor (order+1)/(eta0 d) (defaults 3 and 0.8 when
 * <= 0); the paper names PML on all faces without a formulation. */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    double courant;
    double dt;
    int32_t bc[6];
    int32_t pml_cells[6];
    double pml_order;
    double pml_sigma_factor;
} mpx_grid_desc;

/* One entry of the per-cell material table (Methods, "Numerical Model":
 * eps_r, sigma, Ms, alpha, gamma are spatially dependent).  is_pec != 0 makes
 * every edge touching the cell a perfect conductor.  Ms > 0 makes the cell
 * magnetic. */
typedef struct {
    double eps_r, sigma;
    int32_t is_pec;
    double Ms, alpha, gamma_abs;
} mpx_material;

/* Soft current source on the E_component edges of a box given in that
 * component's natural index space: J(t_{n+1/2}) = table[n] (A/m^2), zero
 * past the end of the table; it enters the E update as
 * E <- ca E + cb (curl H - J) (the J_src of the E update in Methods). */
typedef struct {
    int32_t component;              /* 0..2 = Jx, Jy, Jz */
    int32_t i0, j0, k0, ni, nj, nk;
    const double *table;            /* host, float64, copied */
    int64_t n_table;
} mpx_source_desc;

/* Probe sampled after every `every`-th full step (at t_{n+1}: the steps
 * n+1 = every, 2 every, ... counted from the step it was added at; 0 means
 * 1) into a ring buffer of `capacity` samples.  FIELD: field =
 * MPX_EX..MPX_HZ at natural index (i,j,k) (H probes must lie outside PML
 * slabs).  MEAN_M and FILM_ENERGY use `film` (films are numbered by their
 * lowest linear cell index).  EM_ENERGY records the W_EM of mpx_energy at
 * that time (the exactly conserved discrete energy of the leap-frog scheme
 * without sources, losses and films; not defined with PML faces); it reads
 * every field value of the grid once per sample, so a stride keeps its cost
 * small. */
typedef struct {
    int32_t kind;
    int32_t field;
    int32_t i, j, k;
    int32_t film;
    int32_t every;
    int64_t capacity;
} mpx_probe_desc;

/* ABI version of the loaded library (MPX_ABI_VERSION). */
uint32_t mpx_abi_version(void);

/* Create a simulation on HIP device `hip_device`.  `hip_stream` is a
 * hipStream_t the caller owns (it must outlive the handle) or NULL, in which
 * case the library creates and owns a non-blocking stream at default
 * priority.  All device work of the handle is ordered on that stream.
 * Errors: MPX_E_INVALID for non-positive sizes or spacings, courant outside
 * (0, 1] when dt <= 0, an explicit dt > 0 above the 3-D Yee stability limit
 * 1 / (c sqrt(dx^-2 + dy^-2 + dz^-2)) (or not finite), a one-sided periodic
 * axis, PML slabs that leave no interior cell on an axis (all checked before
 * any device call); MPX_E_DEVICE / MPX_E_NOMEM from HIP. */
mpx_status mpx_create(const mpx_grid_desc *grid, mpx_precision precision, int32_t hip_device,
                      void *hip_stream, mpx_sim **out);

/* Release every device and host resource of the handle (NULL is a no-op). */
mpx_status mpx_destroy(mpx_sim *sim);

/* Natural dims of a field (dims[3] = 1, or 3 for the M fields) and the size
 * in bytes of a host buffer that holds it (float64 in MPX_F64 mode and for
 * every M field, float32 for E/H in MPX_F32 mode). */
mpx_status mpx_query_field(const mpx_sim *sim, int32_t field, int64_t dims[4], int64_t *bytes);

/* Material table (n <= 256 entries) and one uint8 id per cell, host array of
 * nx*ny*nz bytes, x fastest.  Finds the films (bounding boxes of connected
 * magnetic cells, boxes closer than two cells merged) and resets M to zero.
 * Errors: MPX_E_INVALID for an id >= n, a magnetic cell inside or next to a
 * PML slab, or > 64 films; MPX_E_UNSUPPORTED for a film that touches a
 * non-periodic domain face or wraps partially around a periodic one;
 * MPX_E_STATE once a MEAN_M or FILM_ENERGY probe exists (it names a film of
 * the previous map: set the materials first). */
mpx_status mpx_set_materials(mpx_sim *sim, const mpx_material *table, int32_t n, const uint8_t *cell_ids);

/* Uniform static bias field H0 (A/m), part of H_eff (Methods: H_eff collects
 * the EM field and the static bias). */
mpx_status mpx_set_bias(mpx_sim *sim, double H0x, double H0y, double H0z);

/* M = Ms_site u at every magnetic face site (u normalised here; the paper
 * saturates the film along the bias).  This state is also M0 for the
 * MPX_DM_* fields.  MPX_E_STATE before mpx_set_materials. */
mpx_status mpx_init_magnetization(mpx_sim *sim, double ux, double uy, double uz);

/* Add a source (at most 16).  *id receives its index. */
mpx_status mpx_add_source(mpx_sim *sim, const mpx_source_desc *src, int32_t *id);

/* Add a probe (at most 64).  Samples start with the next step.
 * Errors: MPX_E_INVALID (kind, index, film, capacity < 1, every < 0),
 * MPX_E_STATE (film or energy probe before mpx_set_materials),
 * MPX_E_UNSUPPORTED (an H probe inside a PML slab, EM_ENERGY with PML
 * faces). */
mpx_status mpx_add_probe(mpx_sim *sim, const mpx_probe_desc *probe, int32_t *id);

/* Advance nsteps full steps: H/M half step, E step, H/M half step each
 * (consecutive H/M half steps are done in one pass).  Asynchronous on the
 * handle's stream; no host synchronisation inside.  MPX_E_STATE before
 * mpx_set_materials. */
mpx_status mpx_step(mpx_sim *sim, int64_t nsteps);

/* Wait for the handle's stream; reports MPX_E_NONFINITE if a probe saw a
 * non-finite value, MPX_E_DEVICE on a HIP error. */
mpx_status mpx_synchronize(mpx_sim *sim);

/* Copy a field out (natural dims) to host (dst_is_device = 0) or device
 * memory.  E and H into device memory: strided device-to-device copies on the
 * handle's stream, no host staging; M fields (film sites only) are gathered
 * on the host.  The device copies run on the handle's stream: work of other
 * streams on dst must be complete before the call.  Synchronises.
 * MPX_E_RANGE if dst_bytes is below mpx_query_field's size. */
mpx_status mpx_read_field(mpx_sim *sim, int32_t field, void *dst, int64_t dst_bytes, int32_t dst_is_device);

/* Copy the sub-box box = (i0,j0,k0,ni,nj,nk) of a field (natural index
 * space of that field) out, x fastest, ni*nj*nk elements per component (the M
 * fields: 3 components, component-major).  Synchronises.  MPX_E_INVALID if
 * the box leaves the field's natural dims, MPX_E_RANGE if dst_bytes is too
 * small. */
mpx_status mpx_read_field_region(mpx_sim *sim, int32_t field, const int32_t box[6], void *dst, int64_t dst_bytes,
                                 int32_t dst_is_device);

/* Overwrite a field (natural dims, the element type of mpx_query_field).
 * E values on PEC edges and on the faces of non-periodic walls are held at
 * zero; H values on the upper wall faces are not stored; M values are kept
 * only at magnetic sites.  MPX_DM_* fields are read-only.  The values pass
 * through host memory (the PEC edges are masked there), also from a device
 * source; mpx_field_storage gives copy-free device access. */
mpx_status mpx_write_field(mpx_sim *sim, int32_t field, const void *src, int64_t src_bytes, int32_t src_is_device);

/* Copy the recorded samples of probe `id`, oldest first, into dst (float64;
 * `capacity` counts samples).  *n_written = samples copied, or the number
 * required with MPX_E_RANGE. */
mpx_status mpx_read_probe(mpx_sim *sim, int32_t id, double *dst, int64_t capacity, int64_t *n_written);

/* Discrete EM energy at the current integer time,
 * dV/2 [sum_edges eps_e E^2 + mu0 sum_faces (H^2 - (dt/(2 mu0))^2 (curl E)^2)],
 * and the Zeeman term -mu0 dV sum_c sum_{family-c sites} H0_c M_c.  Computed
 * on the device in float64.  MPX_E_UNSUPPORTED with PML faces. */
mpx_status mpx_energy(mpx_sim *sim, double *W_em, double *W_zeeman);

/* Zero-copy access to the library's own storage of an E or H component
 * (field 0..5), for callers that keep fields in device tensors without
 * copies (in place of binding caller-owned buffers: the stored lattice is
 * padded, which the library owns).  Returns the device pointer of site
 * (0, 0, 0) and the element strides along x, y, z: stored site (i, j, k),
 * 0 <= i < nx, 0 <= j < ny, 0 <= k < nz, is element i + strides[1] j +
 * strides[2] k (float32 or float64 as the precision; x fastest, strides[1]
 * >= nx).  Sites of the natural dims beyond nx, ny or nz (wall edges and
 * faces) are not stored; they are zero.  `bytes` (may be NULL) is the
 * allocation's size.  The pointer stays valid until mpx_destroy; reads and
 * writes through it must be ordered with the handle's stream (a write must
 * keep PEC edges at zero).  Errors: MPX_E_INVALID (field, null pointers),
 * MPX_E_STATE under a fused schedule (mpx_set_schedule > 0: the fields move
 * between two buffers there). */
mpx_status mpx_field_storage(mpx_sim *sim, int32_t field, void **device_ptr, int64_t strides[3], int64_t *bytes);

/* mpx_energy without any device allocation, for callers that cannot
 * allocate (code running under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the per-block partial sums live in a
 * static device array of 2^21 doubles (16 MiB) that each GPU the library runs
 * on holds until the process ends.  Same results as mpx_energy, bitwise.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (several threads or handles) race.
 * Errors as mpx_energy, plus MPX_E_RANGE for a grid of more than 1048560
 * blocks of 64 x 4 cells (ceil(nx/64) ceil(ny/4) nz). */
mpx_status mpx_energy_noalloc(mpx_sim *sim, double *W_em, double *W_zeeman);

/* Step count, time = step dt, dt and number of films. */
mpx_status mpx_info(const mpx_sim *sim, int64_t *step, double *time, double *dt, int32_t *n_films);

/* Cell box (i0,j0,k0,ni,nj,nk) and magnetic cell count of film `film`. */
mpx_status mpx_film_box(const mpx_sim *sim, int32_t film, int32_t box[6], int64_t *ncells);

/* Steps captured per HIP graph by mpx_step (default 64; 0 launches every
 * kernel directly). */
mpx_status mpx_set_graph_steps(mpx_sim *sim, int32_t steps);

/* Step schedule.  fused = 0 (default): a separate E pass and H/M pass per
 * step, each in place with one thread per slot.  fused = 1..5: one fused
 * stencil pass per step (the E step and the merged H/M half-step pair in one
 * z-marching sweep over ping-pong buffers, z-chunks of `kchunk` planes; 0
 * keeps the current chunk, default 16): 1 = register-blocked sweep (64 x 4
 * columns per block, each thread recomputes the neighbour edges it needs);
 * 2..5 = LDS-staged sweep over 64 x 8 tiles (2: two rows per thread, >= 2
 * waves per SIMD; 3: two rows, >= 4 waves; 4: one row, >= 2 waves; 5: one
 * row, >= 4 waves).  fused = 6: the separate passes on 64 x 4 tiles also
 * on grids at least 512 cells wide (which schedule 0 runs on 256 x 1 tiles).
 * All give bitwise identical results.  Errors: MPX_E_INVALID for fused
 * outside 0..6 or kchunk < 0. */
mpx_status mpx_set_schedule(mpx_sim *sim, int32_t fused, int32_t kchunk);

/* Kernel timing with HIP events on the handle's stream.  With every > 0,
 * mpx_step launches every `every`-th step's kernels directly and brackets
 * three groups of them with events; the every - 1 steps between two timed
 * ones replay a captured graph (unless mpx_set_graph_steps(sim, 0)); 0 turns
 * timing off.  Results are the same bits either way.
 * mpx_kernel_time fills avg_ms[3] (average device time per timed launch,
 * ms) and launches[3] for the last mpx_step call: 0 = the main stencil
 * kernel (fused pass, or the E pass of the two-pass schedule), 1 = the H/M
 * pass of the two-pass schedule with the film's second half step (0 launches
 * when fused), 2 = the film's first half step and the probes. */
mpx_status mpx_set_timing(mpx_sim *sim, int32_t every);
mpx_status mpx_kernel_time(mpx_sim *sim, double *avg_ms, int64_t *launches);

/* Human-readable description of the last error on this handle. */
const char *mpx_last_error(const mpx_sim *sim);

/* ---- Gradients by the discrete adjoint ----------------------------------
 *
 * Runs nsteps time steps forward from the current state (like mpx_step) and
 * returns the loss L = dt * sum over steps n = loss_from+1 .. nsteps of the
 * EM energy of film `film` at integer time n (the film-energy probe's sum:
 * over the film's magnetic cells, 1/2 eps0 eps_r times the mean over its four
 * edges of E_c^2 plus 1/2 mu0 times the mean over its two faces of H_c^2,
 * summed over c, times the cell volume), together with its exact gradients
 * by reverse time stepping of the discrete scheme (the transposes of the E
 * step, of the H/M half steps and of the closed-form trapezoidal LLG solve,
 * with the CPML recursions; Methods, "Numerical Model"):
 *   dL_dH0[3]  with respect to the uniform bias H0 (A/m),
 *   dL_deps    with respect to eps_r of each cell of eps_box (i0, j0, k0,
 *              ni, nj, nk; x fastest), every cell taken as its own parameter,
 *   dL_dMs     with respect to Ms of each cell of ms_box (x fastest): through
 *              the face values Ms_s (mean over the face's cells) in the LLG
 *              solve and, when the run starts at step 0, through the initial
 *              magnetisation M0 = Ms_s u.
 * The run is cut into segments of `checkpoint_every` steps (0:
 * ceil(sqrt(nsteps))).  Under schedule 0 the reverse sweep reads, per step,
 * a tape of film-region and eps-box values: the last segments keep the tape
 * their forward run writes, as far as mpx_set_adjoint_memory allows, and
 * every other segment takes a checkpoint (a full field state) and is run
 * again from it, writing the tape, before its reverse steps.  Memory is
 * about (segments without a kept tape) + 12 field states, plus one
 * segment's tape, plus the kept tapes.  On return the handle holds the
 * state after nsteps (step counter advanced, probes recorded as by
 * mpx_step).
 * Host output buffers; boxes must lie inside the grid.  Synchronous.
 * Errors: MPX_E_INVALID (arguments), MPX_E_STATE (materials / magnetisation
 * not set), MPX_E_NOMEM / MPX_E_DEVICE. */
mpx_status mpx_adjoint(mpx_sim *sim, int64_t nsteps, int64_t loss_from, int32_t film, int32_t checkpoint_every,
                       const int32_t eps_box[6], const int32_t ms_box[6], double *loss, double *dL_dH0,
                       double *dL_deps, double *dL_dMs);

/* The same gradients (dL_dH0[3], dL_deps over eps_box, dL_dMs over ms_box,
 * as for mpx_adjoint) of a weighted trace of one E component at one edge:
 *   L = sum over i = 0 .. nsteps-1 of weights[i] * E_field(i, j, k) after
 *       step i+1,
 * i.e. the inner product of a field probe's record with a weight sequence.
 * Spectral functionals of a probe trace (a mode's amplitude at a frequency,
 * the frequency split of the two hybrid modes) are functions of the record;
 * their gradients follow by the chain rule with weights = dF/d(record) (the
 * anti-crossing splitting of Results, "Numerically Predicted Strong
 * Magnon-Photon Coupling Phenomena", is one: its derivative with respect to
 * the trace gives the weights).
 *   field      0, 1, 2 for E_x, E_y, E_z;
 *   ijk        a stored site (0 <= ijk[a] < the grid's size on axis a);
 *   weights    nsteps finite host values (read during the call only).
 * Tape schedules only (mpx_set_adjoint_schedule 0 or 2).  Memory, checkpoints and
 * the state on return as for mpx_adjoint.  Synchronous.
 * Errors: MPX_E_INVALID (arguments, a non-finite weight), MPX_E_STATE,
 * MPX_E_UNSUPPORTED under schedule 1, MPX_E_NOMEM / MPX_E_DEVICE. */
mpx_status mpx_adjoint_probe(mpx_sim *sim, int64_t nsteps, int32_t field, const int32_t ijk[3],
                             const double *weights, int32_t checkpoint_every, const int32_t eps_box[6],
                             const int32_t ms_box[6], double *loss, double *dL_dH0, double *dL_deps,
                             double *dL_dMs);

/* Reverse-sweep schedule of mpx_adjoint (same gradients up to rounding):
 *   0 (default) tape: each checkpoint segment is recomputed once while the
 *     values the adjoint maps read are taped, then its adjoint steps run
 *     from the tape (one captured graph replayed per segment, unless graphs
 *     are off: mpx_set_graph_steps(sim, 0));
 *     Where no film's reach (its face box grown by one slot) meets a CPML
 *     slab, the transposes of the two half steps around an integer time run
 *     as one field pass;
 *   1 plain: every reverse step reloads its input state and recomputes its
 *     half steps (the reference the tape schedule is tested against);
 *   2 tape, every half-step transpose in a pass of its own (the same bits
 *     as 0).
 * Errors: MPX_E_INVALID for another value. */
mpx_status mpx_set_adjoint_schedule(mpx_sim *sim, int32_t schedule);

/* Device memory the tape schedule may spend on keeping the tapes of the
 * forward run, so that those segments are not run a second time (the
 * gradients are the same bits either way):
 *   -1 (default) as much as fits, with the checkpoints of the other
 *      segments, in three quarters of the device memory free at the call;
 *    0 none: every segment is recomputed from its checkpoint;
 *   >0 at most that many bytes (whole segments' tapes).
 * Errors: MPX_E_INVALID for a value below -1. */
mpx_status mpx_set_adjoint_memory(mpx_sim *sim, int64_t max_bytes);

/* ---- Batched stepping (many simulations per launch) --------------------
 *
 * A batch groups n >= 1 simulation handles of one precision on one device,
 * each with materials set (and magnetisation initialised where it has
 * films), typically the same device under different bias fields or
 * geometries (a parameter sweep).  mpx_batch_step advances every member by
 * nsteps time steps with one fused stencil launch per step covering all
 * members' tiles, and one launch each for their film half steps and probes,
 * so that small grids still fill the chip (with the separate-pass schedule:
 * one launch per pass).  Each member's results are
 * bitwise identical to stepping it alone with mpx_step under the same tile
 * variant.  Sources, probes and films of each member behave exactly as for
 * a lone handle (its probe ring and step counter advance).
 *
 * The batch keeps pointers to the handles: they must outlive it and must not
 * be re-configured (materials, sources, probes, schedule) while it exists;
 * fields may be read and written between calls.  Work runs on the first
 * member's stream, ordered after each member's stream on entry and before
 * it on exit.  Errors: MPX_E_INVALID for null/duplicate handles or mixed
 * precision/device, MPX_E_STATE for a member not ready to step,
 * MPX_E_DEVICE for HIP failures (sticky on the batch). */
typedef struct mpx_batch mpx_batch;

mpx_status mpx_batch_create(mpx_sim *const *sims, int32_t n, mpx_batch **out);
mpx_status mpx_batch_destroy(mpx_batch *batch);

/* Schedule 0..5 (as for mpx_set_schedule) and z-chunk (0 keeps the current
 * one) of the batched step; defaults are those of the first member. */
mpx_status mpx_batch_set_schedule(mpx_batch *batch, int32_t variant, int32_t kchunk);

/* Steps per captured HIP graph (rounded up to even; 0 launches directly). */
mpx_status mpx_batch_set_graph_steps(mpx_batch *batch, int32_t steps);

mpx_status mpx_batch_step(mpx_batch *batch, int64_t nsteps);
mpx_status mpx_batch_synchronize(mpx_batch *batch);
const char *mpx_batch_last_error(const mpx_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* MPX_H */
