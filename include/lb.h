/*
 * lb.h - C ABI of the MI355X (gfx950) library for the binary free-energy
 * lattice Boltzmann method of Pooley, Kusumaatmaja and Yeomans, "Contact line
 * dynamics in binary lattice Boltzmann simulations" (arXiv:0812.1282).
 *
 * One call of lb_step advances a D2Q9 lattice by whole timesteps. Each
 * timestep is one fused HIP sweep that, at every fluid node:
 *   - pulls the post-collision populations f_i and g_i of the previous step
 *     from the neighbours (Eqs. (stream1), (stream2)), bouncing back on solid
 *     neighbours (mid-link bounce-back, Sec. IV and Sec. V.B);
 *   - forms rho, phi and u (Eq. (moments));
 *   - evaluates the isotropic gradient and Laplacian of phi (Appendix A,
 *     Eq. (best)) from an LDS tile, with ghost values of phi at solid nodes
 *     that impose the wall gradient d_perp phi = xi / kappa (Sec. II);
 *   - forms mu = A phi + B phi^3 - kappa lap phi and p0 = rho/3 + A phi^2/2
 *     + 3 B phi^4 / 4 (Eqs. (chempot), (p0); the paper's a is B = -A);
 *   - forms tau(phi) (Eq. (tau)) and the equilibria of Appendix A, with u = 0
 *     at boundary nodes when Step 2 of Sec. VI is enabled;
 *   - collides f with BGK (Eq. (latbolt)) or MRT (Eqs. (mrtlb), (Matrix),
 *     (diag)) and g with BGK (Eq. (gevo));
 *   - writes the post-collision populations of the node.
 *
 * Conventions
 *   - Node (x, y), 0 <= x < nx, 0 <= y < ny, has host index y*nx + x. The
 *     lattice is periodic in x and y; walls are solid nodes of a mask.
 *   - Velocities: e0 = (0,0), e1 = (1,0), e2 = (-1,0), e3 = (0,1), e4 = (0,-1),
 *     e5 = (1,1), e6 = (-1,-1), e7 = (-1,1), e8 = (1,-1) (Sec. III.A).
 *   - The state at step n is S_n: the post-streaming, pre-collision
 *     populations. Host population arrays hold 9 planes of nx*ny values,
 *     plane i first (index i*nx*ny + y*nx + x).
 *   - d_perp points from the wall into the fluid, so d_perp phi < 0 makes the
 *     phi > 0 phase wet the wall (contact angle below 90 degrees, measured
 *     through the phi > 0 phase).
 *
 * Errors: every entry point returns LB_OK (0) or a negative LB_E* code and
 * never throws; lb_last_error() returns the calling thread's last message.
 * Host arrays passed in are borrowed for the duration of the call only.
 * Asynchronous device failures surface at the next synchronising call.
 *
 * Profiling: lb_init, lb_step, lb_batch_init, lb_batch_step, the autotuner,
 * graph capture and graph replay each open a roctx range (host time), seen
 * by a profiler's marker trace; without a profiler they cost nothing
 * measurable.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_EINVAL (-1)   /* invalid argument (sizes, tau <= 1/2, non-finite input, NULL) */
#define LB_ENOMEM (-2)   /* device or host allocation failed, or a buffer is too small */
#define LB_EHIP (-3)     /* a HIP runtime call failed */
#define LB_ENUMERIC (-4) /* a diagnostic found a non-finite value */
#define LB_ENODATA (-5)  /* a measurement found too few points / no wall intersection */
#define LB_EIO (-6)      /* checkpoint file could not be written or read */

/* Collision operator for f (g always uses BGK, Eq. (gevo)). */
#define LB_BGK 0
#define LB_MRT 1

/* Storage of the populations in device memory. LB_F64 stores f and g in FP64
 * and computes in FP64. The others compute in FP32 on deviations from the rest
 * state of a bulk phase at rho_ref: LB_F32 stores f_i minus that rest value and
 * g in FP32; LB_F16S / LB_BF16S store the f_2, f_4..f_8 deviations and g_1..g_8
 * in 16 bits (scaled by powers of two; f_i and g_i of the same direction share
 * one 32-bit word) and the f_0, f_1, f_3 deviations and g_0 in 32 bits. In every shifted format g_0 is kept relative to the nearest of
 * -1, 0, 1, and the 32-bit populations are formed from the rounded others, so
 * that the stored populations of a node carry its rho, momentum and phi to
 * FP32 precision of small values.
 * Bytes per node per buffer: 144 (FP64), 72 (FP32), 44 (16-bit), 104 (LB_F64C),
 * 52 (LB_F32C); two buffers, or one plus 8 bytes with lb_params.inplace. */
#define LB_F64 0
#define LB_F32 1
#define LB_F16S 2
#define LB_BF16S 3
/* Compressed g (tau_phi = 1 only, Sec. III.A with tau_phi = 1 makes every
 * post-collision g an equilibrium): instead of g_0..g_8 a node stores the four
 * numbers its g^eq is made of (phi, Gamma mu and the velocity of g^eq), and a
 * receiving node forms g^eq_i of its neighbour from them; f as in LB_F64 /
 * LB_F32. 13 values per node instead of 18. The dynamics are those of the
 * uncompressed format; only the g populations of S_0 read back differently (as
 * g_0 = phi_0, g_i = 0), which does not enter any later step because the first
 * collision replaces g by g^eq of phi_0. lb_init rejects tau_phi != 1. */
#define LB_F64C 4
#define LB_F32C 5

typedef struct lb_handle lb_handle;
typedef struct lb_batch lb_batch;

typedef struct {
    int32_t nx, ny;       /* lattice size, each >= 3 */
    double A, B;          /* Landau coefficients: mu = A phi + B phi^3 - kappa lap phi */
    double kappa;         /* gradient-energy coefficient, Eq. (freeen) */
    double Gamma;         /* mobility parameter of g^eq, Eq. (Mobility) */
    double tau_alpha;     /* tau_rho in the phi = +1 phase, > 1/2 */
    double tau_beta;      /* tau_rho in the phi = -1 phase, > 1/2 */
    double tau_phi;       /* relaxation time of g, > 1/2 */
    double rho_ref;       /* reference density of the 16-bit shifted storage */
    int32_t collision;    /* LB_BGK or LB_MRT */
    int32_t storage;      /* LB_F64, LB_F32, LB_F16S, LB_BF16S, LB_F64C, LB_F32C */
    int32_t zero_u_feq;   /* Step 2 of Sec. VI: u = 0 at boundary nodes in f^eq */
    int32_t zero_u_geq;   /* the same for g^eq */
    int32_t diag_every;   /* enqueue the non-finite check every k steps (0 = never) */
    int32_t tau_clamp;    /* 0: tau is Eq. (tau) in the node's phi, also where |phi| > 1;
                             1: phi is clamped to [-1, 1] first, so tau stays between
                             tau_beta and tau_alpha (keeps tau > 1/2 where phi
                             overshoots a bulk value and that bulk tau is close to 1/2) */
    int32_t inplace;      /* 0: two population buffers, each step pulls from one into
                             the other. 1: one buffer updated in place (LB_F64 and
                             LB_F32, single lattices only): even steps take a node's
                             populations from its neighbours' slots and return them
                             there, odd steps read and write the node's own slots, so
                             every node reads and writes the same slots and no second
                             buffer is needed; the phi of the nodes along tile borders
                             is formed by a pre-pass into a plane of 8 bytes per node.
                             Results are bit-identical to inplace = 0. */
    int32_t tau_lut;      /* 0: tau from Eq. (tau). n >= 2 (at most 2^24): the table
                             of Sec. VI, n values of tau evenly spaced from tau_beta
                             to tau_alpha (evenly in viscosity too); each node takes
                             the entry nearest its Eq. (tau) value, the lower one on
                             a tie (so tau stays within the bulk range) */
    int32_t bounce;       /* LB_MIDLINK or LB_LATTICE_NODE */
} lb_params;

/* Wall treatment (lb_params.bounce). LB_MIDLINK: mid-link bounce-back (Sec. V.B,
 * Fig. 9a). LB_LATTICE_NODE: the wall lies on the boundary nodes (Fig. 9b): a
 * solid node with a fluid neighbour keeps the populations that stream into it
 * and sends each back the way it came on the next step, so a population
 * returns to the node it left after two steps; at S_0 it holds what the
 * equilibria of its fluid neighbours send into it. LB_F64 and LB_F32 with
 * inplace = 0. Mass is conserved over fluid and wall nodes together; the sums
 * of lb_diagnostics cover the fluid nodes only. */
#define LB_MIDLINK 0
#define LB_LATTICE_NODE 1

typedef struct {
    double sum_rho;       /* FP64 sum of rho over fluid nodes of S_n */
    double sum_phi;       /* FP64 sum of phi over fluid nodes */
    double kinetic;       /* FP64 sum of rho |u|^2 / 2 */
    double max_u;         /* max |u| */
    int64_t n_fluid;      /* number of fluid nodes */
    int64_t step;         /* n */
} lb_diag;

/* Tile shape of the sweep: block_x columns per workgroup (64, 128, 256, 512 or 1024;
 * LB_F64C up to 512) and
 * rows_per_block rows walked by each workgroup (1 .. 1024). */
typedef struct {
    int32_t block_x;
    int32_t rows_per_block;
} lb_tuning;

/* Fill p with the defaults of the paper's Sec. IV set-up (a = kappa = 0.04,
 * tau = 1, Gamma = 0.1, BGK, FP64, rho_ref = 1) for an nx x ny lattice. */
int lb_default_params(int32_t nx, int32_t ny, lb_params* p);

/* Bytes of device memory one lattice with these parameters needs, for a
 * caller that provides its own buffer to lb_init_ext. */
int lb_workspace_bytes(const lb_params* p, size_t* bytes);

/*
 * Create a lattice whose state S_0 is the equilibrium (Appendix A) of the
 * initial fields, with the initial velocity in both f^eq and g^eq.
 *   solid      nx*ny bytes, nonzero = solid node (required). A fluid node
 *              whose eight neighbours are all solid is rejected.
 *   wall_dphi  nx*ny values of d_perp phi, read at solid nodes (NULL = 0, a
 *              neutral 90-degree wall).
 *   phi0       nx*ny initial order parameter (required).
 *   rho0, ux0, uy0  nx*ny (NULL = rho_ref, 0, 0). Values at solid nodes are
 *              ignored.
 *   stream     hipStream_t on which every kernel of this handle runs (NULL =
 *              the null stream); borrowed, must outlive the handle.
 * lb_init allocates the device memory itself; lb_init_ext uses a caller
 * buffer of at least lb_workspace_bytes bytes (256-byte aligned) that must stay
 * valid until lb_free. Errors: LB_EINVAL, LB_ENOMEM, LB_EHIP.
 */
int lb_init(const lb_params* p, const uint8_t* solid, const double* wall_dphi,
            const double* phi0, const double* rho0, const double* ux0, const double* uy0,
            void* stream, lb_handle** out);
int lb_init_ext(const lb_params* p, const uint8_t* solid, const double* wall_dphi,
                const double* phi0, const double* rho0, const double* ux0, const double* uy0,
                void* stream, void* device_buffer, size_t buffer_bytes, lb_handle** out);

/* Enqueue nsteps >= 0 timesteps on the handle's stream; does not block. The
 * steps are replayed from HIP graphs that the first call captures (on an
 * internal stream; windows of 1, 2, 4, ..., 32 steps for either parity, with
 * and without the periodic check at their first step), so every later call,
 * of any length, replays graphs only. */
int lb_step(lb_handle* h, int64_t nsteps);

/* Synchronise and copy the moments of S_n (Eq. (moments)) to host arrays of
 * nx*ny doubles; any pointer may be NULL. Solid nodes read 0. */
int lb_read_fields(lb_handle* h, double* phi, double* rho, double* ux, double* uy);

/* Synchronise and copy S_n out: f and g, each 9*nx*ny doubles (NULL to skip).
 * Solid nodes read 0. */
int lb_read_populations(lb_handle* h, double* f, double* g);

/* Synchronise; FP64 conservation sums and kinetic energy of S_n. Returns
 * LB_ENUMERIC (with d filled) if any of them, or an earlier periodic check,
 * is not finite. */
int lb_diagnostics(lb_handle* h, lb_diag* d);

/* lb_diagnostics without allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same reduction kernels and the same result bit for bit; the
 * per-block partial sums, the finished record and a flag word live in a fixed
 * device array of the library (2 MiB + 320 bytes, 2^15 records of 256 nodes;
 * each GPU the library runs on holds its own copy until the process ends)
 * instead of the lattice's memory. Lattices of at most 2^23 nodes (LB_EINVAL
 * beyond). The array keeps the last call's contents and is shared by every
 * call on that GPU: calls that overlap on one GPU (several threads or streams)
 * race. Synchronises the handle's stream. */
int lb_diagnostics_noalloc(lb_handle* h, lb_diag* d);

/*
 * Contact angle (Sec. IV): every axis link between two fluid nodes whose phi
 * values have opposite signs gives the phi = 0 crossing by linear
 * interpolation; crossings inside [x_lo, x_hi) x [y_lo, y_hi] (x and y taken at
 * the periodic image nearest the window centre) are fitted by a least-squares
 * circle in FP64, and the angle between the circle and the wall plane
 * y = y_wall, whose normal into the fluid is (0, wall_dir) with wall_dir = +1
 * or -1, is returned in degrees, measured through the phi > 0 phase. Outputs
 * may be NULL except theta_deg. LB_ENODATA if fewer than 3 crossings are found
 * or the circle does not reach the wall.
 */
int lb_contact_angle(lb_handle* h, double x_lo, double x_hi, double y_lo, double y_hi,
                     double y_wall, int32_t wall_dir, double* theta_deg, double* xc,
                     double* yc, double* radius, int64_t* n_points);

/* Length of the phi > 0 column in a channel (Sec. VII): the FP64 sum of
 * (1 + phi)/2 over fluid nodes with x_lo <= x < x_hi, divided by width. */
int lb_fill_length(lb_handle* h, int32_t x_lo, int32_t x_hi, double width, double* length);

/* Replace the wall gradient field (nx*ny, read at solid nodes; NULL = 0).
 * Takes effect from the next enqueued step. */
int lb_set_wall_dphi(lb_handle* h, const double* wall_dphi);

/* Write / read a checkpoint: parameters, step count, mask, wall field and the
 * device state, bit for bit. lb_load needs a handle of identical parameters;
 * it clears the handle's record of an earlier non-finite periodic check, so a
 * handle that blew up can resume from a good checkpoint. */
int lb_save(lb_handle* h, const char* path);
int lb_load(lb_handle* h, const char* path);

/* Tile shape: set (lb_set_tuning), read (lb_get_tuning), or pick by timing
 * candidate shapes on the handle's own stream with the state restored
 * afterwards (lb_autotune: 64..1024 columns x 1..128 rows; each candidate
 * timed over about steps_per_trial steps as replays of one captured graph,
 * the way lb_step runs them). The choice never changes results. A new lattice
 * starts with the shape lb_autotune chose for the same problem earlier in the
 * process on this kind of device, else with the tallest strips and widest
 * tiles (256 x 32 down to 64 x 4) that give at least one workgroup per CU;
 * a lattice whose step moves under 64 MB takes one-row strips (its step time
 * is the latency of a strip's row walk, not bandwidth). */
int lb_set_tuning(lb_handle* h, const lb_tuning* t);
int lb_get_tuning(lb_handle* h, lb_tuning* t);
int lb_autotune(lb_handle* h, int32_t steps_per_trial, lb_tuning* chosen);

/* Step count n of the current state. */
int lb_get_step(lb_handle* h, int64_t* step);

/* Release the handle and the device memory it allocated. NULL is a no-op. */
int lb_free(lb_handle* h);

/* Thread-local message of the last error (never NULL). */
const char* lb_last_error(void);

/* Eq. (theory) of Sec. IV: d_perp phi at the wall for an equilibrium contact
 * angle theta (degrees, 0..180) with mu = A phi + B phi^3 - kappa lap phi,
 * B = -A > 0. */
int lb_dphi_for_angle(double theta_deg, double kappa, double A, double B, double* dphi);

/* Streaming-copy rate of the device: time `repeats` copies of `bytes`
 * (>= 1 MiB) between two scratch buffers it allocates and frees, with three
 * copy kernels (one 16-byte element per thread and iteration; four in flight
 * with nontemporal stores; four with nontemporal loads and stores) at 2, 4, 8
 * and 16 workgroups of 256 threads per CU, and return the best read + write
 * rate in GB/s. A reference for the sweep's achieved bandwidth, not part of the
 * method. */
int lb_bandwidth_probe(size_t bytes, int32_t repeats, void* stream, double* gbs);

/*
 * Batched ensembles: n independent lattices (own sizes, masks, parameters and
 * initial fields) advanced together, one fused launch per timestep over the
 * tiles of all members, replayed from a HIP graph. Every member must share
 * storage, collision and the Step 2 flags and have inplace = 0; arrays are per member as in
 * lb_init. lb_batch_step enqueues nsteps for every member. With tuning NULL,
 * lb_batch_init picks the tile shape with lb_batch_autotune (4 timed steps per
 * candidate); lb_batch_autotune times the candidate shapes over the whole
 * ensemble with the state restored afterwards and keeps the fastest. The tile
 * order is fixed by the tiling: members are dealt to the 8 XCDs, largest
 * first, each to the XCD with the least work so far (a member with more than
 * an eighth of the work is first cut into contiguous runs of equal work, at
 * most an eighth each, dealt the same way), and each XCD takes its tiles
 * largest first. The choice never changes results.
 */
int lb_batch_init(int32_t n, const lb_params* params, const uint8_t* const* solid,
                  const double* const* wall_dphi, const double* const* phi0,
                  const double* const* rho0, const double* const* ux0,
                  const double* const* uy0, void* stream, const lb_tuning* tuning,
                  lb_batch** out);
int lb_batch_step(lb_batch* b, int64_t nsteps);
int lb_batch_read_fields(lb_batch* b, int32_t member, double* phi, double* rho, double* ux,
                         double* uy);
int lb_batch_read_populations(lb_batch* b, int32_t member, double* f, double* g);
int lb_batch_contact_angle(lb_batch* b, int32_t member, double x_lo, double x_hi,
                           double y_lo, double y_hi, double y_wall, int32_t wall_dir,
                           double* theta_deg);
int lb_batch_autotune(lb_batch* b, int32_t steps_per_trial, lb_tuning* chosen);

/* Schedule of a batch's timesteps. LB_SCHEDULE_STEPWISE: one launch per step over
 * every member's tiles (the tile table above). LB_SCHEDULE_PERSISTENT: a window
 * of steps (up to 32, the graph windows of lb_step) is one launch of as many
 * workgroups as fit on the device (at most two steps' tiles), which take
 * (step, tile) items in order from a counter and sweep a tile as soon as the
 * tiles around it (within one tile, same member) have finished the previous
 * step: no barrier between members or
 * steps, so members of different sizes and the end of one step overlap the
 * start of the next. A step with the periodic check runs stepwise. Members
 * narrower than block_x get proportionally taller strips under either
 * schedule, so every tile holds about block_x x rows_per_block nodes. Needs
 * block_x 128, 256 or 512, strips of at least 3 rows and no lattice-node
 * members (LB_EINVAL otherwise). Results are identical under both schedules.
 * spin_limit: polls a waiting workgroup makes before it gives up (0 = the
 * default, 2^20; a wait also gives up after about one second); when one gives
 * up, every workgroup leaves and every later read of the batch (fields,
 * populations, contact angle) returns LB_EHIP (the state is then invalid).
 * lb_batch_autotune (and lb_batch_init without a tuning) times both schedules
 * and keeps the faster. */
#define LB_SCHEDULE_STEPWISE 0
#define LB_SCHEDULE_PERSISTENT 1
int lb_batch_set_schedule(lb_batch* b, int32_t schedule, uint32_t spin_limit);
int lb_batch_get_schedule(lb_batch* b, int32_t* schedule);
int lb_batch_get_tuning(lb_batch* b, lb_tuning* t);
int lb_batch_free(lb_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* LB_H */
