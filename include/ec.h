/*
 * ec.h - C ABI of the MI355X (gfx950) FFT eigenstrain / interaction-energy solver.
 *
 * Method: Santos-Gueemes, Ortiz, Segurado, "An FFT based approach to account
 * for elastic interactions in OkMC" (arXiv 2403.09158).
 *   - Sec. 3.1: defects enter as eigenstrains; a loop carries sym(b x n)/e in a
 *     slab of thickness e extruded from its area, a point-defect cluster a
 *     dilatation in a small region (here a sphere, eps* = v I).
 *   - Sec. 3.2: periodic equilibrium with eigenstrain, solved in Fourier space by
 *     the Green operator built from the inverse acoustic tensor; then
 *     sigma = C:(eps - eps*).
 *   - Sec. 3.4: voxel-centre grid x = h (m + 1/2) and centred frequency labels.
 *   - Sec. 2: interaction energy in the Betti-reciprocity form.
 *   - Appendix B (OkMC algorithm): a moved defect changes the total field by
 *     its own field difference (superposition), which is what the incremental
 *     update computes.
 *
 * Units: lengths nm, stiffness and stress GPa, energies eV.
 * Fields are structure-of-arrays [6][n][n][n] with x fastest (linear voxel id
 * (z*n + y)*n + x), component order xx, yy, zz, yz, xz, xy, tensor components
 * (shear not doubled), so A:B = A_xx B_xx + A_yy B_yy + A_zz B_zz
 * + 2 (A_yz B_yz + A_xz B_xz + A_xy B_xy).
 *
 * Error behaviour: every entry point returns an ec_status; nothing throws across
 * the boundary.  On error the state is left unchanged (strong guarantee) and a
 * message is available from ec_last_error().  The calls that also return
 * energies after changing the state (ec_update_defect with E_out, ec_okmc_step)
 * are a change followed by an energies call: if the change succeeded and the
 * energies fail, the state holds the change and the error is returned.  The
 * self terms of a new list whose set-up cannot allocate are left to the next
 * energies call, which reports the failure.  Ownership: the caller owns every
 * pointer it passes in (defect records are copied during the call; output
 * buffers are written, never retained); the library owns every ec_ctx/ec_state
 * and the device memory behind them until the matching destroy call.
 * Streams: work is enqueued on the caller's HIP stream (a hipStream_t passed as
 * void*; NULL = the null stream).  Calls that return host data synchronise that
 * stream.  One host thread at a time may use a given ec_state; calls on one
 * state execute in call order.
 */
#ifndef EC_H
#define EC_H

/* The library is built with hidden symbols; these entry points are its only
 * exports. */
#define EC_API __attribute__((visibility("default")))

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ec_ctx ec_ctx;     /* one per device: allocator hooks, HBM ledger, cached Green windows */
typedef struct ec_state ec_state; /* one per replica: resident eps*, sigma (FP64), spectrum, footprints, energies */

typedef enum {
  EC_OK = 0,
  EC_ERR_ARG = 1,    /* invalid argument or invalid defect record */
  EC_ERR_SIZE = 2,   /* grid size not supported (see ec_problem.n) */
  EC_ERR_ADMIT = 3,  /* would exceed the context's HBM budget */
  EC_ERR_DEVICE = 4, /* HIP runtime or allocation failure */
  EC_ERR_STATE = 5   /* call out of order (e.g. energies before any solve) */
} ec_status;

typedef enum {
  EC_FP64 = 0, /* FP64 storage and arithmetic throughout */
  EC_FP32 = 1  /* FP32 storage of the spectra between passes; FP64 arithmetic in
                  registers, FP64 eigenstrain, resident stress and energies */
} ec_precision;

typedef enum {
  EC_MEAN_STRESS_ZERO = 0, /* xi = 0 bin: <eps> = <eps*>, so <sigma> = 0 (default) */
  EC_MEAN_STRAIN_ZERO = 1  /* xi = 0 bin: <eps> = 0 */
} ec_mean_bc;

typedef enum {
  EC_NYQ_PAPER = 0 /* even n: the centred label set of Sec. 3.4 with the real part
                      of the complex solution, i.e. the Green operator averaged over
                      the all -n/2 and all +n/2 representatives of a Nyquist bin */
} ec_nyquist;

/* Periodic cubic cell of n^3 voxels and side L, cubic stiffness C11, C12, C44.
 * frame: the crystal orientation, row-major 3x3 whose rows are the cell's x, y
 * and z axes as unit vectors in cube coordinates (the simulations of Secs. 4 and 6
 * take x = [111]/sqrt3, y = [-1-12]/sqrt6, z = [1-10]/sqrt2); all zeros for
 * cube axes along x, y, z.  Rows must be orthonormal to 1e-9 with determinant
 * +1 (EC_ERR_ARG otherwise).  Defects are given in cell coordinates either way.
 * n must be one of 8 16 24 32 45 48 64 96 128 129 160 240 256 512; anything
 * else gives EC_ERR_SIZE.  The odd sizes (45, and 129 = 3 x 43, the grid of the
 * simulations of Secs. 4 and 6) have no Nyquist bin: every centred label of Sec. 3.4
 * lies in -(n-1)/2 .. (n-1)/2, and minimum images lie in the same range. */
typedef struct {
  int32_t n;
  int32_t prec; /* ec_precision */
  int32_t bc;   /* ec_mean_bc */
  int32_t nyq;  /* ec_nyquist */
  double L;
  double C11, C12, C44;
  double frame[9];
} ec_problem;

typedef enum { EC_LOOP = 0, EC_SPHERE = 1 } ec_kind;

/* One defect (104 bytes).  Loops: centre c, in-plane radius, Burgers vector b,
 * habit normal (must be parallel to an integer lattice direction with
 * components up to 8), slab thickness (0 = one voxel h).  Eigenstrain
 * sym(b x n_hat)/e inside {|d.n_hat| in [-e/2, e/2), in-plane |d| <= radius}.
 * Spheres: eps* = eig_v * I inside {|d| <= radius}.  d is the minimum-image
 * offset of a voxel centre from c.  Membership is exact integer arithmetic on
 * coordinates quantised to h/1024.  Rejected (EC_ERR_ARG): radius <= 0,
 * |b| = 0, a normal that is not a small-integer direction, extent
 * radius (+ e/2 for loops) >= L/2, non-finite values. */
typedef struct {
  int32_t kind; /* ec_kind */
  int32_t reserved;
  double c[3];
  double radius;
  double b[3];
  double normal[3];
  double thickness;
  double eig_v;
} ec_defect;

/* Device-memory hooks.  alloc returns device memory usable on `stream` or NULL;
 * both may be NULL, in which case hipMalloc / hipFree are used. */
typedef void* (*ec_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*ec_free_fn)(void* p, void* stream, void* user);

/* Create a context on HIP device `device` with an HBM admission budget (bytes;
 * 0 = the device's free memory at creation).  Caches Green-kernel windows per
 * (n, C, bc). */
EC_API ec_status ec_ctx_create(int device, size_t hbm_budget_bytes, ec_alloc_fn alloc_fn, ec_free_fn free_fn,
                        void* user, ec_ctx** out);
/* Destroy every state of a context before the context itself. */
EC_API void ec_ctx_destroy(ec_ctx* ctx);

/* Bytes the context has admitted so far, and its budget. */
EC_API ec_status ec_ctx_ledger(const ec_ctx* ctx, size_t* used, size_t* budget);

/* Number of executable HIP graphs the context holds for batched hops
 * (ec_update_batch with use_graph on a non-null stream). */
EC_API ec_status ec_ctx_graphs(const ec_ctx* ctx, int32_t* count);

/* Thread-local text of the last error raised on this thread (never NULL). */
EC_API const char* ec_last_error(void);

/* Create a replica state for one problem; reserves its resident fields in the
 * ledger (EC_ERR_ADMIT if the budget would be exceeded). */
EC_API ec_status ec_state_create(ec_ctx* ctx, const ec_problem* problem, ec_state** out);
EC_API void ec_state_destroy(ec_state* st);

/* Bytes of device memory the state holds (fields, spectrum, footprints). */
EC_API ec_status ec_state_bytes(const ec_state* st, size_t* bytes);

/* Full solve (Sec. 3.2, 3.4): rasterise defs[0..ndef) (host array, copied),
 * Fourier-space Green solve, sigma = C:(eps - eps*) kept resident in FP64.
 * When nothing read the whole stress field since the state's previous solve,
 * the solve stores sigma only at the voxels the defects cover (all that the
 * energies read) and keeps the stress spectrum; the rest of the field is then
 * formed, bit for bit as a whole-field solve would have, by the first call that
 * needs it (field outputs, updates, jump probes, dipole energies, dislocations,
 * stored-type energies), on that call's stream.
 * Optional outputs eps_out / sig_out ([6][n^3], float for EC_FP32 states,
 * double for EC_FP64 states) on the device (out_on_device != 0) or on the host;
 * NULL skips them.  Replaces any previous defect list of the state. */
EC_API ec_status ec_solve_fields(ec_state* st, const ec_defect* defs, int32_t ndef, void* hip_stream, void* eps_out,
                          void* sig_out, int32_t out_on_device);

/* Per-defect interaction energies of the current defect list, in input order
 * (Sec. 2, Betti form written with the eigenstrain):
 *   E_i = sum_{j != i} E_ij,   E_ij = -h^3 c sum_x eps*_i(x) : sigma_j(x),
 * evaluated as -h^3 c E_i:S_i - B_i with S_i the FP64 compensated sum of the
 * resident stress over the footprint of i and B_i the exact discrete self term
 * (c = 1 GPa nm^3 in eV).  E_out holds ndef doubles (device or host). */
EC_API ec_status ec_interaction_energies(ec_state* st, void* hip_stream, double* E_out, int32_t out_on_device);

/* For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ec_interaction_energies
 * that allocates nothing.  E_dev is a device buffer of ndef doubles, written
 * on hip_stream without synchronising.  When the self terms must be computed
 * again (after an update that changed a footprint's shape), their work list,
 * per-defect offsets and partial sums live in a fixed scratch area of the
 * library on each device (about 6.3 MB, held until the process ends) instead
 * of state buffers; it serves at most 16384 defects and 262144 self-term work
 * items (EC_ERR_SIZE beyond).  The kernel and class windows must already cover
 * the list (EC_ERR_STATE otherwise: one ec_interaction_energies call builds
 * them).  Every call on one device shares the scratch area, so calls that
 * overlap on one device (other streams, other states or contexts) race. */
EC_API ec_status ec_interaction_energies_noalloc(ec_state* st, void* hip_stream, double* E_dev);

/* Move defect idx to the record *moved (Appendix B: subtract the old field,
 * add the new one).  By linearity only the eigenstrain difference is solved;
 * the resident FP64 stress is accumulated and, if E_out != NULL, all ndef
 * energies are returned as in ec_interaction_energies (an error there leaves
 * the move made). */
EC_API ec_status ec_update_defect(ec_state* st, int32_t idx, const ec_defect* moved, void* hip_stream, double* E_out,
                           int32_t out_on_device);

/* Several whole-voxel hops at once, one per state (Appendix B's move, as
 * ec_update_defect): states[k] are distinct solved states of one shape (the
 * same n, precision, stiffness and frame), idx[k] the moved defect of each and
 * moved[k] its record after the hop, a translation of its current record by
 * whole voxels (same shape and eigenstrain; any other move is EC_ERR_ARG: use
 * ec_update_defect).  The k hops run as one launch per pass over all k
 * replicas' data (batched persistent passes); with use_graph != 0 and a
 * non-null stream the launch sequence is captured once per (shape, k, stream)
 * in a HIP graph and replayed with the new hops (direct launches otherwise).  E_dev: NULL or k device buffers (NULL entries allowed) of
 * each state's ndef doubles, the energies after its hop; the states' own
 * energies are refreshed as ec_interaction_energies does.  Nothing is
 * synchronised; k in [1, 16].  Results are the same, bit for bit, as k calls
 * of ec_update_defect. */
EC_API ec_status ec_update_batch(ec_state* const* states, const int32_t* idx, const ec_defect* moved, int32_t k,
                                 void* hip_stream, double* const* E_dev, int32_t use_graph);

/* ---- stored defect types and the shift theorem (Sec. 3.3, eq. shift) ------ */

/* Store a defect type: the prototype *proto is rasterised at its own centre X0
 * (the reference position), and its eigenstrain spectrum eps*_hat_0(xi) and
 * stress spectrum sigma_hat_0(xi) (the Green step of the solve; at xi = 0 the
 * mean stress of the problem's mean condition) are kept on the device with the
 * state: two half spectra in the state's storage precision, charged to the
 * ledger (EC_ERR_ADMIT if they do not fit).  *type receives the type's index
 * (0, 1, ... in storing order, at most 64 per state).  Synchronises the stream. */
EC_API ec_status ec_type_store(ec_state* st, const ec_defect* proto, void* hip_stream, int32_t* type);

/* Interaction energies (eV, host array E_out of k doubles) of a defect of a
 * stored type translated to each of k positions X[3 p .. 3 p + 2] (nm, any real
 * values: whole-voxel offsets from X0 translate the voxel field exactly, others
 * give its trigonometric interpolation), with the state's resident stress
 * (its last solve or update):
 *   E_p = -h^3 c sum_x eps*_0(x - (X_p - X0)) : sigma_others(x),
 * the translated eigenstrain being the real part of the inverse transform of
 * exp(-i xi . (X_p - X0)) eps*_hat_0(xi) (centred labels of Sec. 3.4; at an even
 * n's Nyquist bins the phase is averaged over the -n/2 and +n/2 representatives).
 * sigma_others is the resident stress, minus, when X_excl is not NULL, the
 * type's own stress translated to X_excl (the moving defect itself, when the
 * state's list holds it there).  EC_ERR_STATE before the first solve.  The
 * resident stress is transformed once per call and the positions are taken
 * 16 per pass over the spectra; the state's work spectrum is overwritten.
 * Synchronises the stream. */
EC_API ec_status ec_type_energies(ec_state* st, int32_t type, const double* X, int32_t k, const double* X_excl,
                                  void* hip_stream, double* E_out);

/* ---- jump probes (the OkMC loop of App. B; biased jumps of Sec. 5) ---------- */

/* For every defect i and each of its njump (1..64) candidate whole-voxel jumps
 * jumps[(i*njump + j)*3 + {0,1,2}] (x, y, z offsets in voxels, |component| <= 8
 * and below half the cell; host array), the change of the defect's
 * interaction energy with all the other defects if it alone were translated
 * by that jump (eV):
 *   dE_ij = E_i(X_i + lambda_ij) - E_i(X_i),
 * from the resident stress and the defect's own field (a window of the
 * periodic kernel, grown to cover the jumps); nothing is moved.
 * dE_out: ndef*njump doubles, host or device (out_on_device), or NULL; the
 * values stay with the state for ec_jump_select until the next solve or
 * update.  Refreshes the energies as ec_interaction_energies does. */
EC_API ec_status ec_jump_energies(ec_state* st, const int32_t* jumps, int32_t njump, void* hip_stream,
                                  double* dE_out, int32_t out_on_device);

/* Biased jump frequencies of the last ec_jump_energies call,
 *   nu_ij = 1/2 nu0 exp(-(Em_i + dE_ij / 2) / kT)   (barrier raised by half
 * the energy change), and for each defect the jump on its frequency line
 * R_k = sum_{j <= k} nu_ij whose interval holds xi_i in (0, 1]: the first j
 * with xi_i <= R_j / R_tot.  Em, xi: ndef doubles (host; eV and the random
 * numbers drawn by the caller); nu0 in 1/s, kT in eV.  nu_out (ndef*njump
 * doubles) and choice_out (ndef int32) host or device (out_on_device), either
 * may be NULL (xi may be NULL when choice_out is).  EC_ERR_STATE when the
 * defect list changed since the jump energies were computed. */
EC_API ec_status ec_jump_select(ec_state* st, const double* Em, double nu0, double kT, const double* xi,
                                void* hip_stream, double* nu_out, int32_t* choice_out, int32_t out_on_device);

/* One time step of the parallel OkMC loop (Sec. 5 and App. B) on the solved
 * state.  Every defect draws its event count N_i over dt from the Poisson law
 * with its nominal frequency nu_i = nu0 exp(-Em_i / kT): N_i = 0 when
 * u_i <= exp(-nu_i dt).  Each defect with N_i > 0 takes one jump, chosen as in
 * ec_jump_select from its biased frequencies against the field at the start of
 * the step (all defects probed against the same field); the chosen jumps are
 * then made together and the field of the new positions solved.
 *   jumps: host int32 [ndef][njump][3] as in ec_jump_energies;
 *   Em, u, xi: host, ndef doubles each (u, xi in (0, 1]: the caller's random
 *   numbers for the gate and the selection);
 *   dt > 0 in s, or <= 0 for the paper's fixed step 1 / max_i nu_i;
 *   choice_out: host, ndef int32 (the jump index taken, -1 for none), or NULL;
 *   E_out: host, ndef doubles (energies after the step), or NULL.
 * The state's centres move by whole voxels in its quantised units, exactly;
 * the caller's record of defect i moves by h * jumps[i][choice_i].  Errors in
 * the arguments leave the state unchanged. */
EC_API ec_status ec_okmc_step(ec_state* st, const int32_t* jumps, int32_t njump, const double* Em, double nu0,
                              double kT, double dt, const double* u, const double* xi, void* hip_stream,
                              int32_t* choice_out, double* E_out);

/* ---- dislocation lines (Sec. 3.1, field dislocation mechanics) -------------- */

/* An infinite straight dislocation line along a cell axis (56 bytes): a point
 * p on it (nm, cell coordinates), the axis (0 = x, 1 = y, 2 = z), its sense
 * (+1 or -1 along the axis) and its Burgers vector b (nm, cell coordinates). */
typedef struct {
  double p[3];
  int32_t axis;
  int32_t sense;
  double b[3];
} ec_line;

/* Set the state's dislocation lines (nlines in [0, 64]; 0 removes them).  The
 * Burgers vector density of each one-voxel subsegment is spread to the four
 * grid points around the line (the eight around the subsegment midpoint, which
 * lies on a voxel-centre level); the Nye tensor alpha = b (x) t rho gives the
 * incompatible plastic distortion U_hat_ij = -i xi_k / xi^2 e_jkl alpha_hat_il
 * (xi != 0; straight lines have no compatible part), and sym(U) is solved as an
 * eigenstrain with the state's stiffness and frame.  The lines' stress is kept
 * as a background added to the resident stress of this and every later solve,
 * so energies, jump probes, dipole energies and OkMC steps include each
 * defect's interaction with the lines.  Lines must have |b| > 0, finite values,
 * axis in {0, 1, 2} and sense +-1 (EC_ERR_ARG otherwise). */
EC_API ec_status ec_set_dislocations(ec_state* st, const ec_line* lines, int32_t nlines, void* hip_stream);

/* A dislocation path (56 bytes): a closed polyline through vertices
 * verts[first .. first + count) (3 doubles each, nm, cell coordinates), the last
 * joined to the first shifted by `shift` (nm): zero for a loop (count >= 3), a
 * nonzero lattice vector of the cell (integer multiples of L per axis, |m| <= 64)
 * for a line through the periodic cell in any direction (count >= 1).  b is the
 * Burgers vector (nm); the line sense t runs along the vertex order. */
typedef struct {
  int32_t first;
  int32_t count;
  double shift[3];
  double b[3];
} ec_path;

/* Set the state's dislocation paths (npaths in [0, 256]; 0 removes them):
 * field dislocation mechanics in any direction (Sec. 3.1).  Every segment is
 * cut into the fewest equal pieces no longer than h, and each piece's Nye
 * tensor b (x) dl / h^3 is spread to the eight grid points around its midpoint
 * with trilinear weights; U_hat_ij = -i xi_k / xi^2 e_jkl alpha_hat_il at
 * xi != 0 (curl U^p = -alpha), and at xi = 0 the loops' compatible part, the
 * mean plastic distortion -b (x) A / V with A = 1/2 sum_j v_j x v_{j+1} the
 * vector area of a loop (a loop counterclockwise about n has the slipped-area
 * distortion -b (x) n; it changes the mean stress only under
 * EC_MEAN_STRAIN_ZERO).  sym(U^p) is solved as an eigenstrain with the state's
 * stiffness and frame, and the stress is kept as a background added to the
 * resident stress of this and every later solve, as for ec_set_dislocations
 * (both kinds may be present).  At most 2^20 pieces in all; finite values,
 * |b| > 0 (EC_ERR_ARG otherwise).  Synchronises the stream. */
EC_API ec_status ec_set_dislocation_paths(ec_state* st, const ec_path* paths, int32_t npaths, const double* verts,
                                          int32_t nverts, void* hip_stream);

/* ---- dipole-tensor approximation (Sec. 2.1) --------------------------------- */

/* Interaction energy of every defect in the dipole approximation (eV): the
 * field of the other defects taken as constant over the defect, at the voxel
 * that holds its centre x_c,
 *   E_i^dip = -P_i : eps_others(x_c) = -h^3 c m_i E_i : sigma_others(x_c),
 * with P_i = m_i h^3 C:E_i its dipole tensor (m_i footprint voxels) and
 * sigma_others = the resident stress minus the defect's own (from the kernel
 * window), for comparison with the exact energies of ec_interaction_energies.
 * E_out: ndef doubles, host or device (out_on_device). */
EC_API ec_status ec_dipole_energies(ec_state* st, void* hip_stream, double* E_out, int32_t out_on_device);

/* ---- inspection (tests, benchmarks) ---------------------------------------- */

/* Footprints of the current defect list: counts[ndef] and, if ids != NULL, the
 * concatenated voxel ids in defect order (each defect's ids ascending after a
 * full solve).  Host buffers; synchronises.  *total receives the id count. */
EC_API ec_status ec_state_footprints(ec_state* st, int32_t* counts, int32_t* ids, int64_t ids_capacity, int64_t* total);

/* Copy a resident field to a host buffer of 6*n^3 doubles, component-major
 * [6][n^3] like every field this interface hands out (the resident stress is
 * kept voxel-major and converted): which = 0 sigma, 1 eps (total strain),
 * 2 eps* (eigenstrain). Synchronises. */
EC_API ec_status ec_state_field(ec_state* st, int32_t which, double* host_out);

/* Self terms B_i (eV) of the current defect list, host buffer of ndef doubles. */
EC_API ec_status ec_state_self_terms(ec_state* st, double* host_out);

/* Kernel timing: when enabled, HIP events bracket every kernel the state
 * launches; ec_profile_read returns, per kernel family, the launch count,
 * summed milliseconds and the algorithmic bytes moved per launch.  Families:
 * 0 raster, 1 x-forward, 2 y-pass, 3 z-pass (fused with the Green operator),
 * 4 x-inverse + stress, 5 energy reduction, 6 self term, 7 other. */
#define EC_NPROF 8
EC_API ec_status ec_profile_enable(ec_state* st, int32_t on);
/* Families timed while profiling is enabled: bit f of family_mask for family
 * f (every family by default), so that a caller can time one family without
 * the events of the others in its stream; other bits: EC_ERR_ARG. */
EC_API ec_status ec_profile_select(ec_state* st, int32_t family_mask);
EC_API ec_status ec_profile_read(ec_state* st, int64_t* launches, double* ms, double* bytes_per_launch);

/* ---- kernel-level entry points (parity tests of single passes) -------------- */

/* Forward transform of a real [6][n^3] FP64 host field with this state's
 * kernels: writes the half spectrum [6][n][n][n/2+1] complex128 (interleaved
 * re, im; unnormalised forward DFT) to host_out. */
EC_API ec_status ec_debug_forward(ec_state* st, const double* host_field, double* host_out);

/* Green step alone: host half spectrum of eps* ([6][n][n][n/2+1] complex128)
 * in, half spectrum of sigma = S(xi):eps*_hat out (S = C Gamma C - C, zero at
 * xi = 0), with the state's Nyquist rule. */
EC_API ec_status ec_debug_green(ec_state* st, const double* host_spec_in, double* host_spec_out);

/* Inverse transform of a host half spectrum to a real [6][n^3] host field
 * (scaled by 1/n^3, imaginary parts of the kx = 0 and n/2 planes dropped). */
EC_API ec_status ec_debug_inverse(ec_state* st, const double* host_spec, double* host_out);

#ifdef __cplusplus
}
#endif

#endif /* EC_H */
