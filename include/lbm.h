/*
 * liblbm -- fused lattice-Boltzmann BGK collide-stream step with the enhanced
 * local interpolated bounce-back (ELIBB) boundary condition of Marson,
 * Thorimbert, Latt & Chopard, "Enhanced single-node boundary condition for the
 * Lattice Boltzmann Method" (arXiv 2009.04604), for AMD Instinct MI355X (gfx950).
 *
 * Conventions used by every call
 * ------------------------------
 * - Lattice units throughout.  Node index n = x + nx * (y + ny * z),
 *   0 <= x < nx, 0 <= y < ny, 0 <= z < nz (nz == 1 for D2Q9).
 * - Direction order (Sec. II.A uses the standard velocity sets):
 *     D2Q9   0:(0,0) 1:(1,0) 2:(-1,0) 3:(0,1) 4:(0,-1) 5:(1,1) 6:(1,-1) 7:(-1,1) 8:(-1,-1)
 *     D3Q19  0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..10 = (+-1,+-1,0); 11..14 = (+-1,0,+-1);
 *            15..18 = (0,+-1,+-1); each group in sign order (+,+),(+,-),(-,+),(-,-).
 *     D3Q27  0..18 as D3Q19; 19..26 = the corners (+-1,+-1,+-1) in sign order
 *            (+,+,+),(+,+,-),(+,-,+),(+,-,-),(-,+,+),(-,+,-),(-,-,+),(-,-,-).
 * - Population arrays exchanged with the host are [Q][N] float64, N = nx*ny*nz.
 * - Host pointers passed in are caller-owned and only read (or written) during
 *   the call.  Device memory is library-owned unless the caller hands an arena.
 * - Every call returns LBM_OK (0) or a negative code; lbm_last_error() then
 *   gives a message for the calling thread.  A failed call leaves the domain as
 *   it was, except where stated.
 * - All device work is enqueued on the domain's stream (a hipStream_t, e.g.
 *   torch.cuda.current_stream().cuda_stream); only calls that return data to
 *   the host synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid argument; nothing was changed                  */
  LBM_ENOMEM = -2,    /* device or host allocation failed                       */
  LBM_EDEVICE = -3,   /* HIP runtime error (no device, launch failure, ...)     */
  LBM_EUNSTABLE = -4, /* NaN/Inf in the populations (returned by lbm_macros)    */
  LBM_ESTATE = -5     /* call not valid in the domain's current state           */
};

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1, LBM_D3Q27 = 2 };

/* Collision models (Sec. II.A): BGK (eq. LB-BGK) or TRT (TRT models paragraph).
 * With a body force, Guo's source term is split like the populations under TRT:
 * (1 - omega+/2) on its symmetric and (1 - omega-/2) on its antisymmetric part. */
enum { LBM_BGK = 0, LBM_TRT = 1 };

/* Storage of the populations.  Collision arithmetic is FP64 for LBM_F64 and
 * FP32 for the others; the 16-bit forms store h_i = f_i - w_i rounded as
 * lbm_domain_desc.rounding says and convert back to FP32 on load. */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16_SHIFTED = 2, LBM_BF16_SHIFTED = 3 };

/* Rounding of the 16-bit stores of the node update (lbm_domain_desc.rounding).
 * LBM_ROUND_NEAREST: to nearest even.  LBM_ROUND_STOCHASTIC: up or down with
 * probabilities proportional to the distances, so the rounding error has zero
 * mean; a per-step change of a population smaller than half a unit in the last
 * place then survives on average instead of being discarded every step, which
 * is what stalls a slowly converging flow stored in BF16 (stochastic rounding
 * against this stagnation: Croci and Giles, IMA J. Numer. Anal. 2022, on the heat
 * equation in low precision).  The random bits come from a counter-based hash
 * of the node's slot and the domain's own step count, so results are
 * deterministic and the same for a domain stepped alone or in a batch.  Only
 * for the 16-bit storages; initial and imported states round to nearest. */
enum { LBM_ROUND_NEAREST = 0, LBM_ROUND_STOCHASTIC = 1 };

/* Boundary variants (Sec. II.D).  ELIBB-FQ is the default.  UQ and FQ fall back
 * to ELIBB-F below q_cutoff.  LBM_HWBB is half-way bounce-back with Ladd's
 * moving-wall term (eq. ME-solid-to-fluid). */
enum { LBM_ELIBB_FQ = 0, LBM_ELIBB_F = 1, LBM_ELIBB_UQ = 2, LBM_ELIBB_U = 3, LBM_HWBB = 4 };

/* Estimators of the non-equilibrium part of the wall populations (Sec. II,
 * approximation of the wall populations; App. C): the bounced non-equilibrium
 * of the boundary node (eq. neqbb-s, the default), or the regularised one
 * rebuilt from the node's non-equilibrium stress and the wall velocity
 * (eq. fi_neq). */
enum { LBM_NEQ_BOUNCEBACK = 0, LBM_NEQ_REGULARIZED = 1 };

/* Domain faces: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z. */
enum { LBM_FACE_NONE = -1 };

typedef struct lbm_domain_s* lbm_domain;

typedef struct {
  int32_t lattice;       /* LBM_D2Q9, LBM_D3Q19 or LBM_D3Q27                          */
  int32_t nx, ny, nz;    /* lattice size; nz must be 1 for D2Q9                       */
  int32_t periodic;      /* bit0 x, bit1 y, bit2 z                                    */
  int32_t storage;       /* LBM_F64 / LBM_F32 / LBM_F16_SHIFTED / LBM_BF16_SHIFTED    */
  double tau;            /* BGK relaxation time tau = taubar + 1/2 (eq. LB-BGK), > 0.5 */
  double force[3];       /* constant body-force density (Guo forcing); zeros = off    */
  double rho0, u0[3];    /* initial equilibrium state                                 */
  int32_t outlet_face;   /* face with zero-gradient outflow, or LBM_FACE_NONE; must be
                            on a non-periodic axis                                     */
  void* stream;          /* hipStream_t for all device work; NULL = default stream     */
  void* arena;           /* optional caller-owned device memory for the two population
                            buffers (>= lbm_arena_bytes(desc, mask) bytes, 256-byte
                            aligned); NULL = the library allocates them               */
  size_t arena_bytes;
  int32_t layout;        /* LBM_LAYOUT_COMPACT (default): only fluid nodes are stored;
                            LBM_LAYOUT_DENSE: every node (plus a halo layer on
                            non-periodic axes)                                          */
  int32_t collision;     /* LBM_BGK (default) or LBM_TRT                               */
  double magic;          /* TRT magic parameter Lambda > 0 (eq. magic-parameter):
                            omega+ = 1/tau relaxes the symmetric parts,
                            omega- with (1/omega+ - 1/2)(1/omega- - 1/2) = Lambda the
                            antisymmetric parts; the paper uses 3/16.  Ignored by BGK. */
  int32_t rounding;      /* LBM_ROUND_NEAREST (default) or LBM_ROUND_STOCHASTIC
                            (16-bit storages only)                                     */
} lbm_domain_desc;

enum { LBM_LAYOUT_COMPACT = 0, LBM_LAYOUT_DENSE = 1 };

/* Bytes of the two population buffers of a domain (what an arena must hold).
 * fluid_mask (host, N bytes) is needed for the compact layout; NULL gives the
 * dense-layout size, an upper bound. */
size_t lbm_arena_bytes(const lbm_domain_desc* d, const uint8_t* fluid_mask);

/* Create a domain (Sec. II.A lattice, eq. LBE).  fluid_mask: host, N bytes, 1 =
 * fluid node, 0 = solid.  All fluid nodes start at f^eq(rho0, u0) (eq.
 * Eq2ndOrder).  Faces on non-periodic axes are walls or the outlet; every
 * population they leave missing must be covered by lbm_set_boundary_links
 * before the first step.  Errors: LBM_EINVAL (sizes, among them 2^31 or more
 * stored nodes per population array, tau <= 0.5, enum values, outlet face on a
 * periodic axis; all checked before any device call), LBM_ENOMEM, LBM_EDEVICE. */
int lbm_init_domain(const lbm_domain_desc* d, const uint8_t* fluid_mask, lbm_domain* out);

/* Install the cut-link list (replaces any previous list) -- Sec. II.B-E.
 * A link (node, dir) names the population f_dir that is missing at the fluid
 * boundary node `node` after streaming, because node - c_dir is solid or lies
 * beyond a non-periodic face.  Its f_dir(x_F, t+1) is rebuilt by eq.
 * ELIBB-general from the node's own time-t data:
 *   q      (0, 1]: |x_W - x_F| / |c_dir|, x_W the first wall crossing
 *   uw_t   [3*n] wall velocity at x_W at time t (NULL: wall at rest)
 *   uw_t1  [3*n] wall velocity at x_W at time t+1 (NULL: equal to uw_t)
 * Velocity triples are (x, y, z) per link; z ignored for D2Q9.
 * Validation (LBM_EINVAL, message names the first offending link): node is a
 * fluid node; 1 <= dir < Q; node - c_dir is not a fluid node; the pair is not
 * covered by the outlet; 0 < q <= 1; no duplicate (node, dir); every missing
 * population of every fluid node is covered by a link or by the outlet; variant
 * in range; q_cutoff >= 0 (the paper uses 0.01).  Host arrays are copied. */
int lbm_set_boundary_links(lbm_domain d, int64_t n_links, const int64_t* node, const int8_t* dir,
                           const double* q, const double* uw_t, const double* uw_t1,
                           int32_t variant, double q_cutoff);

/* Selects the wall non-equilibrium estimator of every cut link of the domain
 * (eq. ELIBB-approximations).  LBM_NEQ_BOUNCEBACK: f_i^neq(x_W) is taken as the
 * bounced non-equilibrium f_ibar - f^eq_ibar of the boundary node F (eq.
 * neqbb-s), pre-collision for the wall population at t+1 and post-collision for
 * the post-collision one.  LBM_NEQ_REGULARIZED: f_i^neq(x_W) is the third-order
 * Hermite reconstruction of eq. fi_neq,
 *   w_i [ 9/2 H_i2 : Pi + 27/2 H_i3 : (u_w Pi) ]  (c_s^2 = 1/3),
 * with Pi the non-equilibrium stress sum_j c_j c_j (f_j - f^eq_j) of node F
 * (the stress at the wall taken as the stress at F) -- before collision, with
 * u_w(t+1), for the wall population at t+1; after collision, with u_w(t), for
 * the post-collision one.  Takes effect from the next step and stays when the
 * links are replaced.  Any lattice, storage, collision and layout; for a moving
 * sphere it must be chosen before lbm_set_moving_sphere.  Errors: LBM_EINVAL for
 * an unknown mode, LBM_ESTATE on a domain that already has a moving sphere. */
int lbm_set_wall_neq(lbm_domain d, int32_t mode);

/* A rigid sphere in prescribed motion (Sec. II.E moving boundaries): centre
 * x_c(t) = x0 + amplitude sin(2 pi t / period) direction, translational velocity
 * V(t) = amplitude (2 pi / period) cos(2 pi t / period) direction, constant
 * angular velocity omega.  Before every step t -> t+1 the library rebuilds on the
 * device the fluid mask and the cut links of the sphere at time t (q by the exact
 * ray-sphere intersection, u_w(t) = V(t) + omega x (x_W - x_c(t)),
 * u_w(t+1) = V(t+1) + omega x (x_W - x_c(t))), and refills nodes that were solid
 * at t-1 and are fluid at t with f^eq(rho_bar, V(t) + omega x (x - x_c(t))),
 * rho_bar the mean density of their neighbours fluid at t-1 and t (rho0 if none).
 * The LIR refill of the paper is not reproduced (its algorithm is only in a
 * figure); this equilibrium refill replaces it.  Requirements (LBM_ESTATE
 * otherwise): dense layout, no outlet, an all-fluid initial mask, no links and
 * no step taken yet.  The state is reset to f^eq(rho0, u0) on the fluid nodes of
 * time 0. */
int lbm_set_moving_sphere(lbm_domain d, const double x0[3], double radius, double amplitude, double period,
                          const double direction[3], const double omega[3], int32_t variant, double q_cutoff);

/* The same rigid sphere (Sec. II.E moving boundaries) on a prescribed path of
 * any form: sample k (k = 0 .. n_samples-1, host arrays [n_samples][3], (x, y,
 * z), copied) gives the centre x_c(k) and the translational velocity V(k) at
 * step k; omega is the constant angular velocity.  The geometry of time t is
 * built from x_c(t), V(t) and V(t+1) exactly as for lbm_set_moving_sphere, so
 * the domain can take n_samples - 2 steps in all; lbm_step and lbm_batch_step
 * refuse (LBM_ESTATE) a call that would step past the path.  The sampled
 * centres of lbm_set_moving_sphere's sinusoid reproduce it to the bit.  The
 * sweep region is the samples' bounding box grown by the radius.  Requirements
 * as for lbm_set_moving_sphere (LBM_ESTATE); LBM_EINVAL for n_samples < 2, a
 * non-positive radius, non-finite samples, or a sweep that does not fit in half
 * the box on some axis. */
int lbm_set_moving_sphere_path(lbm_domain d, double radius, const double omega[3], int64_t n_samples,
                               const double* centre, const double* velocity, int32_t variant, double q_cutoff);

/* The same, with the angular velocity sampled too (omega: host array
 * [n_samples][3], copied): the geometry of time t takes the wall velocities
 * u_w(t) = V(t) + Omega(t) x r and u_w(t+1) = V(t+1) + Omega(t+1) x r at each
 * link's wall point (r from the centre at t), the refill and the force the
 * rigid-body velocity V(t) + Omega(t) x r.  Constant samples reproduce
 * lbm_set_moving_sphere_path to the bit.  Errors as lbm_set_moving_sphere_path
 * (LBM_EINVAL also for a non-finite Omega sample). */
int lbm_set_moving_sphere_motion(lbm_domain d, double radius, int64_t n_samples, const double* centre,
                                 const double* velocity, const double* omega, int32_t variant, double q_cutoff);

/* Several rigid spheres (1 .. 4) in prescribed motion in one domain (Sec. II.E
 * moving boundaries), each as in lbm_set_moving_sphere_motion: radius[s], and
 * per sample k and sphere s the centre, translational velocity and angular
 * velocity at [k][s][0..2] of centre, velocity, omega (host arrays
 * [n_samples][n_spheres][3], copied).  A node is solid when it lies in or on any
 * sphere; a cut link takes the first crossing over the spheres (the first
 * sphere in the list wins a tie) and that sphere's wall velocities; a fresh
 * node takes the rigid-body velocity of the sphere whose surface is nearest.
 * The sweep region is the union of the spheres' sweep boxes.  The surfaces must
 * stay more than two nodes apart at every sample (LBM_EINVAL otherwise, naming
 * the pair and the sample).  Force tracking gives one force and torque per
 * sphere (lbm_moving_forces).  Other errors as lbm_set_moving_sphere_motion. */
int lbm_set_moving_spheres(lbm_domain d, int32_t n_spheres, const double* radius, int64_t n_samples,
                           const double* centre, const double* velocity, const double* omega, int32_t variant,
                           double q_cutoff);

/* Advance n_steps >= 0 time steps; asynchronous on the domain's stream.  Each
 * step is the lattice Boltzmann equation of Sec. II.A (eq. LBE) split into the
 * local collision -- BGK (eq. LB-BGK) with the second-order equilibrium (eq.
 * Eq2ndOrder), or TRT (eq. magic-parameter), plus Guo's force term when a body
 * force is set -- and the exact pull streaming f_i(x, t+1) = f*_i(x - c_i, t);
 * then every cut link is rebuilt from its boundary node's own time-t data by the
 * enhanced single-node bounce-back of Sec. II.C-E (eq. ELIBB-general with the
 * variant's weights of eq. poli_coeff and the moving-wall term of eq.
 * ME-solid-to-fluid).  With a moving sphere the geometry of the next step is
 * rebuilt after each step.  LBM_EINVAL for n_steps < 0, LBM_ESTATE if links are
 * missing, LBM_EDEVICE if a launch fails. */
int lbm_step(lbm_domain d, int32_t n_steps);

/* Moments of the current pre-collision state (time t), Sec. II.A: rho = sum_i
 * f_i and rho u = sum_i c_i f_i (+ F/2 with Guo forcing), as rho [N] and u [N*D]
 * (node-major: u[n*D + a]) -- solid nodes get 0 -- and sums = {mass, mom_x,
 * mom_y, (mom_z), residual} summed over fluid nodes in FP64 in a fixed order
 * (same result every call for the same state).  The mass is the quantity whose
 * drift Sec. III.B measures (mean density fluctuation); the residual is the
 * relative L2 change of the velocity field in the form of eq. rRMSE,
 * ||u - u_prev|| / ||u|| over fluid nodes, with u_prev the field of the
 * previous lbm_macros call (the initial field for the first call): called
 * every k steps it is the residual at lag k.  Any pointer may be NULL (all
 * host, caller-owned).  Synchronises the stream.  Returns LBM_EUNSTABLE if a
 * NaN/Inf was found in rho or u (outputs are still written), LBM_ENOMEM /
 * LBM_EDEVICE on allocation or device errors. */
int lbm_macros(lbm_domain d, double* rho, double* u, double* sums);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the moments and FP64 sums of
 * lbm_macros with no allocation, no host transfer and no synchronisation.
 * rho [N], u [N*D] (node-major; either may be NULL) and sums [8] are DEVICE
 * pointers owned by the caller; everything is enqueued on the domain's stream
 * and is complete when that stream is.  sums = {mass, mom_x, mom_y, mom_z, 0,
 * sum |u|^2, number of fluid nodes with a NaN/Inf moment, 0} (mom_z = 0 for
 * D2Q9; no residual: its previous field would need N*D doubles of storage).
 * The block partial sums live in a 64 KiB file-scope device array (one per
 * GPU, held until the process ends; any lattice size fits, the kernel walks
 * the lattice with at most 1024 workgroups), so calls that overlap on one GPU
 * (several streams, several threads) race on it and must be serialised by the
 * caller.  Field values are identical to lbm_macros'; the sums agree to
 * rounding (another summation tree).  Errors: LBM_EINVAL for a null domain or
 * sums, LBM_EDEVICE when the scratch address could not be found on the
 * domain's device or a launch fails. */
int lbm_macros_noalloc(lbm_domain d, double* rho, double* u, double* sums);

/* Export / import the pre-collision populations f_i(x, t) as [Q][N] float64
 * (solid nodes read as 0 and are ignored on import).  For 16-bit storage the
 * import rounds to the storage format.  At a zero-gradient outlet an inward
 * population equals, by construction, the same population one node upstream;
 * on import that upstream value is kept.  Both synchronise the stream. */
int lbm_get_state(lbm_domain d, double* f);
int lbm_set_state(lbm_domain d, const double* f);

/* Groups of cut links for lbm_momentum_exchange (e.g. one per object): group[k]
 * in [0, n_groups) for the k-th link in the order given to
 * lbm_set_boundary_links; group NULL with n_groups = 1 puts every link in one
 * group (the default).  Host array copied.  LBM_ESTATE without a static link
 * list (moving sphere), LBM_EINVAL for ids out of range or n_groups outside
 * [1, 4096].  Installing new links resets the grouping. */
int lbm_set_link_groups(lbm_domain d, const int32_t* group, int32_t n_groups);

/* Force exerted by the fluid on each group of walls during the last step (Sec.
 * II "Force computation": the Galilean-invariant momentum exchange), summed in
 * FP64 in a fixed order over the group's links (x_F, i):
 *   F = (c_ibar - u_w) f*_ibar(x_F, t-1) - (c_i - u_w) f_i(x_F, t),
 * t the current time, u_w the link's wall velocity at t (uw_t of the links),
 * f*_ibar the post-collision population leaving x_F towards the wall and f_i the
 * rebuilt one.  force: n_groups x 3 doubles (z = 0 for D2Q9), caller-owned.
 * Synchronises the stream.  LBM_ESTATE for a moving-sphere domain, without
 * links, or before the first step after the links or the state were installed. */
int lbm_momentum_exchange(lbm_domain d, double* force);

/* Force and torque on each group of walls during the last step: the forces of
 * lbm_momentum_exchange, and the torque T = sum over the group's links of
 * r x F_link, r = x_W - centre[group] taken as the minimum image on periodic
 * axes, x_W = x_F - q c_i the link's wall point (the paper's force section names
 * the torque without fixing its lever arm; the wall point is where the link's
 * momentum exchange acts).  centres: n_groups x 3 doubles (NULL: the origin);
 * force, torque: n_groups x 3 doubles, caller-owned (torque is along z for
 * D2Q9).  Same errors as lbm_momentum_exchange. */
int lbm_force_torque(lbm_domain d, const double* centres, double* force, double* torque);

/* Force and torque on a moving sphere (lbm_set_moving_sphere), Sec. II "Force
 * computation": its links are rebuilt every step, so the momentum exchange of a
 * step must be taken before the rebuild.  With tracking on (on = 1), every
 * lbm_step call evaluates, after its last step and over the links of the
 * geometry that step used (time t),
 *   F = sum (c_ibar - u_w) f*_ibar(x_F, t) - (c_i - u_w) f_i(x_F, t+1),
 *   T = sum r x F_link,  r = x_W - x_c(t) (minimum image), x_W = x_F - q c_i,
 * u_w = V(t) + omega x r, summed in FP64 in a fixed order; lbm_moving_force
 * copies the result out (force, torque: 3 doubles each, caller-owned;
 * synchronises the stream).  With several spheres (lbm_set_moving_spheres)
 * each link counts for the sphere that holds its solid node, with that
 * sphere's x_c, V and omega, and lbm_moving_forces copies n_spheres (the
 * domain's count, LBM_EINVAL otherwise) forces and torques out as
 * [n_spheres][3] each; lbm_moving_force is the one-sphere form (LBM_EINVAL
 * with several).  Batched steps (lbm_batch_step) do not evaluate it.
 * Errors: LBM_ESTATE without a moving sphere, with tracking off, or when the
 * last step was not taken by lbm_step with tracking on; LBM_ENOMEM when the
 * per-link scratch cannot be allocated (done by lbm_set_force_tracking). */
int lbm_set_force_tracking(lbm_domain d, int32_t on);
int lbm_moving_force(lbm_domain d, double* force, double* torque);
int lbm_moving_forces(lbm_domain d, int32_t n_spheres, double* force, double* torque);

/* Change the stream used by later calls. */
int lbm_set_stream(lbm_domain d, void* stream);

/* Launch options (no effect on results): LBM_OPT_XCD_REMAP = 1 deals the
 * workgroups so that each of the 8 XCDs walks a contiguous range of rows
 * (neighbouring rows then share an L2); 0 keeps the hardware round-robin.
 * Default: 1 for the compact layout, 0 for the dense one. */
enum { LBM_OPT_XCD_REMAP = 0 };
int lbm_set_launch_option(lbm_domain d, int32_t option, int32_t value);

typedef struct {
  int64_t n_nodes, n_fluid, n_boundary_nodes, n_links;
  int64_t population_bytes;   /* both buffers                         */
  int64_t link_bytes;         /* boundary-node and link records       */
  int64_t steps_done;
  int32_t q, storage;
} lbm_domain_info;

int lbm_get_info(lbm_domain d, lbm_domain_info* info);

/* Release every resource of the domain (does not free a caller arena). */
int lbm_free_domain(lbm_domain d);

/* ---------------------------------------------------------------------------
 * Batched stepping: many domains of different sizes advance together.  Per
 * step there is one persistent multi-domain launch for each group of domains
 * that share lattice, storage and layout, followed by the batched rebuild of
 * the moving spheres among them; the launches of two steps are captured once
 * into a HIP graph and replayed.  Every node's arithmetic is the same as in
 * lbm_step, so results are bit-identical to stepping each domain alone, for
 * every launch choice.
 * ------------------------------------------------------------------------- */
typedef struct lbm_batch_s* lbm_batch;

/* stream: the stream of every member domain (NULL = default stream). */
int lbm_batch_create(void* stream, lbm_batch* out);

/* Advance each of the n domains by n_steps >= 0 (asynchronous on the stream,
 * like lbm_step).  Every domain must have its links or moving sphere set, use the
 * batch's stream and appear once (LBM_EINVAL / LBM_ESTATE otherwise).  A call
 * with another membership than the previous one synchronises the stream first.
 * With LBM_BATCH_AUTOTUNE on and no tuned choice for this batch's shape class,
 * the first 49 steps of the call run the autotuner (and still count as steps). */
int lbm_batch_step(lbm_batch b, const lbm_domain* ds, int32_t n, int32_t n_steps);

/* Launch choices (no effect on results):
 *   LBM_BATCH_GRAPH     1 (default) replay captured step pairs, 0 eager launches
 *   LBM_BATCH_GRID      0 one workgroup per tile of 4 row segments; k > 0 a
 *                       persistent grid of k workgroups per compute unit; -1 tuned
 *   LBM_BATCH_ORDER     0 tiles in call order; 1 the same, each XCD given a
 *                       contiguous share; 2 largest domain first, XCD shares; -1 tuned
 *   LBM_BATCH_AUTOTUNE  1 tune automatically in lbm_batch_step, 0 (default) not */
enum { LBM_BATCH_GRAPH = 0, LBM_BATCH_GRID = 1, LBM_BATCH_ORDER = 2, LBM_BATCH_AUTOTUNE = 3 };
int lbm_batch_set_option(lbm_batch b, int32_t option, int32_t value);

/* Autotuner: one warm-up step, then every (grid in {0, 2, 4, 6}) x (order in {0,
 * 1, 2}) candidate runs steps_per_candidate real steps (the domains advance by
 * 1 + 12 steps_per_candidate in total) timed with HIP events; the fastest is
 * kept for the shape class (lattice, storage, layout, log2 of the tile count)
 * and used by later calls unless an option forces another.  Synchronises. */
int lbm_batch_autotune(lbm_batch b, const lbm_domain* ds, int32_t n, int32_t steps_per_candidate);

/* Launch choice of the first group and the autotuner's best time per step (us). */
int lbm_batch_get_choice(lbm_batch b, int32_t* grid, int32_t* order, double* us_per_step);

/* Synchronises the stream and releases the batch (not its domains). */
int lbm_batch_free(lbm_batch b);

/* One-shot form: a temporary batch on ds[0]'s stream, eager launches;
 * synchronises. */
int lbm_step_batch(const lbm_domain* ds, int32_t n, int32_t n_steps);

/* Bandwidth calibration (not part of the method): copy `arrays` FP32 arrays of
 * n elements from src to dst (device pointers, caller-owned, arrays of
 * `stride` elements laid one after another), element e of each array at
 * offset shift + e; one element of every array per lane, 64-lane waves over 64
 * consecutive elements, as the step kernel's population streams; for 9, 19
 * and 27 arrays a lane issues all its loads before its stores.  shift 0:
 * every wave's run starts on a 256 B boundary (if src and dst are 256 B
 * aligned); 1..31: every run straddles cache lines.  Asynchronous on stream.
 * The caller times it; read + write bytes = 2 * 4 * n * arrays.  LBM_EINVAL
 * unless n >= 0, arrays >= 1, 0 <= shift < 64 and stride >= n + shift. */
int lbm_stream_probe(const float* src, float* dst, int64_t n, int64_t stride, int32_t arrays, int32_t shift,
                     void* stream);

/* Thread-local message of the last failed call ("" if none). */
const char* lbm_last_error(void);

/* ---------------------------------------------------------------------------
 * Host geometry builder: fluid mask and cut links with exact intersections
 * (Sec. II.B: q = |x_W - x_F| / |c_i|, first wall crossing along the link).
 * A node is fluid iff it is strictly inside the fluid region; a node exactly
 * on a wall is solid (its neighbours get q = 1).
 * ------------------------------------------------------------------------- */
typedef struct lbm_geometry_s* lbm_geometry;

int lbm_geometry_create(int32_t lattice, int32_t nx, int32_t ny, int32_t nz, int32_t periodic,
                        int32_t outlet_face, lbm_geometry* out);
/* Sphere (3D) or disk (D2Q9, centre z ignored): solid inside (solid_inside=1) or
 * outside.  Wall velocity u_w = V + Omega x (x_W - centre) (minimum image on
 * periodic axes).  V, Omega may be NULL (zero). */
int lbm_geometry_add_sphere(lbm_geometry g, const double centre[3], double radius, int32_t solid_inside,
                            const double V[3], const double Omega[3]);

/* Circular cylinder of infinite extent along z, its axis through centre (the
 * cylindrical Couette geometry of Sec. III.B on a 3D lattice): the sphere's
 * rules with distances taken in the xy-plane; wall velocity
 * u_w = V + Omega x r, r the xy-offset of x_W from the axis.  A link along z never
 * crosses it.  On D2Q9 it is the disk.  LBM_EINVAL for a null geometry or centre,
 * a radius that is not finite and > 0, or a non-finite centre or motion. */
int lbm_geometry_add_cylinder(lbm_geometry g, const double centre[3], double radius, int32_t solid_inside,
                              const double V[3], const double Omega[3]);
/* n >= 0 solid-inside spheres at rest: centres [3n], radii [n]. */
int lbm_geometry_add_spheres(lbm_geometry g, int64_t n, const double* centres, const double* radii);
/* Plane wall parallel to a non-periodic face at distance q_face in (0, 1] from
 * the first node layer.  Wall velocity uw (NULL = rest); profile 1 scales it by
 * 4 (y + 1/2)(ny - 1/2 - y) / ny^2 at the wall point (parabolic inlet across y).
 * LBM_EINVAL for a face on a periodic axis, q_face outside (0, 1], a profile
 * other than 0 or 1, or a non-finite velocity. */
int lbm_geometry_add_face_wall(lbm_geometry g, int32_t face, double q_face, const double uw[3],
                               int32_t profile);

/* Classify nodes and find every cut link.  Outputs counts. */
int lbm_geometry_build(lbm_geometry g, int64_t* n_fluid, int64_t* n_links);
/* Copy the results of lbm_geometry_build: mask [N]; node, dir, q [n_links];
 * uw_t, uw_t1 [3*n_links] (any may be NULL). Links are ordered by node, dir. */
int lbm_geometry_get(lbm_geometry g, uint8_t* mask, int64_t* node, int8_t* dir, double* q,
                     double* uw_t, double* uw_t1);
/* Owner of each link (n_links int32, same order): the index of the sphere in
 * order of addition, or (number of spheres + index of the face wall).  shape
 * may be NULL when there are no links. */
int lbm_geometry_get_shapes(lbm_geometry g, int32_t* shape);
int lbm_geometry_free(lbm_geometry g);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
