/*
 * rtmm.h -- C ABI of the MI355X radiation-step library (librtmm.so).
 *
 * The library advances the specific intensities of discrete-ordinates
 * radiative transfer in the reduced-speed-of-light approximation on a periodic
 * Voronoi mesh, as in Chang, Davis & Jiang, "Time Dependent Radiation
 * Hydrodynamics on a Moving Mesh": transport written as a finite-volume
 * conservation law with per-face, per-angle upwind fluxes in the frame of the
 * moving face (section 2.2), followed by the per-cell implicit source update
 * that couples every angle to the gas energy and momentum (section 2.3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Return value: RT_OK (0) or a negative RT_E* code.  rt_strerror() names a
 *    code; rt_last_error() returns the message of the calling thread's last
 *    failing call.  Nothing throws or exits across this ABI.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = null stream).
 *    Step calls only enqueue work on it: they never synchronise and never
 *    allocate; scratch is sized when the mesh is uploaded.  rt_mesh_upload,
 *    rt_mesh_free and rt_diagnostics synchronise `stream`.
 *  - Memory: "device" pointers are HIP device memory owned by the caller,
 *    contiguous, at least 8-byte aligned; "host" pointers are host memory read
 *    during the call only.  The library owns the rt_mesh and everything in it.
 *  - Layouts: per-cell vectors are [N][3] row-major; intensities are [N][K]
 *    row-major (angle fastest); limited gradients are [N][3][K].
 *  - Precision: with dtype RT_F64 intensity arrays are double; with RT_F32 they
 *    are float and transport runs in float, while the gas state, the opacities,
 *    the moment sums, the temperature root and the energy/momentum bookkeeping
 *    stay double.
 *  - Units: intensities are carried in energy-density units (equilibrium value
 *    a T^4 / 4 pi), so E_r = 4 pi sum_k W_k I_k and F_r = 4 pi c sum_k W_k n_k I_k.
 *    The gas temperature is T = (E_g - |rho v|^2 / 2 rho) / (rho cv).
 *  - Concurrency: calls on one mesh must not overlap in time on different
 *    streams (they share the mesh's scratch buffers).
 */
#ifndef RTMM_H
#define RTMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTMM_VERSION 1

enum {
  RT_OK = 0,
  RT_EINVAL = -1,     /* invalid argument (null pointer, bad size, bad value) */
  RT_ENOMEM = -2,     /* device allocation failed (upload only) */
  RT_EHIP = -3,       /* a HIP runtime call or kernel launch failed */
  RT_ENONFINITE = -4, /* non-finite values found (diagnostics) */
  RT_ESTATE = -5      /* the mesh was not prepared for this call (missing upload flag) */
};

enum { RT_F64 = 0, RT_F32 = 1 };              /* rt_params.dtype */
enum { RT_UPWIND1 = 0, RT_PLM_VL2 = 1 };      /* rt_params.scheme */

/* rt_mesh_upload flags: which scratch to allocate. */
enum {
  RT_MESH_PLM = 1,     /* half-step intensities and limited gradients for RT_PLM_VL2 */
  RT_MESH_ADJOINT = 2  /* one [N][K_max] adjoint buffer for rt_step_adjoint */
};

/* Kinds of marked cells (rt_marked_upload). */
enum {
  RT_CELL_BOUNDARY = 1, /* relaxation to a boundary state (section 2.4) */
  RT_CELL_EMITTER = 2   /* comoving emission at a radiation temperature (section 2.5) */
};

#define RT_K_MAX 128
#define RT_NDIAG 10
#define RT_SRC_TAPE 10 /* doubles per cell of a source tape (rt_step_taped, rt_step_adjoint_run) */

typedef struct rt_mesh rt_mesh;
typedef struct rt_marked rt_marked;

/* Physical and numerical parameters of one call. */
typedef struct {
  double c_red;   /* reduced speed of light cbar (transport speed, section 2.1), > 0 */
  double c_light; /* speed of light c (Lorentz factors, gas coupling), >= c_red */
  double a_rad;   /* radiation constant a, >= 0 */
  double cv;      /* specific heat: rho cv = rho k_B / (mu (gamma - 1) m_p) of eq. 26, > 0 */
  double dt;      /* time step, > 0 */
  int32_t dtype;  /* RT_F64 or RT_F32 */
  int32_t scheme; /* RT_UPWIND1 or RT_PLM_VL2 */
} rt_params;

/* Layout of an angle set (rt_angles.layout). */
enum {
  RT_ANGLES_GENERAL = 0,           /* no assumption */
  RT_ANGLES_ANTIPODAL = 1,         /* K even; dir[k + K/2] = -dir[k] and weight[k + K/2] = weight[k] for k < K/2 */
  RT_ANGLES_ANTIPODAL_ADJACENT = 2 /* K even; dir[2p + 1] = -dir[2p] and weight[2p + 1] = weight[2p] for p < K/2 */
};

/* Discrete ordinates: K unit directions and weights summing to one (device memory). */
typedef struct {
  int32_t K;            /* 1 <= K <= k_max of the mesh (and <= RT_K_MAX) */
  int32_t layout;       /* RT_ANGLES_*: an antipodal claim must first pass rt_angles_check() */
  const double *dir;    /* device [K][3], unit vectors */
  const double *weight; /* device [K], sum = 1 */
} rt_angles;

const char *rt_strerror(int code);
const char *rt_last_error(void);
int rt_version(void);

/*
 * Detect the layout of an angle set from HOST copies of its arrays: *layout is
 * RT_ANGLES_ANTIPODAL when K is even and, exactly, dir[k + K/2] = -dir[k] and
 * weight[k + K/2] = weight[k] for every k < K/2; else RT_ANGLES_ANTIPODAL_ADJACENT
 * when, exactly, dir[2p + 1] = -dir[2p] and weight[2p + 1] = weight[2p] for every
 * p < K/2; else RT_ANGLES_GENERAL.  Both antipodal layouts let the step kernel serve
 * each pair of opposite angles with one dot product per face (the paper's direction
 * sets are octant-symmetric); in the adjacent one the two intensities of a pair are
 * neighbours in a row, so each lane moves them with one 2-element access and a
 * cell's lanes read a neighbour row in half as many accesses.  Measured at 80 angles:
 * the adjacent order is the faster one for the FP64 form, the K/2 order for FP32.
 * Errors: RT_EINVAL on NULL pointers or K outside [1, RT_K_MAX].
 */
int rt_angles_layout(int32_t K, const double *dir, const double *weight, int32_t *layout);

/*
 * Verify the layout an angle set claims, against its DEVICE arrays, and record the
 * verified claim.  The paired kernels that serve the antipodal layouts take the
 * antipode's direction as -n_k and its weight as W_k (section 2.3's quadrature of
 * the moments and of the comoving weights W~ = N W / Gamma^2), so every call that
 * receives an angle set claiming RT_ANGLES_ANTIPODAL or RT_ANGLES_ANTIPODAL_ADJACENT
 * refuses it with RT_EINVAL unless this call recorded that exact claim (same K,
 * layout, dir and weight pointers).  RT_ANGLES_GENERAL needs no check: the general
 * kernels hold for any set.  The call copies dir [K][3] and weight [K] to the host
 * (synchronising `stream`), checks that every direction is a unit vector (within
 * 1e-10) and that the weights are non-negative and sum to one (within 1e-10), for
 * every layout, then classifies them as rt_angles_layout does and returns RT_EINVAL
 * (recording nothing) when the claim differs from what the arrays hold.
 * The arrays must not change while the claim is recorded: call rt_angles_release
 * before changing or freeing them.  Errors: RT_EINVAL (NULL, K outside
 * [1, RT_K_MAX], unknown layout, a direction that is not a unit vector, a negative or
 * non-finite weight, weights that do not sum to one, false claim), RT_EHIP.
 */
int rt_angles_check(const rt_angles *angles, void *stream);

/* Forget every recorded claim on the arrays of `angles` (no-op when there is none). */
int rt_angles_release(const rt_angles *angles);

/*
 * Upload a periodic Voronoi mesh and prepare it for steps (section 2: cells,
 * faces, and the face velocity of eq. 9).  All arrays are HOST memory:
 *   gen_pos[N][3]   generator positions r_i
 *   com[N][3]       cell centres of mass s_i (reconstruction origin)
 *   vol[N]          cell volumes of the tessellation (> 0)
 *   mesh_vel[N][3]  generator velocities w_i, held fixed over the run
 *   face_cells[F][2] cell pair (i, j) of each face, i != j
 *   face_shift[F][3] image of j adjacent to i is gen_pos[j] + shift * box
 *   face_area[F]    (> 0), face_normal[F][3] unit, from i towards j,
 *   face_centroid[F][3] in the frame of i
 *   box             periodic box side
 * The library computes on the device each face's normal speed w~.n (eq. 9),
 * the half-face table grouped by cell (a compressed-row index, so every cell
 * gathers its fluxes without atomics) and the rate of change of each cell
 * volume D_i = sum_faces A (w~.n) (outward positive; the volume update is
 * V^{n+1} = V^n + dt D_i).  k_max bounds K in later calls; flags (RT_MESH_*)
 * select scratch.  Errors: RT_EINVAL (sizes, indices out of range, area <= 0,
 * non-unit normal, a cell whose faces do not close: |sum A n| > 1e-8 V^(2/3), a
 * non-finite position, centre of mass, velocity or centroid), RT_ENOMEM, RT_EHIP.
 * All checks run on the host before any device memory is allocated.  On error *out
 * is NULL.  Synchronises `stream`.
 */
int rt_mesh_upload(rt_mesh **out, int64_t n_cells, int64_t n_faces, int32_t k_max, int32_t flags,
                   const double *gen_pos, const double *com, const double *vol, const double *mesh_vel,
                   const int32_t *face_cells, const int8_t *face_shift, const double *face_area,
                   const double *face_normal, const double *face_centroid, double box, void *stream);

/* Release the mesh and its device memory (NULL is accepted).  Synchronises the device. */
int rt_mesh_free(rt_mesh *mesh);

/* Sizes of an uploaded mesh (any output pointer may be NULL). */
int rt_mesh_info(const rt_mesh *mesh, int64_t *n_cells, int64_t *n_faces, int64_t *n_half_faces,
                 int32_t *k_max, int32_t *flags);

/* Copy the face normal speeds w~.n [F] (eq. 9) and the volume rates D [N] into
 * device arrays (either may be NULL).  Asynchronous on `stream`. */
int rt_mesh_geometry(const rt_mesh *mesh, double *face_speed, double *vol_rate, void *stream);

/*
 * Transport alone over params->dt (section 2.2), on `stream`:
 *  RT_UPWIND1: per face and angle the face-frame speed s = cbar n_k.n_f - w~.n_f
 *    picks the upwind cell; the charge dt A s I_up leaves the cell the normal
 *    points out of (eq. 8); I_out = (V I_in - sum of charges) / V_new.
 *  RT_PLM_VL2: the van Leer two-stage form (section 2, steps 2b-5) without the
 *    source: a first-order half step gives I_half, whose limited linear
 *    reconstruction (rt_gradient) gives the face states of the full step.
 * I_in [N][K] (device, dtype) and I_out must not overlap.  vol [N] (device) holds
 * V^n on entry and V^{n+1} = V^n + dt D on return.  RT_ESTATE if RT_PLM_VL2 is
 * asked of a mesh uploaded without RT_MESH_PLM.
 */
int rt_transport_step(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I_in,
                      void *I_out, double *vol, void *stream);

/*
 * Implicit source update over params->dt (section 2.3, the four-step
 * algorithm), in place on I [N][K]:
 *  1. lab moments E^n, F^n;  2. boost each angle to the comoving frame
 *  (Gamma_k = gamma (1 - v.n_k/c), I~ = Gamma^4 I, W~ = N W / Gamma^2), solve the
 *  temperature equation with J~ eliminated for T^{n+1};  3. implicit update of
 *  every I~_k and boost back;  4. E_g += (c/cbar)(E^n - E^{n+1}),
 *  rho v += (F^n - F^{n+1}) / (c cbar).
 * rho, kP, kJ, ks [N] (device) are read; mom [N][3] and etot [N] are updated in
 * place; T_new [N] (device, nullable) receives T^{n+1}.  J~ is eliminated in
 * the corrected form J~ = (S_I + y kP S_G a T^4/4pi)/(1 - y ks S_G), y = dt cbar rho
 * (the printed eq. 29 drops rho and misplaces kJ), with 1 - y ks S_G evaluated
 * as S_1 + y kJ S_G, S_1 = sum W~/(1 + y (kJ+ks) Gamma), which has no
 * cancellation.  The quartic A T^4 + B T - C = 0 is solved by Newton's method
 * from above in FP64.
 */
int rt_source_implicit(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, void *I,
                       const double *rho, double *mom, double *etot, const double *kP, const double *kJ,
                       const double *ks, double *T_new, void *stream);

/*
 * One radiation step: transport then source.  RT_UPWIND1: one fused pass (each
 * intensity row read once and written once).  RT_PLM_VL2: stage 1 = first-order
 * transport and source over dt/2 (its gas changes are discarded), stage 2 =
 * reconstructed fluxes of the half-step state applied to the start-of-step
 * charges over dt, then the source over dt on the start-of-step gas.
 * Arguments as rt_transport_step and rt_source_implicit; I_in and I_out must not
 * overlap.
 */
int rt_step(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I_in, void *I_out,
            double *vol, const double *rho, double *mom, double *etot, const double *kP, const double *kJ,
            const double *ks, double *T_new, void *stream);

/*
 * One RT_UPWIND1 step as rt_step (transport, section 2.2, then the source,
 * section 2.3, in one fused pass) that also records what a reverse of the step needs.
 * I_star [N][K] (device, dtype, nullable) receives the transported intensities, i.e.
 * the source's input: the value rt_step_adjoint needs for this step.  src_tape
 * [N][RT_SRC_TAPE] (device, double, nullable) receives per cell what
 * rt_step_adjoint_run needs of this step besides its output I_out: the values of the
 * source solve (section 2.3, steps 1-2)
 * that it reuses instead of solving again, 1 / sum_k W_k Gamma_k^-2, the weighted sums
 * S1 = sum Wt r, SG = sum Wt Gamma r, SI = sum Wt Gamma^4 I* r (Wt = W Gamma^-2 / that
 * sum, r = 1 / (1 + y chi Gamma)), 1 / (S1 + y kJ SG) and the new temperature T^{n+1};
 * then the start-of-step volume V^n and gas momentum (rho v)^n (3 values).  At least
 * one of the two must be given.  I_out and vol, mom, etot, T_new receive exactly what
 * rt_step gives.  I_in, I_out and I_star must not overlap.  RT_EINVAL for RT_PLM_VL2.
 */
int rt_step_taped(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I_in, void *I_out,
                  void *I_star, double *vol, const double *rho, double *mom, double *etot, const double *kP,
                  const double *kJ, const double *ks, double *T_new, double *src_tape, void *stream);

/*
 * Limited linear reconstruction of every angle (section 2.2 item ii): the
 * Voronoi gradient estimator of S10 with the geometric cell volumes, limited by
 * the Barth-Jespersen factor so that extrapolations from the centre of mass to
 * every face centroid stay within the range of the cell and its neighbours.
 * I [N][K] (device, dtype) in, grad [N][3][K] (device, dtype) out.  Needs a mesh
 * uploaded with RT_MESH_PLM (RT_ESTATE otherwise): it holds the estimator's weights
 * (one vector per half-face and one per cell, formed at upload) and the
 * reconstruction offsets.  The upload refuses a PLM mesh whose face records of 16
 * consecutive cells would not fit in the LDS a workgroup may use, so this call does
 * not fail for that reason.
 */
int rt_gradient(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I, void *grad,
                void *stream);

/*
 * Reverse (adjoint) of one RT_UPWIND1 rt_step for the gradient of a scalar loss.
 * Inputs of the forward step: I_star = intensities after transport (the source
 * input), vol_n = V^n, rho, mom_n, etot_n (gas before the source), kP, kJ, ks.
 * Adjoints: lamI [N][K] (dtype) holds dL/dI^{n+1} on entry and dL/dI^n on
 * return; lamE [N] and lamM [N][3] hold dL/d(etot, mom)^{n+1} on entry and
 * dL/d(etot, mom)^n on return; dL_dkP, dL_dkJ [N] are incremented (nullable;
 * they may be the same array, which then receives both partials: the gradient
 * with respect to a tied opacity kP = kJ).
 * The temperature root enters through the implicit function theorem.  As in the
 * forward source, the per-angle arithmetic is done in the intensities' type (FP32
 * with RT_F32) and every sum over angles and every per-cell value in FP64.  Needs
 * a mesh uploaded with RT_MESH_ADJOINT (RT_ESTATE otherwise).
 */
int rt_step_adjoint(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I_star,
                    const double *vol_n, const double *rho, const double *mom_n, const double *etot_n,
                    const double *kP, const double *kJ, const double *ks, void *lamI, double *lamE, double *lamM,
                    double *dL_dkP, double *dL_dkJ, void *stream);

/*
 * Reverse of n_steps consecutive RT_UPWIND1 steps, each recorded with rt_step_taped
 * and a source tape: the same adjoint as rt_step_adjoint called for steps
 * n_steps - 1 down to 0, in n_steps + 1 launches instead of 2 n_steps.  Each launch
 * but the first and last transposes the transport of step n + 1 and reverses the
 * source of step n in one pass, so dL/dI between them never goes to memory, and the
 * source reverse reads the forward's own sums and temperature from the tape
 * (section 2.3; through the temperature root by the implicit function theorem).  It
 * reads each step's output, not its transported intensities: the source update
 * inverts to Gamma^4 I* + y Gamma S = I' Gamma^4 / r, so the forward need not store I*.
 * I_next, src_tape: host arrays of n_steps device pointers; entry i belongs to step i
 * of the run: its output intensities (the I_out of its rt_step_taped call, kept
 * unchanged) and its source tape (which holds the step's start-of-step volume and
 * momentum, so no other state is needed).  rho, kP, kJ, ks as in the forward steps.  lamI [N][K] (dtype) holds dL/dI after the last step on entry and
 * dL/dI before step 0 on return; lamE, lamM, dL_dkP, dL_dkJ as in rt_step_adjoint.
 * Uses the mesh's RT_MESH_ADJOINT buffer (RT_ESTATE without it), so calls on one mesh
 * are serialised by their stream.  n_steps = 0 does nothing.  A NULL entry, an
 * I_next[i] overlapping lamI or the mesh's adjoint buffer, or a misaligned tape give
 * RT_EINVAL before any launch; after a failed launch the adjoints hold unspecified
 * values.
 */
int rt_step_adjoint_run(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, int32_t n_steps,
                        const void *const *I_next, const double *const *src_tape, const double *rho,
                        const double *kP, const double *kJ, const double *ks, void *lamI, double *lamE,
                        double *lamM, double *dL_dkP, double *dL_dkJ, void *stream);

/*
 * Emergent-flux loss L = sum_f u_f A_f 4 pi c sum_k W_k (n_k.n_f) I_up(f,k),
 * the radiative flux through each weighted face with the upwind intensity of
 * each angle (chosen by the sign of n_k.n_f).  face_weight [F] (device, signed:
 * the sign orients the face, zero for faces outside the loss).  *loss (device
 * double) is overwritten; when seed != NULL, dL/dI is ADDED to seed [N][K]
 * (dtype).  Deterministic: no atomics.
 */
int rt_flux_loss(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I,
                 const double *face_weight, double *loss, void *seed, void *stream);

/*
 * rt_flux_loss for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, kernels
 * and results (bit for bit) as rt_flux_loss, but the per-workgroup partial sums live in a
 * static device array of the library (2 MiB on every device it runs on, held until the
 * process ends) instead of the mesh's scratch, and the call allocates nothing, on the
 * device or the host.  Limit: one partial sum per workgroup of 16 cells (K a multiple of
 * 16 or above 64) or 32 cells (other K), at most 261888 of them, i.e. meshes of up to
 * 4,190,208 or 8,380,416 cells; larger meshes get RT_EINVAL.  Every partial the fold reads
 * is written by the same call, so nothing needs clearing between calls.  All calls on one
 * device share its array: calls that overlap in time on one device (other streams, other
 * threads) race and must be serialised by the caller.  The mesh's device must be current
 * (RT_EINVAL otherwise).  Errors as rt_flux_loss, plus RT_EHIP if the array's device
 * address cannot be found.
 */
int rt_flux_loss_noalloc(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I,
                         const double *face_weight, double *loss, void *seed, void *stream);

/*
 * Multigroup implicit source update over params->dt (section 2.3, frequency
 * groups coupled only through the gas temperature), in place.  G groups
 * (1 <= G <= 16) of K angles each: I [G][N][K] (device, dtype, group-major),
 * kP, kJ, ks [G][N] (device), group_weight [G] (device): group j enters the
 * moments and the gas energy and momentum equations with weight Wg_j.  Per
 * group the comoving sums and J~_j are those of rt_source_implicit; the
 * temperature solves A T^4 + B T - C = 0 with
 *   A = dt c rho a sum_j Wg_j kP_j S1_j / D_j,
 *   C = rho cv T^n + 4 pi dt c rho sum_j Wg_j kJ_j SI_j / D_j.
 * The emission of group j is kP_j a T^4 / 4pi, so a Planck split over groups is
 * carried by kP_j.  rho, mom, etot, T_new as in rt_source_implicit.
 */
int rt_source_implicit_mg(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, int32_t G,
                          const double *group_weight, void *I, const double *rho, double *mom, double *etot,
                          const double *kP, const double *kJ, const double *ks, double *T_new, void *stream);

/*
 * One multigroup RT_UPWIND1 step: every group's [N][K] slab of I_in is
 * transported (section 2.2) into I_out, the volumes advance once, then
 * rt_source_implicit_mg runs on I_out.  Arguments as rt_step and
 * rt_source_implicit_mg; I_in and I_out ([G][N][K]) must not overlap.
 * RT_EINVAL for RT_PLM_VL2.
 */
int rt_step_mg(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, int32_t G,
               const double *group_weight, const void *I_in, void *I_out, double *vol, const double *rho,
               double *mom, double *etot, const double *kP, const double *kJ, const double *ks, double *T_new,
               void *stream);

/*
 * Implicit source update with temperature-dependent opacities over params->dt
 * (section 2.3, where the temperature equation is solved by Newton-Raphson
 * iteration), in place on I [N][K].  Power laws at T^{n+1}:
 * kP(T) = kP0 (T/T_ref)^bP, kJ(T) = kJ0 (T/T_ref)^bJ (kP0, kJ0 [N] device;
 * T_ref > 0; |bP|, |bJ| <= 20); ks [N] is constant.  With J~ eliminated the
 * temperature equation is f(T) = rho cv (T - T^n) + dt c rho [kP a T^4 S1 -
 * 4 pi kJ SI] / D = 0, whose comoving sums depend on T through kJ.  The root is
 * bracketed from T^n (doubling up while f < 0, halving down while f > 0) and
 * found by Newton steps kept inside the bracket (bisection otherwise) to a step
 * of at most 1e-14 T, which is taken as it is.  Where f has several roots this gives the one reached from
 * T^n.  With bP = bJ = 0 it gives the root of rt_source_implicit's quartic.
 * Per-angle arithmetic is FP64 in both precision forms.  Other arguments as
 * rt_source_implicit.
 */
int rt_source_implicit_kT(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, void *I,
                          const double *rho, double *mom, double *etot, const double *kP0, const double *kJ0,
                          const double *ks, double T_ref, double bP, double bJ, double *T_new, void *stream);

/*
 * One RT_UPWIND1 step with temperature-dependent opacities: upwind transport
 * (as rt_transport_step) into I_out, then rt_source_implicit_kT on I_out.
 * Arguments as rt_step and rt_source_implicit_kT.  RT_EINVAL for RT_PLM_VL2.
 */
int rt_step_kT(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I_in, void *I_out,
               double *vol, const double *rho, double *mom, double *etot, const double *kP0, const double *kJ0,
               const double *ks, double T_ref, double bP, double bJ, double *T_new, void *stream);

/*
 * Upload a set of marked cells: boundary cells (section 2.4) and radiation
 * emitters (section 2.5), applied by rt_marked_apply after each step.  HOST
 * arrays, n entries (n >= 0; the cells distinct, 0 <= cell < n_cells):
 *   cell[n]       cell index in a mesh of n_cells cells
 *   kind[n]       RT_CELL_BOUNDARY or RT_CELL_EMITTER
 *   T_eff[n]      radiation temperature (>= 0); S = a T_eff^4 / 4 pi
 *   dir[n][3]     unit direction; the cell's directions of interest are the
 *                 angles with n_k . dir >= cos_open
 *   cos_open[n]   opening cosine (> 1 selects no direction)
 *   tau           relaxation time of boundary cells (> 0)
 * All arguments are validated on the host before any device memory is
 * allocated: RT_EINVAL names the first bad entry.  RT_ENOMEM, RT_EHIP.
 * Synchronises `stream`.
 */
int rt_marked_upload(rt_marked **out, int64_t n_cells, int64_t n, const int32_t *cell, const int32_t *kind,
                     const double *T_eff, const double *dir, const double *cos_open, double tau, void *stream);

/* Release a set of marked cells (NULL is accepted).  Synchronises the device. */
int rt_marked_free(rt_marked *set);

/*
 * Apply the marked cells over params->dt, in place, on `stream` (never
 * allocates).  Boundary cells, with f = min(dt/tau, 1): I_k <- I_k - (I_k - I0_k) f
 * where I0_k = S in the directions of interest and 0 otherwise (absorbing), and
 * rho v <- rho v (1 - f) with the kinetic energy that goes with it taken from the
 * total gas energy (the density is not evolved by the radiation step).  Emitter
 * cells, in the directions of interest only: the comoving emission-absorption
 * term at T_eff integrated implicitly, I~' = (I~ + x S)/(1 + x) with
 * I~ = Gamma^4 I, Gamma = gamma (1 - v.n/c), x = dt Gamma cbar rho kP; the gas is
 * not changed.  I [N][K] (device, dtype), rho, kP [N] and mom [N][3], etot [N]
 * (device, FP64).  RT_EINVAL if the set was uploaded for another cell count.
 */
int rt_marked_apply(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const rt_marked *set,
                    void *I, const double *rho, double *mom, double *etot, const double *kP, void *stream);

/*
 * Angle moments of every cell (section 2.1: the zeroth, first and second moments of
 * the intensity, as radiation energy density, flux and pressure tensor).  With the
 * intensities in energy-density units, E_r = 4 pi sum_k W_k I_k,
 * F_r = 4 pi c sum_k W_k n_k I_k and P_r = 4 pi sum_k W_k n_k n_k I_k (c = c_light).
 * I [N][K] (device, params->dtype); moments [N][10] (device, FP64, written):
 * (E_r, F_x, F_y, F_z, P_xx, P_yy, P_zz, P_xy, P_xz, P_yz).  Only params->dtype and
 * params->c_light are used (the other fields must still be valid).  Enqueues one
 * kernel and never allocates.  RT_EINVAL if I and moments overlap.
 */
int rt_moments(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I, double *moments,
               void *stream);

/*
 * Conservation diagnostics into out[RT_NDIAG] (HOST), the totals of section 2.3.1's
 * energy and momentum balance in the reduced-speed-of-light approximation (eqs. 37-38,
 * the radiation parts weighted by c/cbar and 1/(c cbar) as in eqs. 17-18): sum V E_g,
 * sum V (c/cbar) E_r, sum V rho v (3), sum V F_r/(c cbar) (3), min I, and the
 * number of non-finite entries of I, etot and mom.  The source update keeps
 * E_g + (c/cbar) E_r and rho v + F_r/(c cbar) of every cell unchanged, and transport
 * conserves sum V I of every angle, so the first two totals and the two momentum
 * totals sum to constants on a periodic mesh.  Synchronises `stream`.
 * Returns RT_ENONFINITE (with out filled) when that count is non-zero.
 */
int rt_diagnostics(rt_mesh *mesh, const rt_params *params, const rt_angles *angles, const void *I,
                   const double *vol, const double *etot, const double *mom, double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* RTMM_H */
