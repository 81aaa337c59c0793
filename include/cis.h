/*
 * cis.h - C ABI of the MI355X (gfx950) interval linearize-and-discretize
 * library for contact-implicit continuous-time successive convexification
 * (CI-SCvx, arxiv 2604.09993).
 *
 * What is computed (paper references are to arxiv 2604.09993):
 *  For every interval k = 0..N-1 between trajectory nodes, the time-dilated
 *  augmented system x~' = s (f(x,u), Omega(x,u)) on tau in [0,1]
 *  (Sec. IV-B, eq. aug-dynamics) with first-order-hold controls
 *  u(tau) = (1-tau) U_k + tau U_{k+1} (Sec. IV-B parameterization, Sec. VI) is
 *  integrated by classical RK4 with K uniform substeps, starting at node X_k.
 *  f is planar maximal-coordinate multibody dynamics with joint forces and
 *  normal/split-friction contact forces (Sec. II-A, eq. ct-dynamics); Omega
 *  holds the integral cross-complementarity integrands (Sec. III, Prop. 1;
 *  Sec. IV-A eq. aux-dynamics) and one continuous-time constraint-violation
 *  integrand.  Together with the state, the variational equations are
 *  integrated through the same RK4 stages (internal numerical
 *  differentiation, Sec. VI), giving the exact derivatives of the discrete
 *  map F~_k = F~(X_k, U_k, U_{k+1}, s_k) of eq. intg-aug-sys-param:
 *     A_k  = dF~_k/dX_k,  Bm_k = dF~_k/dU_k,  Bp_k = dF~_k/dU_{k+1},
 *     S_k  = dF~_k/ds_k,  defect d_k = F~_k - X_{k+1}  (eq. cito-augdyn).
 *
 * Sizes: nb bodies, nj revolute joints, nc contacts;
 *   n = 6 nb (poses and velocities), n_y = nc + 1 integral states,
 *   nx = n + n_y (augmented state), m = 3 nj + 3 nc controls
 *   (joint torques, world-frame joint forces, [lam_n, lam_t+, lam_t-] per
 *   contact), P = nb + 2 parameters p = (mu, e, m_0 .. m_{nb-1}).
 * State order: x~ = (x_0,y_0,th_0, .., v_0 .. , y_cc_0 .., y_ctcs).
 *
 * Memory layout ("SoA", interval or node index contiguous, all DEVICE
 * pointers owned by the caller, element type given by cis_shape.dtype):
 *   X      [nx][ld_node]      node k, component r at X[r*ld_node + k], k <= N
 *   U      [m][ld_node]
 *   s      [N]                dilation of interval k (physical length)
 *   params [P]
 *   A      [nx][nx][ld_int]   interval k, row r, column c at A[(r*nx+c)*ld_int + k]
 *   Bm, Bp [nx][m][ld_int]
 *   S, defect, xprop, seed [nx][ld_int]
 *   ckpt   [K/C][n][ld_int]   x (without y) at substeps 0, C, 2C, ..
 *   gX     [nx][ld_node], gU [m][ld_node], gs [N], gparams [P]
 * ld_node >= N+1 and ld_int >= N.  Every pointer must be aligned to the
 * element size.
 *
 * Concurrency and ownership: no call allocates, frees, copies host<->device or
 * synchronizes; work is enqueued on `stream` (a hipStream_t; NULL = the
 * default stream) and errors in device execution surface at the caller's next
 * synchronization.  A cis_model is an immutable host object and may be used
 * from several threads and streams at once.  On any returned error nothing
 * has been enqueued and no output has been written.
 *
 * Non-finite values (NaN, +-inf) in the inputs propagate through the
 * arithmetic and are not checked.  Debug mode: with the environment variable
 * CIS_DEBUG_FINITE set (non-empty, not "0"), cis_discretize,
 * cis_discretize_split, cis_discretize_blocked, cis_discretize_rkf,
 * cis_discretize_paper, cis_defects and cis_discretize_adjoint, after a
 * successful launch, count the non-finite values of every input and output
 * array (the blocks the call reads or writes; checkpoints and workspaces
 * excluded), synchronize the stream, and return CIS_ERR_NONFINITE, with
 * cis_last_error naming each such array and its count ("input X 3, output A
 * 120"); the outputs are then written.  Debug mode allocates, copies and
 * synchronizes: it is not for hot loops, and the allocation-free entry point
 * does not take part in it.
 */
#ifndef CIS_H
#define CIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CIS_OK = 0,
    CIS_ERR_NULL = 1,         /* a required pointer is NULL                  */
    CIS_ERR_DIM = 2,          /* N, K, ld or checkpoint stride out of range  */
    CIS_ERR_LAYOUT = 3,       /* pointer not aligned to the element size     */
    CIS_ERR_DTYPE = 4,        /* unknown dtype or dtype not offered here     */
    CIS_ERR_WORKSPACE = 5,    /* workspace missing or too small              */
    CIS_ERR_MODEL = 6,        /* malformed model description                 */
    CIS_ERR_HIP = 7,          /* the HIP runtime rejected a launch           */
    CIS_ERR_UNSUPPORTED = 8,  /* topology with no compiled kernel            */
    CIS_ERR_NONFINITE = 9     /* debug mode only: non-finite input or output */
} cis_status;

typedef enum { CIS_F64 = 0, CIS_F32 = 1 } cis_dtype;

typedef struct cis_model cis_model;   /* opaque, immutable after creation */

/*
 * Host description of a planar multibody model (Sec. II).  All arrays are
 * HOST pointers, copied by cis_model_create; the caller keeps ownership.
 * Bodies are rigid rods: I_b = m_b * link_length_b^2 / 12.  Joint j connects
 * parent body joint_parent[j] at anchor joint_anchor_parent[j] (parent body
 * frame) to joint_child[j] at joint_anchor_child[j]; its reaction force
 * lambda_j (world frame) acts +lambda on the parent and -lambda on the child
 * (grad h^T lambda, eq. ct-dynamics); torque tau_j plus the spring-damper
 * torque -k (th_c - th_p) - d (w_c - w_p) acts +1x on the child and -1x on
 * the parent.  Contact i sits at contact_point[i] in the frame of
 * contact_body[i].  Terrain: h(P) = P_y - A sin(kappa P_x) (A = 0: flat),
 * signed distance approximated by h/||grad h|| (Sec. VI-B).
 *
 * Compiled topologies: a torso (body 0) with L legs of D links, link d of
 * leg l being body 1 + l*D + d, joint j having child j+1, and the contact of
 * leg l at the last link of that leg (on the torso when D = 0).  (L, D) in
 * {(0,0),(1,0),(1,1),(1,2),(2,1),(2,2),(2,3),(4,3)}; other topologies give
 * CIS_ERR_UNSUPPORTED.
 */
typedef struct {
    int32_t n_bodies, n_joints, n_contacts;
    const double *link_length;          /* [n_bodies], > 0                   */
    const int32_t *joint_parent;        /* [n_joints]                        */
    const int32_t *joint_child;         /* [n_joints]                        */
    const double *joint_anchor_parent;  /* [n_joints][2]                     */
    const double *joint_anchor_child;   /* [n_joints][2]                     */
    const double *joint_stiffness;      /* [n_joints]                        */
    const double *joint_damping;        /* [n_joints]                        */
    const int32_t *contact_body;        /* [n_contacts]                      */
    const double *contact_point;        /* [n_contacts][2]                   */
    double gravity;                     /* m/s^2, acts along -y              */
    double terrain_amplitude;           /* A                                 */
    double terrain_wavenumber;          /* kappa                             */
} cis_model_desc;

/* Problem shape: N intervals (N+1 nodes), K RK4 substeps per interval. */
typedef struct {
    int32_t N;
    int32_t substeps;        /* 1 <= K <= 4096                               */
    int32_t dtype;           /* cis_dtype                                    */
    int32_t layout;          /* cis_discretize, one trajectory: workgroup     */
                             /* layout, 0 = by rule (see cis_discretize),     */
                             /* 1 latency, 2 latency with S on leg lanes,     */
                             /* 3 narrow, 4 throughput; other calls ignore it */
    int64_t ld_node;         /* >= N + 1                                     */
    int64_t ld_int;          /* >= N                                         */
} cis_shape;

/* Library version string (static storage). */
const char *cis_version(void);

/* Human-readable text of a status code (static storage). */
const char *cis_status_string(cis_status st);

/* Detail of the last failure on the calling thread (thread-local storage). */
const char *cis_last_error(void);

/* Validate and copy a model description; *out receives the model.
 * Errors: CIS_ERR_NULL, CIS_ERR_MODEL, CIS_ERR_UNSUPPORTED. */
cis_status cis_model_create(const cis_model_desc *desc, cis_model **out);

/* Release a model (NULL is accepted). */
void cis_model_destroy(cis_model *model);

/* Sizes n, n_y, m, P of a model (any output pointer may be NULL). */
cis_status cis_model_dims(const cis_model *model, int32_t *n, int32_t *n_y, int32_t *m,
                          int32_t *n_params);

/*
 * Linearize and discretize every interval (the per-SCP-iteration hot path,
 * Sec. VI transcription): writes A, Bm, Bp, S, defect and, if xprop is not
 * NULL, F~_k.  Inputs X, U, s, params; U may be NULL only when m = 0, and
 * Bm/Bp likewise.  dtype CIS_F64 or CIS_F32 (all buffers of that type).
 */
cis_status cis_discretize(const cis_model *model, const cis_shape *shape, const void *X,
                          const void *U, const void *s, const void *params, void *A,
                          void *Bm, void *Bp, void *S, void *defect, void *xprop,
                          void *stream);

/*
 * Defects only (no sensitivities): F~_k into xprop (may be NULL), d_k into
 * defect, and, if ckpt is not NULL, the x part of the state at substeps
 * 0, C, 2C, .. with C = ckpt_every (C must divide K; ckpt holds K/C slots).
 * dtype CIS_F64 or CIS_F32.
 */
cis_status cis_defects(const cis_model *model, const cis_shape *shape, const void *X,
                       const void *U, const void *s, const void *params, void *defect,
                       void *xprop, void *ckpt, int32_t ckpt_every, void *stream);

/* Bytes of device workspace cis_discretize_adjoint needs for this shape. */
cis_status cis_adjoint_workspace_size(const cis_model *model, const cis_shape *shape,
                                      size_t *bytes);

/*
 * Reverse-mode sweep (vector-Jacobian product) of the map
 * (X, U, s, p) -> F~ for the cotangent seed lambda_k = dJ/dF~_k
 * (the penalized defect merit of Sec. V is one such J).  Outputs are
 * overwritten, not accumulated:
 *   gX_k = A_k^T lambda_k (k < N), gX_N = 0;
 *   gU_k = Bm_k^T lambda_k + Bp_{k-1}^T lambda_{k-1};
 *   gs_k = S_k^T lambda_k;  gparams = sum_k (dF~_k/dp)^T lambda_k.
 * The substep states are recomputed from ckpt (written by cis_defects with
 * the same ckpt_every).  Reductions over intervals are done in a fixed order
 * (run-to-run bitwise reproducible).  ws must hold
 * cis_adjoint_workspace_size bytes.  dtype CIS_F64 only.
 */
cis_status cis_discretize_adjoint(const cis_model *model, const cis_shape *shape,
                                  const void *X, const void *U, const void *s,
                                  const void *params, const void *ckpt, int32_t ckpt_every,
                                  const void *seed, void *gX, void *gU, void *gs,
                                  void *gparams, void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reverse sweep as cis_discretize_adjoint, same arguments and outputs, with
 * no workspace argument.  Its workspace is a device array inside the library,
 * 8 MiB per GPU (held from the first call on that GPU until the process
 * ends), enough for (2 m + P) N <= 1,048,576 doubles (quad13: N <= 9446);
 * larger shapes return CIS_ERR_WORKSPACE.  Nothing is allocated on any call.
 * Every call on one GPU uses that GPU's single array: calls that overlap on
 * one GPU (concurrent streams, or threads without ordering) race and give
 * undefined results; calls ordered on one stream are safe.  The array keeps
 * the last call's partial sums; every entry a call reads it writes first.
 * Other errors as for cis_discretize_adjoint.
 */
cis_status cis_discretize_adjoint_noalloc(const cis_model *model, const cis_shape *shape,
                                          const void *X, const void *U, const void *s,
                                          const void *params, const void *ckpt,
                                          int32_t ckpt_every, const void *seed, void *gX,
                                          void *gU, void *gs, void *gparams, void *stream);

/* Bytes of device workspace cis_discretize_split needs for this shape (the
 * model must have legs with links, else CIS_ERR_UNSUPPORTED). */
cis_status cis_split_workspace_size(const cis_model *model, const cis_shape *shape,
                                    size_t *bytes);

/*
 * Same outputs as cis_discretize (same discrete map, Sec. IV-B and Sec. VI;
 * dtype CIS_F64 or CIS_F32), computed in two launches for throughput on many
 * intervals.  The first integrates the nominal state, the integral rows and
 * S, and stores every RK stage's Jacobian coefficients in `ws` (a compact
 * record per stage); the second integrates the columns of Phi_x, B- and B+
 * from those records, one wave per leg and one column per lane, reading the
 * coefficients with scalar loads.  Results equal those of cis_discretize up
 * to the order of floating-point sums.  waves (1 or 2): register budget of
 * the second launch in waves per SIMD (2: two workgroups share a compute
 * unit).  ws must hold cis_split_workspace_size bytes, 8-byte aligned; its
 * contents are scratch.  Models without legs with links: CIS_ERR_UNSUPPORTED.
 */
cis_status cis_discretize_split(const cis_model *model, const cis_shape *shape, const void *X,
                                const void *U, const void *s, const void *params,
                                int32_t waves, void *A, void *Bm, void *Bp, void *S,
                                void *defect, void *xprop, void *ws, size_t ws_bytes,
                                void *stream);

/* Bytes of device workspace cis_discretize_rkf needs for this shape (the
 * model must have legs with links, else CIS_ERR_UNSUPPORTED). */
cis_status cis_rkf_workspace_size(const cis_model *model, const cis_shape *shape,
                                  size_t *bytes);

/*
 * The discretize step with the Runge-Kutta-Fehlberg integrator of the paper's
 * transcription (Sec. VI) in place of classical RK4: K fixed steps of
 * Fehlberg's 4(5) pair per interval (stage nodes 0, 1/4, 3/8, 12/13, 1, 1/2
 * of the step), the fourth-order solution propagated, with the variational
 * equations integrated through the same stages (internal numerical
 * differentiation), so A, Bm, Bp and S are the exact derivatives of that
 * discrete map; defect and xprop as for cis_discretize.  err (may be NULL;
 * [N], element type of the shape): for each interval the largest embedded
 * error estimate |h sum_i (bh_i - b_i) K_i| over its steps and all nx rows,
 * bh the fifth-order weights.  Two launches (stage records, then tangent
 * columns) as cis_discretize_split; waves (1 or 2): register budget of the
 * second launch.  ws must hold cis_rkf_workspace_size bytes, 8-byte aligned;
 * its contents are scratch.  dtype CIS_F64 or CIS_F32.  Models without legs
 * with links: CIS_ERR_UNSUPPORTED.
 */
cis_status cis_discretize_rkf(const cis_model *model, const cis_shape *shape, const void *X,
                              const void *U, const void *s, const void *params, int32_t waves,
                              void *A, void *Bm, void *Bp, void *S, void *defect, void *xprop,
                              void *err, void *ws, size_t ws_bytes, void *stream);

/* Sizes of the paper-faithful dynamics variant of a model: nx = 6 nb + 4 nc + 1
 * augmented states and m = nj + 3 nc controls (any output pointer may be NULL). */
cis_status cis_paper_dims(const cis_model *model, int32_t *nx, int32_t *m);

/* Bytes of device workspace cis_discretize_paper needs (FP64; models with legs
 * with links, else CIS_ERR_UNSUPPORTED). */
cis_status cis_paper_workspace_size(const cis_model *model, const cis_shape *shape,
                                    size_t *bytes);

/*
 * The discretize step of the paper-faithful dynamics variant, FP64:
 *  - joint reaction forces are not controls: they are eliminated at the
 *    acceleration level (Sec. II-A, eq. joint-cnstr-acc):
 *      lambda = -(grad h M^-1 grad h^T)^-1 (grad h M^-1 (W + J^T R phi) + c),
 *      c_j = v^T grad^2 h_j v = -w_p^2 a_p + w_c^2 a_c;
 *  - controls u = (tau_0 .. tau_{nj-1}, then (phi_t, phi_n, gamma) per
 *    contact), m = nj + 3 nc, with R phi = t phi_t + n phi_n;
 *  - integral states (eq. aux-dynamics): per contact the integrals of phi_n,
 *    lambda_c = t^T J v + gamma phi_t / sqrt(phi_t^2 + 1), gamma and
 *    rho_c = |mu phi_n|_s - |phi_t|_s, then one violation state integrating
 *    sum_i ramp_s(-phi_n) + ramp_s(-sd) + ramp_s(-gamma) + ramp_s(-rho_c)
 *    (one row of all ones as the mixing matrix); nx = 6 nb + 4 nc + 1;
 *  - classical RK4 with K substeps and FOH controls as cis_discretize, with
 *    the variational equations through the same stages (Sec. IV-B, Sec. VI).
 * Arrays as in the header comment with these nx and m: X [nx][ld_node],
 * U [m][ld_node], A [nx][nx][ld_int], Bm/Bp [nx][m][ld_int], S, defect,
 * xprop [nx][ld_int] (xprop may be NULL).  Two launches (a stage record per
 * interval, then tangent columns); ws must hold cis_paper_workspace_size
 * bytes, 8-byte aligned (scratch).  Errors as for cis_discretize_split;
 * dtype other than CIS_F64: CIS_ERR_DTYPE.
 */
cis_status cis_discretize_paper(const cis_model *model, const cis_shape *shape, const void *X,
                                const void *U, const void *s, const void *params, void *A,
                                void *Bm, void *Bp, void *S, void *defect, void *xprop, void *ws,
                                size_t ws_bytes, void *stream);

/* Composition of the substep blocks of cis_discretize_blocked. */
enum { CIS_COMPOSE_VALU = 0, CIS_COMPOSE_MFMA = 1 };

/* Bytes of device workspace cis_discretize_blocked needs (blocks >= 2 must
 * divide the substep count). */
cis_status cis_blocked_workspace_size(const cis_model *model, const cis_shape *shape,
                                      int32_t blocks, size_t *bytes);

/*
 * Same outputs as cis_discretize (dtype CIS_F64 only), computed with substep
 * blocking: the K substeps of each interval are split into `blocks` blocks
 * of K/blocks substeps.  A checkpointed nominal pass gives the block start
 * states (and the defect and F~); the variational equations of every
 * (block, interval) pair are then integrated in parallel, each from its block
 * start, with the interval's FOH and dilation; finally the block
 * sensitivities X_b = [Phi_b | B-_b | B+_b | S_b] are chained,
 *   A = Phi_{B-1}..Phi_0,  [B- | B+ | S] = sum_b Phi_{B-1}..Phi_{b+1} [B-_b | B+_b | S_b],
 * with dense products on the vector ALUs (CIS_COMPOSE_VALU) or on FP64
 * matrix cores (CIS_COMPOSE_MFMA).  Mathematically equal to cis_discretize
 * (chain rule over the block boundaries); the sums are ordered differently.
 * ws must hold cis_blocked_workspace_size bytes (checkpoints and per-block
 * sensitivities).  Trades (blocks - 1) dense products per interval for a
 * blocks-times shorter sensitivity recursion.
 */
cis_status cis_discretize_blocked(const cis_model *model, const cis_shape *shape, const void *X,
                                  const void *U, const void *s, const void *params,
                                  int32_t blocks, int32_t compose, void *A, void *Bm, void *Bp,
                                  void *S, void *defect, void *xprop, void *ws, size_t ws_bytes,
                                  void *stream);

/* Forms of the discretize step for one trajectory, as chosen by cis_single_tune. */
enum { CIS_FORM_ONE_LAUNCH = 0, CIS_FORM_SPLIT = 1, CIS_FORM_BLOCKED = 2 };
typedef struct {
    int32_t form;            /* CIS_FORM_*                                     */
    int32_t layout;          /* one-launch form: cis_shape.layout (1..4)       */
    int32_t waves;           /* split form: register budget (1 or 2)          */
    int32_t blocks;          /* blocked form: substep blocks (divides K)      */
    int32_t compose;         /* blocked form: CIS_COMPOSE_*                   */
    int32_t from_cache;      /* 1: read from the CIS_TUNE_CACHE file           */
    float ms;                /* time of the choice (best of three), 0 on a hit */
} cis_single_choice;

/*
 * Tuner of the discretize step for one trajectory shape: times, on the
 * caller's inputs, the one-launch kernel in each of its four workgroup
 * layouts (the threads-per-interval mapping), the split form with one and two
 * waves per SIMD (models with legs with links), and (FP64) the substep-blocked
 * form for every block count 2..8 dividing K with VALU and MFMA composition;
 * each candidate best of three runs (HIP events on `stream`).  Returns the
 * fastest in *choice and leaves its outputs in A, Bm, Bp, S, defect, xprop.
 * With CIS_TUNE_CACHE naming a file the choice is looked up first (then
 * nothing is timed) and recorded after tuning, keyed by device, topology,
 * dtype, N and K.  NOT a hot call: allocates the largest workspace any
 * candidate needs, synchronizes the stream and frees it.  shape->layout must
 * be 0.  Errors: those of the candidates' entry points, CIS_ERR_NULL for a
 * missing choice, CIS_ERR_HIP.
 */
cis_status cis_single_tune(const cis_model *model, const cis_shape *shape, const void *X,
                           const void *U, const void *s, const void *params, void *A, void *Bm,
                           void *Bp, void *S, void *defect, void *xprop, cis_single_choice *choice,
                           void *stream);

/* ------------------------------------------------------------------------
 * Batches of trajectories (multiple shooting over many trajectories at once,
 * Sec. VI): the per-interval work of every trajectory is put on one device
 * work list per model, sorted by decreasing substep count, and launched as
 * one kernel per model; the models' kernels run concurrently when the batch
 * is replayed as a HIP graph.
 *
 * A plan binds the buffers of every trajectory at creation (like the
 * single-trajectory calls, all device pointers owned by the caller, same
 * layouts and alignment rules).  Creation is NOT a hot call: it validates,
 * allocates the plan's device memory (descriptors, work lists, and for the
 * reverse sweep the checkpoints and partial sums), uploads it, synchronizes
 * `stream`, and, when asked to tune, times the candidate launch schedules by
 * running the batch (the outputs are then written).  cis_batch_run and
 * cis_batch_graph_run are hot calls: no allocation, no synchronization.  A
 * plan's runs must not overlap each other (they share the plan's device
 * memory); run them on one stream, or order them.
 * ------------------------------------------------------------------------ */
typedef struct cis_batch_plan cis_batch_plan;

/* One trajectory of a batch.  Inputs X, U, s, params and the shape fields
 * mean what they mean for cis_discretize.  Outputs used by CIS_BATCH_DISCRETIZE:
 * A, Bm, Bp, S, defect, xprop (xprop may be NULL).  Used by CIS_BATCH_ADJOINT:
 * defect and xprop (F~ from the forward pass; xprop may be NULL), seed,
 * gX, gU, gs, gparams (as for cis_discretize_adjoint).  Pointers an operation
 * does not use may be NULL. */
typedef struct {
    const cis_model *model;
    int32_t N, substeps;
    int64_t ld_node, ld_int;
    const void *X, *U, *s, *params;
    void *A, *Bm, *Bp, *S, *defect, *xprop;
    const void *seed;
    void *gX, *gU, *gs, *gparams;
} cis_traj;

/* Operations a plan can run (bit mask at creation, one value at run time). */
enum { CIS_BATCH_DISCRETIZE = 1, CIS_BATCH_ADJOINT = 2 };

/* Launch schedule of the discretize kernels, per model.
 *   CIS_SCHED_GRID       one workgroup per (interval, column group) unit;
 *   CIS_SCHED_PERSISTENT a resident grid (occupancy x compute units) takes
 *                        units from a device cursor (reset by the kernel);
 *   CIS_SCHED_TUNE       time both at creation and keep the faster. */
enum { CIS_SCHED_GRID = 1, CIS_SCHED_PERSISTENT = 2, CIS_SCHED_TUNE = 3 };

/* Optional bits of `sched` fixing the form of the reverse sweep (waves per
 * interval) instead of the default: timed at creation with CIS_SCHED_TUNE,
 * else three waves.  4: two waves evaluate alternate stages ahead of the
 * reverse sweep, each evaluation spread over two pipeline steps; 3: one wave
 * evaluates each stage one step ahead (4 and 3 need checkpoints at most 8
 * substeps apart, else 2 is used); 2: replay one chunk ahead; 1: one wave
 * (fewest wave-cycles, for throughput).  At most one of these bits may be
 * set.  The defects pass is likewise timed in its two forms with
 * CIS_SCHED_TUNE. */
enum { CIS_SCHED_ADJ_1 = 0x10, CIS_SCHED_ADJ_2 = 0x20, CIS_SCHED_ADJ_3 = 0x30,
       CIS_SCHED_ADJ_4 = 0x100 };

/* Optional bits of `sched` fixing the register budget of the discretize
 * kernel: CIS_SCHED_WAVES_1 lets it take all the registers its workgroup
 * size allows; CIS_SCHED_WAVES_2 holds it to 256 registers per lane so that
 * two workgroups can share a compute unit (latency hiding, at the price of
 * spills to scratch; CIS_F64 only, else CIS_ERR_DTYPE, except together with
 * CIS_SCHED_SPLIT, whose tangent launch has both budgets in both types).  Workgroups of more
 * than four waves (models with many tangent columns) are held to 256
 * registers in both forms.  Without either bit both FP64 forms are timed
 * with CIS_SCHED_TUNE, and the first is used otherwise.  Setting both bits
 * is an error (CIS_ERR_DIM). */
enum { CIS_SCHED_WAVES_1 = 0x40, CIS_SCHED_WAVES_2 = 0x80 };

/* Optional bits of `sched` fixing the form of the defects pass that the
 * reverse sweep starts from (CIS_BATCH_ADJOINT): CIS_SCHED_DEF_BODY takes
 * two waves per interval (body-lane state recursion and a wave forming the
 * integral rows, as cis_defects), CIS_SCHED_DEF_LANE one wave per interval
 * (element-parallel right-hand side).  Without either bit both are timed
 * with CIS_SCHED_TUNE, and the first is used otherwise.  Setting both bits
 * is an error (CIS_ERR_DIM). */
enum { CIS_SCHED_DEF_BODY = 0x200, CIS_SCHED_DEF_LANE = 0x400 };

/* Optional bits of `sched` fixing the form of the discretize step per model:
 * CIS_SCHED_SPLIT takes the two-launch form of cis_discretize_split for every
 * model with legs with links (others keep the one-launch form);
 * CIS_SCHED_FUSED takes the one-launch form.  Without either bit both forms
 * (and, for the split form, both register budgets of its tangent launch, which
 * CIS_SCHED_WAVES_1/2 otherwise fix) are timed with CIS_SCHED_TUNE, and the
 * one-launch form is used otherwise.  The split form keeps its stage records
 * in plan memory (about 8 (8 + 4 n_j + 4 K R) bytes per interval in FP64, R
 * the record length: 280 for quad13, 120 for cheetah7).  Setting both bits is
 * an error (CIS_ERR_DIM). */
enum { CIS_SCHED_SPLIT = 0x800, CIS_SCHED_FUSED = 0x1000 };

/*
 * Create a plan for n_traj trajectories (all of one dtype; CIS_BATCH_ADJOINT
 * needs CIS_F64).  ckpt_every: substeps between the checkpoints of the reverse
 * sweep; it must divide every trajectory's K, or be 0 to take, per
 * trajectory, the largest divisor of K not above 8.  graph != 0 also builds
 * the HIP graphs used by cis_batch_graph_run.
 * Errors: CIS_ERR_NULL, CIS_ERR_DIM, CIS_ERR_LAYOUT, CIS_ERR_DTYPE,
 * CIS_ERR_UNSUPPORTED (as for the single-trajectory calls, with the offending
 * trajectory named by cis_last_error), CIS_ERR_HIP (allocation, upload,
 * tuning or graph failure).  On error *plan is NULL and nothing is held.
 */
cis_status cis_batch_plan_create(const cis_traj *trajs, int32_t n_traj, cis_dtype dtype,
                                 int32_t ops, int32_t sched, int32_t ckpt_every, int32_t graph,
                                 void *stream, cis_batch_plan **plan);

/* Enqueue one operation (CIS_BATCH_DISCRETIZE or CIS_BATCH_ADJOINT, which
 * must have been requested at creation) of every trajectory on `stream`:
 * the models' launches are issued one after another. */
cis_status cis_batch_run(cis_batch_plan *plan, int32_t op, void *stream);

/* One launch of cis_batch_run for every model group, so that each kernel of
 * an operation can be timed on its own: for CIS_BATCH_DISCRETIZE part 0 is
 * the one-launch kernel or the split form's coefficient-record launch, part 1
 * the split form's tangent launch (nothing for groups in the one-launch form);
 * for CIS_BATCH_ADJOINT part 0 is the defects pass, 1 the reverse sweep, 2
 * the reduction.  Parts of one run must be enqueued in order on one stream
 * (each reads what the previous part wrote).  part out of range: CIS_ERR_DIM. */
cis_status cis_batch_run_part(cis_batch_plan *plan, int32_t op, int32_t part, void *stream);

/* Same work as cis_batch_run, replayed from the plan's HIP graph, in which
 * the models' launches are independent nodes (they may run concurrently). */
cis_status cis_batch_graph_run(cis_batch_plan *plan, int32_t op, void *stream);

/* Description of a plan: number of model groups, and for group g (if
 * 0 <= g < groups) its trajectories, work items (intervals), units per item,
 * the persistent grid size chosen for it (0 = one workgroup per unit), the
 * waves per interval of its reverse sweep (0 without CIS_BATCH_ADJOINT), the
 * register budget of its discretize kernel in waves per SIMD (1 or 2; 0
 * without CIS_BATCH_DISCRETIZE) and the waves per interval of its defects
 * pass (2: body lanes, 1: element lanes; 0 without CIS_BATCH_ADJOINT).  Any
 * output pointer may be NULL. */
cis_status cis_batch_plan_info(const cis_batch_plan *plan, int32_t g, int32_t *groups,
                               int32_t *n_traj, int32_t *n_items, int32_t *units_per_item,
                               int32_t *persist_blocks, int32_t *adjoint_waves,
                               int32_t *waves_per_simd, int32_t *defects_waves);

/*
 * Tuning cache.  With CIS_SCHED_TUNE and the environment variable
 * CIS_TUNE_CACHE naming a file, cis_batch_plan_create looks up each model
 * group's choices (discretize form and register budget, grid or persistent
 * launch, defects form, reverse-sweep waves) under a key made of the device
 * (architecture, compute units), the topology, dtype, operations, the
 * group's number of intervals, its substep range and, with the reverse sweep,
 * its largest checkpoint spacing.  Found: the choices are used without timing.
 * Not found: the group is timed and its choices are added to the file (JSON,
 * written through a temporary file; a missing or unreadable file counts as
 * empty).  *from_cache = 1 when every tuned choice of group g came from the
 * file.  Errors: CIS_ERR_NULL, CIS_ERR_DIM (g out of range).
 */
cis_status cis_batch_plan_tuned_from_cache(const cis_batch_plan *plan, int32_t g,
                                           int32_t *from_cache);

/* Discretize form of group g (0 <= g < groups): *split = 1 when it runs in
 * the split form, with *tangent_waves its register budget (waves per SIMD),
 * else 0 and 0.  Any output pointer may be NULL; g out of range: CIS_ERR_DIM. */
cis_status cis_batch_plan_discretize_form(const cis_batch_plan *plan, int32_t g, int32_t *split,
                                          int32_t *tangent_waves);

/* Release a plan (NULL accepted); synchronizes the device first. */
void cis_batch_plan_destroy(cis_batch_plan *plan);

/* Sizes of the impact-map outputs of a model: n_theta = 10 nc rows of Theta,
 * n_jgv_cols = 7 nb + 2 nc columns of JGv, n_jtc_cols = 14 columns of JTc
 * (any output pointer may be NULL). */
cis_status cis_impact_dims(const cis_model *model, int32_t *n_theta, int32_t *n_jgv_cols,
                           int32_t *n_jtc_cols);

/*
 * Node constraints of the transcribed problem and their Jacobians, for
 * n_nodes nodes at once (Sec. IV-C, eq. cito-impulse and the families
 * Theta^delta, Psi^{delta,eps}; impact model of Sec. II-B, eq. impulse-dynamics).
 * FP64 only.  Per node k, with x~+ = (q+, v+, y+) and x~- = (q-, v-, y-):
 *
 *  G~_k = (q+ - q-, v+ - v*, y+ - y-)                       [nx]
 *    v* = v- + M^-1 (J^T R Phi + grad h^T Lambda), the velocity after the
 *    impact of eq. impulse-dynamics:velocity-change, with the joint impulse
 *    Lambda eliminated by imposing grad h(q) v* = 0 after the impact (the
 *    elimination stated after eq. impulse-dynamics).  Every geometric term
 *    (grad h, J, the contact frame R = [t n]) is taken at the post-impact
 *    pose q+; M = diag(m, m, m L^2/12) per body.
 *  Theta_k, 10 rows per contact i (eq. impulse-dynamics:no-penetration,
 *    eq. elasticity-impact, eq. max-diss-impulse-KKT:stationarity,
 *    eq. impulse-friction-cone, relaxed with FB^delta(a, b) =
 *    a + b - sqrt(a^2 + b^2 + delta) of eq. FB-relax):
 *      FB(Phi_n, sd), FB(Phi_n, w), Phi_n lam - delta, -Phi_n lam - delta,
 *      FB(Gamma, rho), -Phi_n, -sd, -w, -Gamma, -rho          (all <= 0)
 *    with w = n^T J (v+ + e v-), lam = t^T J v+ + Gamma Phi_t / sqrt(Phi_t^2 + 1),
 *    rho = |mu Phi_n|_s - |Phi_t|_s, |a|_s = sqrt(a^2 + 1) - 1.
 *  Psi_k (k < n_nodes - 1) = (y-_{k+1} - y+_k) - (delta for the nc
 *    cross-complementarity states, eps for the violation state)   [ny]
 *
 * Inputs (DEVICE, FP64, node index contiguous like X of cis_discretize):
 *   Xp, Xm [nx][ld_node]   post- and pre-impact augmented states
 *   Phi    [2 nc][ld_node] (Phi_t, Phi_n) of contact 0, then contact 1, ...
 *   Gamma  [nc][ld_node]   friction multipliers
 *   params [P] = (mu, e, masses)
 * Outputs (DEVICE, FP64, node-major, packed; every entry written):
 *   G     [n_nodes][nx]
 *   Theta [n_nodes][10 nc]
 *   JGv   [n_nodes][3 nb][7 nb + 2 nc]  dG~_{velocity rows} / d w with
 *         w = (q+ [3 nb], v- [3 nb], Phi [2 nc], masses [nb])
 *   JTc   [n_nodes][10 nc][14]  dTheta_{10 i + r} / d w_i with
 *         w_i = (q+_b [3], v+_b [3], v-_b [3], Phi_t_i, Phi_n_i, Gamma_i, mu, e),
 *         b the body of contact i
 *   Psi   [n_nodes - 1][ny], or NULL to skip
 * Entries of the full Jacobians outside these blocks are the same for every
 * node and are not written: dG~/d(x~+, x~-) is +I / -I on the pose and
 * integral-state rows, dG~_v/dv+ = I, and every other derivative of G~
 * (v+ rows by q-, y+, y-, Gamma, mu, e) and of Theta (by q-, y+, y-, and the
 * other contacts' variables) is 0; dPsi_k/dy+_k = -I, dPsi_k/dy-_{k+1} = I.
 *
 * delta > 0 and finite, eps finite; ld_node >= max(n_nodes, 1); n_nodes = 0
 * enqueues nothing and checks no pointer.  Phi, Gamma, Theta and JTc may be NULL when nc = 0.
 * Errors: CIS_ERR_NULL, CIS_ERR_DIM, CIS_ERR_LAYOUT (pointers must be 8-byte
 * aligned), CIS_ERR_UNSUPPORTED, CIS_ERR_HIP.
 */
cis_status cis_impact_linearize(const cis_model *model, int32_t n_nodes, int64_t ld_node,
                                const double *Xp, const double *Xm, const double *Phi,
                                const double *Gamma, const double *params, double delta,
                                double eps, double *G, double *Theta, double *JGv, double *JTc,
                                double *Psi, void *stream);

/*
 * Sparse LDL^T factorization of a symmetric quasi-definite matrix (host
 * memory, host code): the reduced KKT system [P + G^T D G + r I, A^T; A, -r I]
 * that the interior-point solver of the SCP driver's convex subproblems
 * factors at every iteration (the prox-linear subproblem of Sec. V, solved in
 * canonical form as in Sec. VI).  Quasi-definite matrices factor in any
 * symmetric order without pivoting, so the caller chooses the elimination
 * order (fill-reducing) and passes the permuted matrix.
 *
 * The matrix (n x n) is given by its upper triangle, diagonal included, in
 * compressed sparse columns: column k holds rows Ai[Ap[k] .. Ap[k+1]-1]
 * (each <= k, any order, no duplicates) with values Ax.
 *
 * cis_ldl_symbolic: elimination tree parent[n] (-1 at roots) and the number
 * of entries Lnz[n] of each column of the unit lower factor L (diagonal
 * excluded); work[n] is scratch.  Returns nnz(L) >= 0, -1 on a NULL pointer
 * or n < 0, -2 on an entry below the diagonal.
 *
 * cis_ldl_numeric: L (columns Lp[n+1], Li/Lx[nnz(L)], strictly lower) and
 * D[n] with A = L D L^T; iwork[3n] and y[n] are scratch.  With sign[n]
 * (+1 / -1: the expected sign of each pivot, e.g. +1 on the primal block and
 * -1 on the multiplier block of a KKT matrix) a pivot d with sign * d <= eps
 * is replaced by sign * delta (dynamic regularization; the factor is then
 * that of a nearby matrix); sign may be NULL (no replacement).  Returns the
 * number of replaced pivots, -1 on a NULL pointer, -2 on a NaN pivot or (sign
 * NULL) a zero pivot.
 *
 * cis_ldl_solve: x <- (L D L^T)^-1 x in place (x[n]).
 * All arrays are caller-owned; nothing is allocated or retained.
 */
int64_t cis_ldl_symbolic(int32_t n, const int32_t *Ap, const int32_t *Ai, int32_t *parent,
                         int32_t *Lnz, int32_t *work);
int32_t cis_ldl_numeric(int32_t n, const int32_t *Ap, const int32_t *Ai, const double *Ax,
                        const int32_t *parent, const int32_t *Lnz, const int8_t *sign, double eps,
                        double delta, int32_t *Lp, int32_t *Li, double *Lx, double *D,
                        int32_t *iwork, double *y);
void cis_ldl_solve(int32_t n, const int32_t *Lp, const int32_t *Li, const double *Lx,
                   const double *D, double *x);

#ifdef __cplusplus
}
#endif

#endif /* CIS_H */
