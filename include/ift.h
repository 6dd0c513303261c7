/*
 * ift.h -- C ABI of the EQ-hyperreduced implicit-feature-tracking assembly
 * library for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for a DG discretisation of a 2-D conservation law
 * posed on a reference domain deformed by a mapping x = X + Psi tau, the
 * element residuals R_e and mesh-distortion residuals N_e, their Jacobians,
 * and the empirical-quadrature (EQ) weighted reduced quantities of
 * Mirhoseini & Zahr, "Accelerated solutions of convection-dominated partial
 * differential equations using implicit feature tracking and empirical
 * quadrature":
 *   - the full-order element loop of eq. (hdm_elem) / (hdm_elem_jac1)
 *     (hdm_assemble);
 *   - the hyperreduced objective J~ of eq. (ift-opt-eqp2) and the stacked
 *     residual F~ of eq. (ift-eqp-res) (eq_assemble_residual);
 *   - the hyperreduced residuals [S~; T~] = J~_z^T F~ of eq. (ift-eqp-res0)
 *     and the Gauss-Newton matrix J~_z^T J~_z of eq. (levmarq-elem)
 *     (eq_assemble_jacobian);
 *   - one Levenberg-Marquardt step of eq. (levmarq-step)/(lmstep) with a
 *     sufficient-decrease line search (rom_gauss_newton_step).
 *
 * Conventions (all arrays row-major, FP64 at the boundary):
 *   - element nodes: 3 vertices (counter-clockwise), then for degree 2 the
 *     mid-edge nodes of edges 0,1,2; edge f joins vertex f and vertex f+1;
 *     face f of an element is edge f.  The mapping has the degree of the
 *     solution (q = p), so geometry nodes and solution nodes coincide per
 *     element.
 *   - state U[(e*nn + i)*nc + c] (element-major; DG blocks are disjoint);
 *     mapping coefficients x[2*gnode + d].
 *   - element DoFs U_e (nue = nn*nc), neighbour face-trace DoFs U_e'
 *     (nun = 3*(p+1)*nc: for face f and edge node k ordered from vertex f to
 *     vertex f+1, the neighbour's DoFs at that node; zero on boundary faces),
 *     element mapping DoFs x_e (nxe = 2*nn).
 *   - mu: host pointer; Burgers: mu[0] (inflow u_b = 1 + bc_mu_scale*mu[0],
 *     or u_b = mu[0] on the left edge with bc_spacetime) and, when the
 *     problem has the source of eq. (burgers), mu[1] = its rate b;
 *     Euler: mu[0] = free-stream Mach number, mu[1] = inflow angle (deg).
 *   - unless stated otherwise, every array argument is a DEVICE pointer
 *     owned by the caller; the library never frees caller memory.
 *   - every call runs on the caller's stream and returns after enqueueing
 *     the work, except where it says it synchronises.
 *
 * Errors: calls return an ift_status.  Negative values are hard errors
 * (arguments rejected before any work was enqueued, or a HIP failure);
 * outputs are then unspecified.  Invalid geometry (mapping Jacobian
 * determinant g <= eps_g at a volume quadrature point) or a non-physical
 * Euler state (rho <= 0 or p <= 0 at a flux evaluation point) at an
 * evaluation point is a soft outcome: the objective is +inf and the element
 * is counted in n_bad; a line search then rejects the point.
 *
 * Handles are not thread-safe: use one handle on one stream at a time.
 */
#ifndef IFT_H
#define IFT_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IFT_OK = 0,
  IFT_EINVAL = -1,      /* bad argument (null pointer, size, index, mesh)  */
  IFT_ENOMEM = -2,      /* device allocation failed                        */
  IFT_EDEVICE = -3,     /* HIP runtime error                               */
  IFT_EBADMESH = -4,    /* invalid geometry at the evaluation point        */
  IFT_ENONPHYS = -5,    /* non-physical state at the evaluation point      */
  IFT_ESINGULAR = -6,   /* Gauss-Newton matrix not positive definite        */
  IFT_ELINESEARCH = -7, /* no sufficient decrease within max_backtrack      */
  IFT_ENOTCONV = -8,    /* iteration limit reached                          */
  IFT_ESCRATCH = -9     /* the workspace exceeds the fixed scratch of the
                           no-allocation entry point                        */
} ift_status;

typedef enum { IFT_BURGERS2D = 0, IFT_EULER2D = 1 } ift_pde;

/* Internal precision (the boundary is always FP64):
 *   IFT_FP64        everything in FP64;
 *   IFT_FP32_ELEM   element fluxes and point Jacobians in FP32, projection,
 *                   Gram and solves in FP64;
 *   IFT_MIXED_BF16  element fluxes and point Jacobians in FP32, the
 *                   projection Phi_e^T J_e [Phi_e Psi_e] on BF16 matrix cores
 *                   with FP32 accumulation; the Gram matrix, gradient and
 *                   objective are accumulated and the normal equations
 *                   solved in FP64.  The batched solver finishes such
 *                   instances with FP64 refinement rounds (see
 *                   rom_gauss_newton_solve_batched). */
typedef enum { IFT_FP64 = 0, IFT_FP32_ELEM = 1, IFT_MIXED_BF16 = 2 } ift_precision;

typedef struct ift_problem ift_problem;
typedef struct ift_rom ift_rom;

/* Mesh and discretisation.  All pointers are HOST pointers, copied at
 * creation.  elem_nbr[e*3+f] is the element across face f or -tag with tag
 * 1 (left), 2 (right), 3 (bottom), 4 (top); interior neighbours must be
 * mutual.  Boundary states (Section 4 reading): Burgers tags 1,3 inflow
 * u+ = 1 + bc_mu_scale*mu[0], or with bc_spacetime = 1 the data of the
 * space-time problem eq. (burgers), u+ = mu[0] on tag 1 (x = 0) and u+ = 1
 * on tag 3 (t = 0); tags 2,4 outflow u+ = u-; Euler tag 1 supersonic inflow
 * u+ = U_inf(mu), tag 2 supersonic outflow, tags 3,4 slip walls;
 * all_farfield != 0 makes every Euler tag an inflow.
 * src_amp != 0 (Burgers only) adds the source of eq. (burgers),
 * s(x) = src_amp exp(mu[1] x) at the mapped physical position x (on the
 * reference domain S = g s); every call then reads mu[0] and mu[1].  Euler
 * problems must leave src_amp = 0 and bc_spacetime = 0 (else IFT_EINVAL). */
typedef struct {
  ift_pde pde;
  int p;                   /* DG degree = mapping degree, 1 or 2          */
  int n_elem;
  int n_gnode;
  const double* X;         /* [n_gnode][2] reference node coordinates      */
  const int* elem_gnodes;  /* [n_elem][nn] geometry node ids               */
  const int* elem_nbr;     /* [n_elem][3]                                  */
  double gamma;            /* ratio of specific heats (Euler)              */
  double kappa;            /* distortion weight, eq. (dist_elem0)          */
  double eps_g;            /* eps of eq. (dist_elem1); also validity bound */
  double bc_mu_scale;      /* Burgers inflow scale                         */
  int all_farfield;
  double src_amp;          /* Burgers source amplitude (0.02 in eq. (burgers); 0: none) */
  int bc_spacetime;        /* Burgers: 1 = space-time boundary data        */
} ift_problem_desc;

ift_status ift_problem_create(const ift_problem_desc* desc, ift_problem** out);
void ift_problem_destroy(ift_problem* prob);
/* Sizes of the problem: nue, nun, nxe, N_u, N_x (any may be NULL). */
ift_status ift_problem_sizes(const ift_problem* prob, int* nue, int* nun, int* nxe,
                             long long* N_u, long long* N_x);
/* The neighbour DoF map built at creation (the assembly operator of the
 * neighbour traces U_e' in eq. (hdm_elem)): Pn HOST, caller-allocated
 * [n_elem][nun]; entry (e, f, k, c) is the index into U of component c of
 * the neighbour across face f at e's edge node k (edge order of e), or -1
 * on a boundary face.  With it the element blocks of hdm_assemble assemble
 * into the global sparse Jacobian dR/dU (the snapshot alignment of
 * eq. (align0)).  IFT_EINVAL for null arguments. */
ift_status ift_problem_neighbour_map(const ift_problem* prob, long long* Pn);

/* Full-order element loop over all n_elem elements (eq. (hdm_elem) and
 * eq. (hdm_elem_jac1), distortion eq. (dist_elem0)-(dist_elem1)).
 * In: U [N_u], x [N_x].  Out (each may be NULL to skip):
 *   R [N_u] global residual (element blocks are disjoint, P_e^T P_E = delta),
 *   N [n_elem], dRdU [n_elem][nue][nue], dRdUn [n_elem][nue][nun],
 *   dRdx [n_elem][nue][nxe], dNdx [n_elem][nxe],
 *   n_bad [1] (int): elements with invalid geometry or state.
 * The Jacobian blocks are computed only if at least one of them is
 * requested. */
ift_status hdm_assemble(ift_problem* prob, const double* mu, const double* U, const double* x,
                        double* R, double* N, double* dRdU, double* dRdUn, double* dRdx,
                        double* dNdx, int* n_bad, hipStream_t stream);

/* The indicator of the greedy search, eq. (greedy0): for each of n_pts
 * reduced solutions (w_p, tau_p) at mu_p, the 2-norm of the full-order DG
 * residual |R(Phi w_p; X + Psi tau_p, mu_p)|_2 over all n_elem elements
 * (eq. (hdm_elem); the distortion is not part of it), evaluated element by
 * element without forming Phi w or X + Psi tau.  All arrays DEVICE: mu
 * [n_pts][2], Phi [N_u][n] and Psi [N_x][m] row-major (the bases the ROM
 * was built from), w [n_pts][n], tau [n_pts][m]; out: norms [n_pts] (+inf
 * where an element has invalid geometry or state), n_bad [n_pts] (may be
 * NULL) the number of such elements.  The argmax over the candidates picks
 * the next training parameter.  The problem keeps a workspace of
 * n_pts * ceil(n_elem / 16) doubles and ints, allocated or grown by the
 * call that first needs it. */
ift_status hdm_residual_norm_batched(ift_problem* prob, int n_pts, const double* mu, const double* Phi, int n,
                                     const double* w, const double* Psi, int m, const double* tau, double* norms,
                                     int* n_bad, hipStream_t stream);

/* Reduced-order model with EQ set {(e_k, rho_k)}, k < n_s.  Phi [N_u][n]
 * and Psi [N_x][m] are DEVICE pointers, only read during creation;
 * eq_elem [n_s] and eq_rho [n_s] are HOST pointers (rho_k >= 0).  Creation
 * gathers Phi_e = P_e^T Phi, Phi_e' = P_e'^T Phi, Psi_e = Q_e^T Psi and
 * X_e = Q_e^T X for every sampled element (end of Section 3.0) into
 * library-owned device memory, with the reduced bases evaluated at the
 * quadrature points.  The per-point workspaces of the single-instance
 * calls are allocated by the first such call (or by ift_rom_reserve), so
 * a handle used only through a batch never holds them; later calls
 * allocate nothing.  Limits: 1 <= n, 0 <= m, n + m <= 64, n_s >= 1.
 * Synchronises the stream of the default device context. */
ift_status ift_rom_create(ift_problem* prob, int n, int m, const double* Phi, const double* Psi,
                          int n_s, const int* eq_elem, const double* eq_rho,
                          ift_precision precision, ift_rom** out);
void ift_rom_destroy(ift_rom* rom);
/* Copies of the gathered operands (device outputs, bit-exact copies of the
 * rows of Phi, Psi, X): Phi_s [n_s][nue][n], Phin_s [n_s][nun][n] (zero rows on
 * boundary faces), Psi_s [n_s][nxe][m], X_s [n_s][nxe]; any may be NULL. */
ift_status ift_rom_get_gathers(ift_rom* rom, double* Phi_s, double* Phin_s, double* Psi_s,
                               double* X_s, hipStream_t stream);

/* Hyperreduced residual at z = (w [n], tau [m]) (device inputs):
 *   Jobj [1]  = sum_k rho_k/2 (|R_e|^2 + N_e^2), +inf if invalid,
 *   Ft [n_s*nue + n_s] = [sqrt(rho_k) R_e (k-major) ; sqrt(rho_k) N_e] or NULL,
 *   PhiT_r [n] = sum_k rho_k Phi_e^T R_e or NULL,
 *   n_bad [1] (int) or NULL. */
ift_status eq_assemble_residual(ift_rom* rom, const double* mu, const double* w, const double* tau,
                                double* Jobj, double* Ft, double* PhiT_r, int* n_bad,
                                hipStream_t stream);

/* Hyperreduced gradient and Gauss-Newton matrix at z = (w, tau):
 *   Jobj [1] as above,
 *   g [n+m] = [S~; T~] (eq. (ift-eqp-res0)),
 *   H [n+m][n+m] = J~_z^T J~_z (eq. (levmarq-elem)),
 *   Jt [n_s*nue + n_s][n+m] = rows sqrt(rho_k)[A_e B_e] then sqrt(rho_k)[0 a_e]
 *     with A_e = dR_e/dU_e Phi_e + dR_e/dU_e' Phi_e', B_e = dR_e/dx_e Psi_e,
 *     a_e = dN_e/dx_e Psi_e, or NULL,
 *   n_bad [1] or NULL. */
ift_status eq_assemble_jacobian(ift_rom* rom, const double* mu, const double* w, const double* tau,
                                double* Jobj, double* g, double* H, double* Jt, int* n_bad,
                                hipStream_t stream);

/* eq_assemble_jacobian for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results (Jobj, g, H, n_bad as
 * above; no Jt), with the workspace (point data, block partials, flag
 * counts; eq_noalloc_scratch_bytes) in one static device array of
 * IFT_NOALLOC_SCRATCH_BYTES that each device holds from the library's load
 * until the process ends.  The call allocates nothing; mu is HOST [2], w, tau,
 * Jobj, g, H, n_bad are DEVICE.  Every call on a device shares its array:
 * calls that overlap on one device (other streams, other threads) race and
 * must be serialised by the caller.  IFT_ESCRATCH when the ROM's workspace
 * exceeds the array (about 4,900 sampled elements of a P2 Euler ROM),
 * IFT_EINVAL on null outputs or a ROM whose D + 1 exceeds 48. */
#define IFT_NOALLOC_SCRATCH_BYTES (32u << 20)
ift_status eq_assemble_jacobian_noalloc(ift_rom* rom, const double* mu, const double* w, const double* tau,
                                        double* Jobj, double* g, double* H, int* n_bad, hipStream_t stream);
/* Bytes of that workspace for this ROM (0 for a NULL handle). */
size_t eq_noalloc_scratch_bytes(const ift_rom* rom);

/* The elemental reduced residuals of eq. (ift-eqp-res0), the data of the
 * EQ-weight training program eq. (eqp-lp)-(eqp-con): for every sampled
 * element k (element e_k = eq_elem[k]) at (mu, w, tau),
 *   C[k] = [S^(e_k); T^(e_k)] = [A_k R_k; a_k N_k] contracted as in g,
 * WITHOUT the weight rho_k (so that sum_k rho_k C[k] = [S~; T~]).  Build the
 * ROM on all elements with rho = 1 to obtain the columns of the program at
 * a training solution.  mu HOST [2]; w, tau, C DEVICE; C [n_s][n + m]
 * row-major.  rho_k must be nonzero. */
ift_status eq_element_contributions(ift_rom* rom, const double* mu, const double* w, const double* tau, double* C,
                                    hipStream_t stream);

/* Batched evaluation: n_pts evaluation points (mu_p, w_p, tau_p) of the same
 * ROM in one launch (e.g. many parameters, or several line-search trial
 * points).  ift_rom_reserve sizes the per-point workspaces for up to
 * max_pts points (it allocates, and synchronises the device); the batched
 * calls then allocate nothing and require n_pts <= max_pts.
 * mu [n_pts][2] (DEVICE; Burgers uses mu[p][0]), w [n_pts][n],
 * tau [n_pts][m]; outputs Jobj [n_pts], g [n_pts][n+m], H [n_pts][n+m][n+m],
 * n_bad [n_pts] or NULL, each with the meaning of the single-point call. */
ift_status ift_rom_reserve(ift_rom* rom, int max_pts);
ift_status eq_assemble_residual_batch(ift_rom* rom, int n_pts, const double* mu, const double* w,
                                      const double* tau, double* Jobj, int* n_bad, hipStream_t stream);
ift_status eq_assemble_jacobian_batch(ift_rom* rom, int n_pts, const double* mu, const double* w,
                                      const double* tau, double* Jobj, double* g, double* H, int* n_bad,
                                      hipStream_t stream);

typedef struct {
  double lambda;       /* LM weight on the tau block (0 = Gauss-Newton)     */
  double c1;           /* sufficient-decrease constant (1e-4)               */
  int max_backtrack;   /* step halvings (30)                                */
  double tol;          /* |S~| <= tol and |T~| <= tol (1e-8)                */
  double tol_mix;      /* mixed-precision batches: gradient norms at which an
                          instance continues in FP64 rounds (<= 0: the
                          default max(tol, 1e-5))                          */
  int max_backtrack_mixed; /* mixed-precision batches: halvings without
                          decrease after which an instance continues in
                          FP64 rounds (<= 0: the default 3)                 */
  int use_qr;          /* rom_gauss_newton_step: 1 solves the least-squares
                          form of eq. (levmarq-step) by Householder QR of
                          the stacked rows (needs n + m + 1 <= 48); 0 the
                          normal equations (lmstep) by Cholesky.  Batched
                          solves use the normal equations and reject 1.    */
  int w_only;          /* rom_gauss_newton_step: 1 steps in w with tau held
                          (dz_tau = 0) and converges on |S~| <= tol alone:
                          the iteration of the paper's initialisation
                          w0 = argmin_w |R~(w, tau0)| (remark rem:solver)  */
} ift_gn_params;

typedef struct {
  double J_old, J_new, alpha, norm_S, norm_T; /* norms at the input point  */
  int n_backtrack;
  int converged;       /* input point meets tol; no step taken              */
  int status;          /* an ift_status                                     */
  int iterations;      /* LM steps taken (batched solve; 0 or 1 for a step) */
  int fallback;        /* batched solve with a warm start: 1 if the plain
                          start was used instead; 2 if the warm start was
                          kept but its line search failed, so the solve
                          restarted from the plain start                   */
  int mixed_iterations; /* batched mixed-precision solve: LM steps taken in
                          mixed-precision rounds (the rest ran in FP64)    */
  int presolve_iterations; /* batched solve with the w-only initialisation:
                          steps taken in w only                           */
} ift_gn_info;

/* One Levenberg-Marquardt step from z_n = (w, tau) (device, in/out):
 * assemble at z_n; if |S~| <= tol and |T~| <= tol report convergence;
 * otherwise solve (H + lambda diag(0, I)) dz = -g (FP64 Cholesky; with
 * params->use_qr the equivalent least-squares problem by Householder QR of
 * the stacked rows, whose workspace the first such call allocates) and
 * backtrack alpha = 1, 1/2, ... until J~(z + alpha dz) <= J~(z) +
 * c1 alpha g.dz, then overwrite (w, tau).  Both objectives of that test
 * come from the residual kernels of eq_assemble_residual, summed in one
 * order (J~(z) is evaluated once more for it).  info is a HOST pointer.
 * Synchronises the stream. */
ift_status rom_gauss_newton_step(ift_rom* rom, const double* mu, double* w, double* tau,
                                 const ift_gn_params* params, ift_gn_info* info, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched solves.  A batch groups n_inst ROM handles (each with its own
 * bases, EQ set and weights; all on one problem, each with n + m + 1 <= 48)
 * that are solved together, each at its own mu, by the Levenberg-Marquardt
 * iteration of rom_gauss_newton_step (same step, line search and stopping
 * rule), advanced on the device without host synchronisation.  The
 * reduced coordinates of all instances are packed: instance i occupies
 * z[zoff[i] .. zoff[i+1]) as (w_i, tau_i), zoff from ift_batch_layout.
 * The batch owns every workspace; a handle is used on one stream at a time.
 * ------------------------------------------------------------------------ */
typedef struct ift_batch ift_batch;

/* roms: host array of n_inst handles (not owned; they must outlive the
 * batch).  IFT_EINVAL when n_inst < 1, a handle is null, the handles do not
 * share one problem and precision, or an instance has n + m + 1 > 48. */
ift_status ift_batch_create(int n_inst, ift_rom* const* roms, ift_batch** out);
void ift_batch_destroy(ift_batch* batch);

/* Packed offsets (HOST arrays of n_inst + 1 ints, either may be null):
 * zoff for z and g (steps of n_i + m_i), hoff for H (steps of (n_i + m_i)^2). */
ift_status ift_batch_layout(const ift_batch* batch, int* zoff, int* hoff);

/* Picks the elements-per-wave work split of the fused assembly for this
 * batch by timing the candidates {4, 8, 16, 32} on the Jacobian assembly at
 * (mu, z) (device arrays as below), with every instance active and with one
 * instance in eight (weighted 4:1 for the late rounds of a solve, where few
 * instances remain; the fastest of four runs each), a larger split being
 * taken only when 3 % faster; the choice is kept by the handle.
 * Synchronises the stream.  *chosen (host, may be null) receives it. */
ift_status ift_batch_autotune(ift_batch* batch, const double* mu, const double* z, int* chosen, hipStream_t stream);

/* [S~; T~], J~_z^T J~_z and J~ of every instance at its (mu, z): mu device
 * [n_inst][2], z device packed; g packed like z, H packed by hoff, Jobj and
 * n_bad device [n_inst] (n_bad may be null).  Same quantities as
 * eq_assemble_jacobian, instance by instance. */
ift_status eq_assemble_jacobian_batched(ift_batch* batch, const double* mu, const double* z, double* Jobj, double* g,
                                        double* H, int* n_bad, hipStream_t stream);

/* Solves every instance from its start z (device, packed, overwritten by
 * the last iterate) at mu (device [n_inst][2]): at most max_it LM steps per
 * instance (max_it >= 0), each as in rom_gauss_newton_step with `params`.
 * info: DEVICE array [n_inst]; per instance J_old = J~ at the start, J_new
 * = J~ at the last iterate, alpha = last accepted step length, norm_S /
 * norm_T at the last iterate, n_backtrack = halvings over all steps,
 * converged, iterations, and status: IFT_OK (converged), IFT_ENOTCONV
 * (max_it reached), IFT_ELINESEARCH, IFT_ESINGULAR, IFT_EBADMESH or
 * IFT_ENONPHYS (invalid iterate).  flags bit 0 = 1: launch the kernels
 * directly instead of replaying the captured HIP graph (same results).
 * flags bit 1 = 1: z holds warm starts (e.g. from ift_mlp_predict); J~ is
 * evaluated (FP64) at each warm start and at the plain start, and an
 * instance starts from the plain start unless its warm start has the
 * smaller J~ (info.fallback = 1 then).  An instance that keeps its warm
 * start and whose line search then fails restarts once from the plain start
 * (info.fallback = 2; its iteration count continues).
 * flags bit 2 = 1: the paper's initialisation (remark rem:solver): each
 * instance first takes steps in w with tau held at its start value (the
 * w_only step of rom_gauss_newton_step) until |S~| <= tol (the mixed-phase
 * tolerance in mixed rounds) or its line search fails, then full steps;
 * all steps count towards max_it (info.presolve_iterations: the w steps).
 * flags bit 3 = 1: adaptive lambda per instance, starting from
 * params->lambda: lambda / 10 after a step accepted at alpha = 1 (0 below
 * 1e-12), max(10 lambda, 1e-8) after a step accepted at alpha < 1.
 * params->use_qr and params->w_only must be 0.
 * The full step z + dz is taken first and tested by the next Jacobian
 * assembly: the sufficient-decrease test at alpha = 1 compares the
 * objectives of two Jacobian assemblies.  A rejected step restores z,
 * re-evaluates J~(z) with the trial residual kernels and backtracks from
 * alpha = 1/2 with trial residual evaluations, so that every test compares
 * objectives summed by the same kernels in the same order.
 * The rounds (Jacobian assembly, LM step, two line-search trials) run in
 * replays of four captured rounds; after each replay the stream is
 * synchronised to read how many instances are still running.  Returns
 * IFT_OK when the launches succeeded (per-instance outcomes are in info). */
ift_status rom_gauss_newton_solve_batched(ift_batch* batch, const double* mu, double* z, const ift_gn_params* params,
                                          int max_it, ift_gn_info* info, int flags, hipStream_t stream);

/* The plain start of the reduced iteration: w0 = Phi^T U_fs(mu), the
 * reduced coordinates of the uniform free stream (Euler) or of the inflow
 * value (Burgers) on every node (Phi has orthonormal columns), and tau0 = 0,
 * the unmapped mesh.  rom_plain_start: mu HOST [2], w and tau DEVICE;
 * rom_plain_start_batched: mu DEVICE [n_inst][2], z DEVICE packed. */
ift_status rom_plain_start(ift_rom* rom, const double* mu, double* w, double* tau, hipStream_t stream);
ift_status rom_plain_start_batched(ift_batch* batch, const double* mu, double* z, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Warm-start network: z0 = y_mean + y_scale * f((mu - x_mean) / x_scale),
 * f = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3 with gelu(t) = t Phi(t), a map
 * from the parameters mu to the reduced coordinates (w, tau) of converged
 * solves, used to seed rom_gauss_newton_solve_batched.  Parameters are one
 * flat FP32 DEVICE array: for each layer W [out][in] row-major, then b.
 * Training (ift_mlp_train) runs full-batch Adam (beta 0.9, 0.999, eps 1e-8)
 * on the mean squared error of the normalised outputs, all in FP32 on the
 * device with fixed-order reductions; inference runs in FP32 or with BF16
 * weights and activations on matrix cores (FP32 accumulation).
 * Limits: n_in <= 8, hidden <= 256, n_out <= 64.
 * ------------------------------------------------------------------------ */
typedef struct ift_mlp ift_mlp;

/* Weights W_l ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a splitmix64 stream
 * seeded with `seed`, biases 0, identity normalisation. */
ift_status ift_mlp_create(int n_in, int hidden, int n_out, unsigned long long seed, ift_mlp** out);
void ift_mlp_destroy(ift_mlp* mlp);
ift_status ift_mlp_num_params(const ift_mlp* mlp, int* n);
ift_status ift_mlp_set_params(ift_mlp* mlp, const float* params, hipStream_t stream);   /* resets Adam */
ift_status ift_mlp_get_params(const ift_mlp* mlp, float* params, hipStream_t stream);
/* HOST arrays x_mean, x_scale [n_in], y_mean, y_scale [n_out] (scales > 0). */
ift_status ift_mlp_set_normalization(ift_mlp* mlp, const double* x_mean, const double* x_scale, const double* y_mean,
                                     const double* y_scale);
/* Loss (mean squared error over samples and outputs) and its gradient at
 * the current parameters for normalised data X [N][n_in], T [N][n_out]
 * (DEVICE, FP32); grad DEVICE [n_params] (may be null), loss HOST (may be
 * null; then the call does not synchronise). */
ift_status ift_mlp_loss_grad(ift_mlp* mlp, const float* X, const float* T, int N, float* grad, double* loss,
                             hipStream_t stream);
/* `steps` Adam steps with learning rate lr on mu [N][n_in], z [N][n_out]
 * (DEVICE, FP64, normalised internally); loss_hist HOST [steps] or null.
 * Synchronises the stream. */
ift_status ift_mlp_train(ift_mlp* mlp, const double* mu, const double* z, int N, int steps, double lr,
                         double* loss_hist, hipStream_t stream);
/* z [N][n_out] (DEVICE, FP64) from mu [N][n_in]; bf16 != 0: BF16 matrix cores. */
ift_status ift_mlp_predict(ift_mlp* mlp, const double* mu, int N, double* z, int bf16, hipStream_t stream);

/* Kernel timing.  While enabled, every launch of the library's element
 * kernels and reductions is bracketed by HIP events on the caller's stream
 * (events are created on first use and reused).  ift_profile_read
 * synchronises on the recorded events and returns, for kernel class
 * `which` (IFT_PROF_*), the number of launches and their summed duration in
 * milliseconds since the last reset.  Not thread-safe. */
enum {
  IFT_PROF_HDM = 0,     /* full-order assembly / values kernels              */
  IFT_PROF_EQ_RES = 1,  /* EQ residual kernel                                */
  IFT_PROF_EQ_JAC = 2,  /* EQ Jacobian assembly + projection kernel          */
  IFT_PROF_GRAM = 3,    /* Gram reduction (both stages)                      */
  IFT_PROF_POINTS = 4,  /* point-physics kernels of the Jacobian paths       */
  IFT_PROF_NKIND = 5
};
ift_status ift_profile_enable(int on);
ift_status ift_profile_reset(void);
ift_status ift_profile_read(int which, int* count, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* IFT_H */
