/*
 * feh.h -- finite-element-projection FFT homogenization on MI355X (gfx950).
 *
 * A C ABI around hand-written HIP kernels that solve small-strain periodic
 * homogenization on a fully structured grid of linear finite elements with
 * the finite-element compatibility projection of Leute et al.,
 * "Elimination of ringing artifacts by finite-element projection in
 * FFT-based homogenization" (arXiv 2105.03297).
 *
 * The method (paper sections cited by title):
 *   - Sec. "Compatibility projection": equilibrium in weak form with test
 *     strains projected by a self-adjoint operator G onto compatible fields;
 *     the strain is the unknown and the mean strain Ebar is the macroscopic
 *     boundary condition (carried by k = 0).
 *   - Sec. "Discrete projection": G built from a discrete derivative symbol,
 *     block diagonal in Fourier space; the DFT only accelerates a convolution.
 *   - Sec. "Linear finite elements": 2 linear triangles per pixel (2D); the
 *     3D generalisation used here is 6 Kuhn tetrahedra per voxel.
 *   - Small-strain appendix: G = B (B^*B)^-1 B^* per wavevector, with
 *     e_T = sym(grad_T u) per element T.
 *   - Discrete Fourier transform appendix: grid, wavevectors, transform pair.
 *
 * The solver runs projected conjugate gradients on G K in strain space in
 * its factored form: every Krylov vector is a nodal displacement field (D
 * reals per voxel), B and B^T are applied as real-space stencils and only
 * (B^*B)^-1, a D x D Hermitian matrix per wavevector, is applied in Fourier
 * space.  This is iterate-for-iterate the same as CG on the strain field,
 * and its converged strain is the canonical FE strain.
 *
 * Conventions
 *   - Grid: dim = 2 or 3, sizes n[0..dim-1]; arrays are C-ordered with the
 *     last axis fastest; N = prod n.  Node (i,j[,k]) is the lower-left
 *     corner of voxel (i,j[,k]); voxel sizes h[a] (Delta_a).
 *   - Elements per voxel n_e: 2D e=0 nodes 00,10,01, e=1 nodes 11,01,10;
 *     3D e = axis paths (x,y,z),(x,z,y),(y,x,z),(y,z,x),(z,x,y),(z,y,x),
 *     tetrahedron with vertices 0, e_a0, e_a0+e_a1, (1,1,1).
 *   - Material: isotropic, per voxel Lame constants (lambda, mu); 2D is
 *     plane strain when set from (E, nu).  E = 0 (vacuum) is accepted.
 *   - Precision: FEH_FP64 runs everything in double.  FEH_FP32 stores and
 *     streams fields, stencils and FFTs in float and applies the
 *     per-wavevector inverse (B^*B)^-1 in float; that inverse is formed in
 *     float from dimensionless phase factors, except at long wavelengths
 *     (|k| h_max below about 1/4), where it is formed in double and rounded
 *     once.  The CG dot products and alpha/beta stay in double (fixed-order
 *     sums), and so do the post-processing sums (<sigma>, W, sensitivities).
 *   - Nodal vector fields at the ABI are [n_load][N][D] and element fields
 *     [n_load][N][n_e][D][D], in the plan's precision (float or double).
 *   - All device pointers are caller-owned device memory (e.g. torch
 *     tensors); the library never allocates or frees device memory: the
 *     caller queries feh_plan_workspace_bytes and hands a buffer to
 *     feh_plan_set_workspace, which the caller keeps alive.
 *   - Every call enqueues its device work on the plan's stream.  Calls that
 *     return host values synchronise that stream before returning.
 *   - Return value: FEH_OK (0) or a negative error code; feh_last_error()
 *     gives a message for the last failure on the calling thread.  No C++
 *     exception crosses the ABI.  A plan is not thread safe.
 */
#ifndef FEH_H
#define FEH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FEH_OK = 0,
    FEH_EINVAL = -1,      /* invalid argument (null pointer, shape, value)     */
    FEH_ENOMEM = -2,      /* workspace missing or too small                    */
    FEH_EHIP = -3,        /* HIP runtime error                                 */
    FEH_ENOCONV = -4,     /* max_iter reached; outputs hold the last iterate   */
    FEH_EBREAKDOWN = -5,  /* CG breakdown (p.q <= 0 or not finite)             */
    FEH_ENOTSUP = -6      /* unsupported (axis too long for the LDS transform,
                             derivative kind outside its dimension)           */
};

enum { FEH_FP64 = 0, FEH_FP32 = 1 };

typedef struct feh_plan feh_plan;
typedef struct feh_batch feh_batch;

typedef struct {
    int32_t iterations;   /* CG iterations performed for this load case           */
    int32_t status;       /* FEH_OK, FEH_ENOCONV or FEH_EBREAKDOWN                */
    double rel_residual;  /* sqrt(r.z / f.M^+f): relative residual in the strain
                             space norm (Euclidean over all elements)            */
    double seconds;       /* host wall time of the whole call that filled the
                             report (set-up, CG, post-processing; the same for
                             every load case of the call)                        */
} feh_report;

/* Create a plan for a dim-dimensional periodic grid n[] with voxel sizes h[]
 * (NULL = unit), n_load load cases solved together, precision FEH_FP64 or
 * FEH_FP32, and a HIP stream (hipStream_t; NULL = default stream).
 * Each n[a] must lie in [2, 4096]; any size is accepted: prime factors up
 * to 13 run as radix butterflies, larger primes (e.g. 17, 151) as direct-DFT
 * passes (O(p) work per output of that pass).  An axis whose points times
 * the components of a transform exceed the LDS tile (4096 points in FP64,
 * 6144 in FP32) gives FEH_ENOTSUP; n_load in [1, 64]; N <= 2^31.  The CG
 * applies K, f and (B^*B)^-1 with the element volume divided by the voxel
 * volume (1/6 in 3D, 1/2 in 2D; one common factor, which leaves every iterate
 * unchanged), and FP32 plans form (B^*B)^-1 from dimensionless phase factors,
 * so no power of the voxel size enters the FP32 arithmetic; FP32 solves are
 * tested at voxel sizes 1e-12 .. 1e12 (the fluctuations, of order
 * |Ebar| n h, must stay inside the FP32 range).  Host-side only: computes the
 * FFT factorisations, twiddle and phase tables (Discrete Fourier transform
 * appendix: k_a = 2 pi m / (n_a h_a)). */
int feh_plan_create(feh_plan **plan, int dim, const int64_t n[], const double h[],
                    int n_load, int precision, void *hip_stream);

/* Batched plan: n_batch microstructures of the same grid, each with its own
 * material and n_load load cases; the plan then carries n_batch * n_load
 * load cases (<= 64), numbered l = b * n_load + j for microstructure b.
 * Every per-load-case array of the entry points below keeps its layout with
 * this numbering; material arrays become [n_batch][N]; load cases of
 * different microstructures never interact (their energy-matrix entries are
 * zero).  Each load case stops on its own, so a batch of easy and hard
 * microstructures costs the hard ones' iterations only for them.
 * feh_plan_create is the case n_batch = 1. */
int feh_plan_create_batch(feh_plan **plan, int dim, const int64_t n[], const double h[],
                          int n_batch, int n_load, int precision, void *hip_stream);

/* Destroy a plan (NULL is a no-op).  Does not free the workspace. */
int feh_plan_destroy(feh_plan *plan);

/* Bytes of device workspace the plan needs (nodal vectors u, r, p, q for
 * every load case, r sized to hold a half spectrum, the half spectrum, the
 * material, tables, partial sums and CG scalars). */
int feh_plan_workspace_bytes(const feh_plan *plan, size_t *bytes);

/* Hand the plan a device buffer of at least feh_plan_workspace_bytes bytes,
 * 256-byte aligned.  Uploads the tables (asynchronously on the stream).
 * The material must be set again after a new workspace. */
int feh_plan_set_workspace(feh_plan *plan, void *dev_ptr, size_t bytes);

/* Material from per-voxel Lame constants (device arrays of N values, or
 * [n_batch][N] for a batched plan, in the plan precision; caller-owned, read
 * once and copied into the workspace).  The isotropic law
 * sigma = lambda tr(e) I + 2 mu e per element is the constitutive map of the
 * paper's small-strain examples (Sec. "Eshelby inhomogeneity": isotropic
 * linear elasticity given by Young's modulus and Poisson's ratio; small-strain
 * appendix for the strain measure).  lambda and mu must be finite with
 * mu >= 0 and lambda + 2 mu / dim >= 0 (checked on the device; FEH_EINVAL
 * otherwise, and the plan keeps no material).  Blocking. */
int feh_set_material_lame(feh_plan *plan, const void *lambda_dev, const void *mu_dev);

/* Material from a phase map (device int32[N] or [n_batch][N], values in
 * [0, n_phase), caller-owned) and a host table E_nu[n_phase][2] = (E, nu)
 * with E >= 0 (E = 0 is vacuum, as in the paper's two-pillar example) and
 * -1 < nu < 0.5, n_phase in [1, 4096].  The paper fixes isotropic linear
 * elasticity by (E, nu) (Sec. "Eshelby inhomogeneity") but does not say which
 * 2D reduction; this library reads it as plane strain:
 * lambda = E nu/((1+nu)(1-2nu)), mu = E/(2(1+nu)) in 2D and 3D.  A phase id
 * outside the table gives FEH_EINVAL (checked on the device).  Blocking. */
int feh_set_material_phases(feh_plan *plan, const int32_t *phase_dev,
                            const double *E_nu_host, int n_phase);

/* Material from a per-voxel Young's modulus field (device, N or [n_batch][N]
 * values in the plan precision, E >= 0 and finite, caller-owned) and a
 * uniform Poisson ratio (-1 < nu < 0.5); the Lame constants follow with the
 * plane-strain reading of feh_set_material_phases.  The plan remembers nu for
 * feh_energy_sensitivity_E.  FEH_EINVAL for a negative or non-finite E
 * (checked on the device).  Blocking. */
int feh_set_material_field(feh_plan *plan, const void *E_dev, double nu);

/* Solve all load cases: find the periodic fluctuation u with zero mean such
 * that the element strains e = Ebar_l + B u satisfy the discrete equilibrium
 * B^T C e = 0 (equivalently G(C e) = 0 with compatible e - Ebar).  This is the
 * weak form of Sec. "Compatibility projection" (test strains projected onto
 * compatible fields, the mean strain Ebar as the macroscopic boundary
 * condition at k = 0), discretised by the linear elements of Sec. "Linear
 * finite elements", with the projection of the small-strain appendix applied
 * in factored form by projected CG (every iterate stays compatible).  Inputs
 * are read, outputs written in caller-owned memory; blocking (host outputs
 * valid on return).  FEH_EINVAL for a non-finite or non-symmetric Ebar, a
 * negative or non-finite tol, max_iter < 1, or no material; FEH_ENOMEM
 * without a workspace.
 *   Ebar_host         [n_load][D][D] symmetric macroscopic strains (host)
 *   tol               stop a load case when sqrt(r.z / f.M^+f) <= tol
 *   max_iter          per load case, >= 1
 *   u0_dev            nullable warm start [n_load][N][D]
 *   u_dev             nullable output fluctuation [n_load][N][D]
 *   strain_dev        nullable output [n_load][N][n_e][D][D]  (Ebar + B u)
 *   stress_dev        nullable output [n_load][N][n_e][D][D]  (C e)
 *   stress_mean_host  nullable [n_load][D][D]  volume average of the stress
 *   energy_host       nullable [n_load][n_load] W_lm = < e_l : C : e_m >
 *   report_host       nullable [n_load]
 * Returns FEH_OK if every load case converged, FEH_ENOCONV or
 * FEH_EBREAKDOWN otherwise (outputs still filled from the last iterate). */
int feh_solve(feh_plan *plan, const double *Ebar_host, double tol, int max_iter,
              const void *u0_dev, void *u_dev, void *strain_dev, void *stress_dev,
              double *stress_mean_host, double *energy_host, feh_report *report_host);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): feh_solve
 * with the workspace taken from a static device array of the library (256 MiB
 * per GPU, held until the process ends) instead of the plan's workspace, and
 * the material passed in as per-voxel Lame constants (lambda_dev, mu_dev as
 * in feh_set_material_lame).  No device memory is allocated or freed; the
 * caller passes inputs and outputs exactly as for feh_solve (same layouts,
 * statuses and report).  The plan needs no workspace of its own; if it has
 * one, its workspace, material and last solution are left untouched (so
 * feh_energy_sensitivity does not see this solve).  FEH_ENOMEM if the plan's
 * workspace (feh_plan_workspace_bytes) exceeds 256 MiB, e.g. beyond about
 * 64^3 voxels x 6 load cases in FP64; FEH_EINVAL with profiling enabled.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (the solve initialises everything it reads): calls that
 * overlap on one GPU, from any plan or thread, race.  Blocking. */
int feh_solve_noalloc(feh_plan *plan, const void *lambda_dev, const void *mu_dev, const double *Ebar_host,
                      double tol, int max_iter, const void *u0_dev, void *u_dev, void *strain_dev, void *stress_dev,
                      double *stress_mean_host, double *energy_host, feh_report *report_host);

/* FFT autotuner: times, on the plan's workspace and stream (blocking), the
 * candidate radix orders of each axis (the orders of the default
 * factorisation and of the radix-4 one) and then fewer rows / pencils per
 * workgroup (1/2, 1/4 of the default) for the last, middle and first axis
 * passes and the two workgroup layouts of the first-axis pass (every load
 * case in one workgroup with the per-wavevector inverses kept in registers,
 * or one workgroup per load case forming them again) and, in 3D, the two
 * stencil tile heights (8 or 16 rows of 32 voxels), each over `reps` runs
 * (< 1: 3), and keeps the fastest.  The
 * transforms stay exact to rounding whatever is chosen; repeated solves on
 * one plan stay bitwise reproducible, two tunings may differ in rounding.
 * Overwrites the workspace vectors (set the material again only if the
 * workspace was also replaced; the material is not touched). */
int feh_plan_autotune(feh_plan *plan, int reps);

/* The plan's FFT schedule: values = [rows per workgroup (last axis),
 * pencils per workgroup (axis 1), pencils per workgroup (axis 0) (0 =
 * default heuristic), axis-0 workgroup layout (1: one workgroup per load
 * case, the default for a power-of-two axis 0; 0: every load case in one
 * workgroup, the default otherwise), stencil tile rows (3D: 8 or
 * 16 rows of 32 voxels; 2D: 1)], then for each axis 0..2 the
 * number of passes followed by the radices in pass order, then 1 if passes
 * whose shape has a compile-time transform may use it (power-of-two axes of
 * 64 to 512 points in the default radix order, the last axis in FP32 from
 * 128 points; the same butterflies and
 * twiddles, with the index arithmetic resolved at compile time) or 0 for
 * the run-time passes throughout (default 1).  Writes at most n_values
 * entries and returns the full length. */
int feh_plan_tuning(const feh_plan *plan, int *values, int n_values);

/* Set the FFT schedule and stencil tile explicitly (e.g. one saved from
 * feh_plan_tuning): the same layout, workgroup sizes >= 0 (0 = default; a
 * value above the default is clamped to it; axis-0 pencils at least a
 * quarter of the default, which sizes the partial sums), axis-0 layout 0 or 1,
 * stencil rows 8 or 16 in 3D (1 in 2D), and per axis radices from
 * {2, 3, 4, 5, 7, 8, 11, 13} or primes above 13 whose product is the
 * transformed length (n_a, n_last/2 for an even last axis), and optionally
 * the trailing compile-time transform flag (0 or 1; kept if absent).
 * FEH_EINVAL leaves the plan unchanged.  Any valid schedule is exact to
 * rounding. */
int feh_plan_set_tuning(feh_plan *plan, const int *values, int n_values);

/* Whether the plan's CG, with its current schedule, keeps the residual as its
 * last-axis half spectrum (1) or as a real field (0); negative on a null
 * plan.  FP32 plans whose last-axis passes take the compile-time transform
 * keep it as a half spectrum: the forward last-axis pass then transforms q
 * and updates the spectral residual in place (the transform is linear), and
 * the next forward pass (middle axis in 3D, first axis in 2D) reads it into
 * the spectrum, which saves about one nodal vector of HBM traffic per
 * iteration.  Both forms give
 * the same iterates up to rounding.  A host-side query for byte accounting. */
int feh_plan_cg_residual_spectral(const feh_plan *plan);

/* Uneven batches: plans of different grids (each possibly a batched plan),
 * each on a created HIP stream (plans may share one), solved together.
 * Plans on different streams run concurrently: each plan's kernels go to
 * its own stream, eagerly or as graphs.  After each plan's set-up, the CG
 * iterations of all plans run in chunks of 4, then 8 iterations per plan; with use_graph != 0 each chunk is one hipGraphLaunch per stream, of
 * a graph of that stream's plans captured once per (chunk, tol, max_iter)
 * and replayed, so a batch of many small grids costs one launch per stream
 * and chunk instead of one per kernel.  Every load case stops on its own (converged load cases return
 * at once from every kernel).  The host reads the stop flags one chunk
 * behind (it queues the next chunk before it looks at the flags after the
 * previous one), so the streams do not idle during the check, and after the
 * last load case stops one more chunk of immediately returning launches
 * runs.  feh_batch_create allocates pinned host memory for the flags and
 * one event per stream.  The batch keeps pointers to the plans (the
 * caller keeps them, their workspaces and materials alive and unchanged
 * while the batch exists; otherwise destroy and re-create the batch).
 * FEH_EINVAL for null or repeated plans or plans on the null stream. */
int feh_batch_create(feh_batch **batch, feh_plan *const *plans, int n_plans);
int feh_batch_destroy(feh_batch *batch);

/* Solve every plan of the batch (no warm start, no field outputs; the
 * fluctuations stay in each plan's workspace for feh_energy_sensitivity).
 *   Ebar_host         [n_plans] pointers, each [n_load of that plan][D][D]
 *   stress_mean_host, energy_host, report_host   nullable tables of
 *                     [n_plans] nullable pointers, per-plan layouts as in
 *                     feh_solve
 * Returns FEH_OK, or the worst per-plan status (FEH_EBREAKDOWN over
 * FEH_ENOCONV); outputs are filled either way. */
int feh_batch_solve(feh_batch *batch, const double *const *Ebar_host, double tol, int max_iter, int use_graph,
                    double *const *stress_mean_host, double *const *energy_host,
                    feh_report *const *report_host);

/* Chunks launched by the last feh_batch_solve (graph launches when
 * use_graph != 0); -1 for a null batch. */
int feh_batch_graph_launches(const feh_batch *batch);

/* Host helper: effective Voigt stiffness C[nv][nv] (engineering shear,
 * order 2D (xx,yy,xy), 3D (xx,yy,zz,yz,xz,xy)) from an energy matrix W of
 * n_load = nv load cases whose Voigt strains are linearly independent:
 * W = E^T C E with E the engineering Voigt strain columns of Ebar. */
int feh_effective_stiffness(int dim, int n_load, const double *Ebar_host,
                            const double *energy_host, double *C_host);

/* Host helper: the weights dJ/dW_lm = (E^-1 G E^-T)_lm of an objective
 * J = sum_IJ G[I][J] C_eff[I][J] (C_eff from feh_effective_stiffness with the
 * same n_load = nv load cases), for feh_energy_sensitivity.
 *   G_host [nv][nv], weight_host [nv][nv] output.  FEH_EINVAL as above. */
int feh_effective_stiffness_weights(int dim, int n_load, const double *Ebar_host, const double *G_host,
                                    double *weight_host);

/* Sensitivities of the energy matrix to the per-voxel Lame constants, for an
 * objective J = sum_lm weight[l][m] W_lm with W_lm = < e_l : C : e_m > (the
 * energy form of the effective stiffness, Sec. "Compatibility projection":
 * the weak form makes each W_ll an energy minimum over compatible
 * fluctuations, so only the explicit dependence on C counts, and the
 * off-diagonal entries follow by polarisation; the adjoint field of W_lm is
 * the forward fluctuation of load case m, no second solve):
 *   grad_lam[v] = sum_lm weight[l][m] < tr e_l tr e_m >_v
 *   grad_mu[v]  = sum_lm weight[l][m] < 2 e_l : e_m >_v
 * where < . >_v sums the elements of voxel v with the weights of the cell
 * average.  For J = sum_IJ G_IJ C_eff_IJ pass weight = E^-1 G E^-T (E the
 * engineering Voigt strain columns of the load cases).
 *   weight_host   [n_load][n_load] host, FP64, finite (not necessarily symmetric)
 *   grad_lam_dev, grad_mu_dev  outputs [N] ([n_batch][N] for a batched plan)
 *                 in the plan precision (caller-owned); weights between load
 *                 cases of different microstructures must be zero
 * Uses the fluctuations left in the workspace by the last feh_solve on this
 * plan (FEH_OK or FEH_ENOCONV); FEH_EINVAL if there is none (no solve yet, a
 * breakdown, or the material or workspace changed since).  Blocking. */
int feh_energy_sensitivity(feh_plan *plan, const double *weight_host, void *grad_lam_dev, void *grad_mu_dev);

/* The same objective differentiated with respect to a per-voxel Young's
 * modulus field at a uniform Poisson ratio (the material of
 * feh_set_material_field; the derivative of the same weak-form energy as
 * feh_energy_sensitivity, through the plane-strain Lame maps of that setter):
 *   grad_E[v] = grad_lam[v] nu / ((1+nu)(1-2nu)) + grad_mu[v] / (2 (1+nu)),
 * written in one pass by the sensitivity kernel (the two Lame fields are not
 * formed).  weight_host as above; grad_E_dev output [N] ([n_batch][N]) in the
 * plan precision, caller-owned.  FEH_EINVAL if the plan's material was not
 * set by feh_set_material_field, and in the cases of feh_energy_sensitivity.
 * Blocking. */
int feh_energy_sensitivity_E(feh_plan *plan, const double *weight_host, void *grad_E_dev);

/* Discrete derivatives of the strain-space solver (Sec. "Discrete
 * projection": the projection is built from the Fourier symbol D(k) of a
 * discrete derivative, one symbol per evaluation point T of a voxel):
 *   FEH_DERIV_FE        linear finite elements: n_e = 2 (2D) / 6 (3D) points,
 *                       the element gradients (Sec. "Linear finite elements")
 *   FEH_DERIV_FD        forward differences, 1 point (Sec. "Finite differences")
 *   FEH_DERIV_CD        central differences, 1 point (same section)
 *   FEH_DERIV_LS        least-squares voxel gradient, 1 point, 2D only
 *                       (Sec. "Least squares")
 *   FEH_DERIV_FOURIER   Fourier derivative i k, 1 point (Eq. original-G)
 *   FEH_DERIV_FOURIER2  Fourier derivative at the two triangle centroids,
 *                       2 points, 2D only (two-point Fourier appendix)
 * Wavevectors k_a = 2 pi m / (n_a h_a) with m in [-n/2, n/2 - 1] (even n) or
 * [-(n-1)/2, (n-1)/2] (odd n). */
enum {
    FEH_DERIV_FE = 0,
    FEH_DERIV_FD = 1,
    FEH_DERIV_CD = 2,
    FEH_DERIV_LS = 3,
    FEH_DERIV_FOURIER = 4,
    FEH_DERIV_FOURIER2 = 5
};

/* Evaluation points per voxel n_e of a derivative kind in dim dimensions;
 * FEH_ENOTSUP if the kind is not defined there. */
int feh_strain_cg_points(int kind, int dim, int *n_points);

/* Device workspace bytes of feh_strain_cg_solve for this plan and kind: the
 * strain-space Krylov vectors x, r, p, q (n_load * n_e * nsym * N reals each,
 * nsym = 3 in 2D, 6 in 3D), their half spectrum, CG scalars and partial
 * sums. */
int feh_strain_cg_workspace_bytes(const feh_plan *plan, int kind, size_t *bytes);

/* Projected CG in strain space (Sec. "Compatibility projection": CG on
 * G(C : e~) = -G(C : Ebar) from e~ = 0, which keeps every iterate compatible)
 * with the projection G of the small-strain appendix built from the symbol of
 * `kind`, applied per wavevector through the FFT:
 *   G(s)_T = sym(D_T (x) M^-1 sum_L s_L . conj(D_L)),
 *   M = 1/2 (|D|^2 I + sum_L D_L D_L^H);
 * modes where the symbol vanishes (k = 0; on even grids also the central
 * difference and least-squares modes where every D_T is zero) are projected
 * out.  The Fourier kinds apply the Hermitian part of G at Nyquist indices
 * (real fields); it is not a projection there, since the Fourier-derivative
 * projection is exact on odd grids only, so on even grids CG can stall near
 * 1e-11 relative and report FEH_ENOCONV at tighter tolerances.  Inner
 * product: Frobenius, equal weights per point.
 * Uses the plan's material, grid and FFT tables (plans of one
 * microstructure: FEH_EINVAL for a batched plan) and leaves the plan's own
 * workspace vectors untouched.
 *   Ebar_host         [n_load][D][D] symmetric macroscopic strains
 *   tol               stop a load case when ||r|| / ||r_0|| <= tol
 *   max_iter          per load case, >= 1
 *   work_dev          caller-owned device buffer, 256-byte aligned, of at
 *                     least feh_strain_cg_workspace_bytes bytes
 *   strain_dev        nullable output [n_load][N][n_e][D][D] (Ebar + e~) in the
 *                     plan precision
 *   stress_mean_host  nullable [n_load][D][D], average of C : e over all points
 *   energy_host       nullable [n_load][n_load], W_lm = < e_l : C : e_m >
 *   report_host       nullable [n_load]; rel_residual = ||r|| / ||r_0||
 * Returns FEH_OK, FEH_ENOCONV or FEH_EBREAKDOWN like feh_solve (outputs
 * filled), FEH_ENOMEM for a missing or short workspace. */
int feh_strain_cg_solve(feh_plan *plan, int kind, const double *Ebar_host, double tol, int max_iter,
                        void *work_dev, size_t work_bytes, void *strain_dev, double *stress_mean_host,
                        double *energy_host, feh_report *report_host);

/* Per load case outcome of feh_finite_strain_solve. */
typedef struct {
    int32_t newton_iterations;  /* Newton steps over all load steps                 */
    int32_t cg_iterations;      /* CG iterations summed over the Newton steps        */
    int32_t status;             /* FEH_OK or FEH_ENOCONV (max_newton in a load step) */
    int32_t pad;
    double rel_equilibrium;     /* ||G P(F)|| / ||P(F)|| at the last check            */
    double rel_increment;       /* ||dF|| / ||F|| of the last Newton step             */
} feh_finite_report;

/* Device workspace bytes of feh_finite_strain_solve: five deformation-gradient
 * fields (F, dF and the CG vectors r, p, q; n_load * n_e * D^2 * N reals each),
 * their half spectrum, CG scalars and partial sums. */
int feh_finite_strain_workspace_bytes(const feh_plan *plan, int kind, size_t *bytes);

/* Finite-strain homogenization (Sec. "Compatibility projection"): find the
 * deformation gradient F = Fbar + F~ (F~ compatible, zero mean; n_e points
 * per voxel for the derivative `kind`, see FEH_DERIV_*) with G P(F) = 0,
 * where G is the gradient projection built from the kind's symbol (Eq.
 * original-G / discrete_projection_op) and P the first Piola-Kirchhoff stress
 * of the isotropic finite-strain linear elastic (Saint Venant-Kirchhoff) law
 * with the plan's per-voxel Lame constants, P = F (lambda tr(E) I + 2 mu E),
 * E = (F^T F - I) / 2; lambda = mu = 0 (vacuum) is allowed.
 * Newton: each step solves G (dP/dF : dF) = -G P(F) by CG from dF = 0 (the
 * right-hand side projected twice), F += dF.  A load case stops when
 * ||G P|| <= equil_tol ||P|| before a step or ||dF|| <= newton_tol ||F||
 * after one (Frobenius norms over the field).  Fbar moves linearly from I in
 * n_steps load steps, each starting from the previous solution plus the
 * uniform increment.  Plans of one microstructure (FEH_EINVAL otherwise).
 *   Fbar_host       [n_load][D][D], det > 0 (F_{i a} = d chi_i / d r_a)
 *   max_newton      Newton steps per load step; max_cg CG iterations per step
 *   work_dev        caller-owned, 256-byte aligned, >= the workspace bytes
 *   F_dev, P_dev    nullable outputs [n_load][N][n_e][D][D], plan precision
 *   P_mean_host     nullable [n_load][D][D], average of P over the points
 *   report_host     nullable [n_load]
 * Returns FEH_OK, or FEH_ENOCONV if a load case did not converge (outputs
 * filled from the last iterate); FEH_ENOTSUP for the Fourier derivatives on a
 * grid with an even axis (their projection is exact on odd grids only, Sec.
 * "Even vs. odd number of grid points", and Newton on it need not converge). */
int feh_finite_strain_solve(feh_plan *plan, int kind, const double *Fbar_host, int n_steps, double newton_tol,
                            double equil_tol, double cg_tol, int max_newton, int max_cg, void *work_dev,
                            size_t work_bytes, void *F_dev, void *P_dev, double *P_mean_host,
                            feh_finite_report *report_host);

/* Test export: q = K p with K = sum_e |e| B_e^T C_e B_e, the stiffness of the
 * linear elements of Sec. "Linear finite elements" (element gradients from the
 * shape functions of its element stencils, one constant strain per element,
 * the plan's isotropic material), p and q [n_load][N][D] in the plan
 * precision, caller-owned.  Overwrites the plan's CG vectors p and q (a
 * following feh_energy_sensitivity still sees the last solve).  FEH_EINVAL
 * without material or for null pointers.  Blocking. */
int feh_apply_operator(feh_plan *plan, const void *p_dev, void *q_dev);

/* Test export: z = M^+ r with M = sum_e |e| B_e^T B_e (K for lambda = 0,
 * mu = 1/2), applied per wavevector as (B^*B)(k)^-1 with z(k = 0) = 0 (Sec.
 * "Discrete projection": the operator is block diagonal in Fourier space and
 * k = 0 carries the mean); z has zero mean.  r, z [n_load][N][D] in the plan
 * precision, caller-owned.  Blocking. */
int feh_apply_preconditioner(feh_plan *plan, const void *r_dev, void *z_dev);

/* Test export: the small-strain projection of the paper's small-strain
 * appendix, G = B (B^*B)^+ B^* (the operator G_ThetaLambda,ijlm there, written
 * for the linear-element derivative), on element fields
 * e [n_load][N][n_e][D][D] in the plan precision (only the symmetric part of e
 * enters; G e is symmetric and compatible), caller-owned.  Blocking. */
int feh_apply_projection(feh_plan *plan, const void *e_dev, void *Ge_dev);

/* Test export: unnormalised forward real-to-half-complex DFT over the grid
 * (sum_r f(r) exp(-i k.r)) of n_load*D real fields [n_load*D][N]; output
 * [n_load*D][n0]..[n_last/2+1] interleaved complex (numpy.fft.rfftn layout). */
int feh_fft_forward(feh_plan *plan, const void *x_dev, void *X_dev);

/* Test export: inverse of feh_fft_forward including the 1/N factor. */
int feh_fft_inverse(feh_plan *plan, const void *X_dev, void *x_dev);

/* Measurement: enable (1) or disable (0) HIP-event timing of every kernel
 * launch inside the CG iterations of feh_solve on the plan's stream, and
 * reset the counters.  Kinds: 0 stencil (q = K p, p.q), 1 alpha, 2 last-axis
 * r2c with r -= alpha q (or, see feh_plan_cg_residual_spectral, the r2c of q
 * with the spectral residual update), 3 middle-axis forward (3D), 4 first
 * axis forward + (B^*B)^-1 + inverse with r.z, 5 middle-axis inverse (3D),
 * 6 last-axis c2r, 7 beta / stop test. */
int feh_profile_enable(feh_plan *plan, int enable);

/* Accumulated milliseconds and launch counts per kind (n_kinds entries,
 * kinds beyond 7 read as zero). */
int feh_profile_read(const feh_plan *plan, double *ms_total, int64_t *launches, int n_kinds);

/* Measurement: copy `bytes` (a multiple of 16; 16-byte aligned, non-overlapping
 * device buffers) from src_dev to dst_dev on the given HIP stream with
 * nontemporal 16-byte loads and stores, asynchronously.  It gives the
 * read+write bandwidth the device attains for a plain streaming copy, the
 * practical ceiling the HBM-bound kernels are compared with.  FEH_EINVAL for
 * null, misaligned or overlapping arguments. */
int feh_stream_copy(void *dst_dev, const void *src_dev, size_t bytes, void *hip_stream);

/* Message of the last error on this thread ("" if none). */
const char *feh_last_error(void);

/* Library version, 10000*major + 100*minor + patch. */
int feh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FEH_H */
