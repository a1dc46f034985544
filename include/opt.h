/*
 * opt.h - C ABI of a matrix-free Gauss-Newton / Levenberg-Marquardt least-squares
 * solver for MI355X (gfx950), after Opt (DeVito et al., arXiv 1604.06525).
 *
 * The solver minimises E(x) = sum_r f_r(x)^2 (Sec. 4) for a fixed set of energies
 * written by hand (the energies defined in Appendix C), on a 2D pixel grid or on
 * a graph.  Every outer iteration linearises F at x and solves the normal
 * equations J^T J d = -J^T F (Sec. 4; the factor 2 on both sides cancels) with a
 * Jacobi-preconditioned conjugate gradient started from d = 0 (Sec. 4.1), whose
 * products J^T F, J^T J p and diag(J^T J) are evaluated on the fly from the
 * unknowns and the energy's data (matrix-free, Secs. 4.1-4.2).  Levenberg-
 * Marquardt adds lambda * diag(J^T J) to the system (Sec. 4).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every function returns 0 on success or a negative OPT_E* code; the message
 *   of the last failure on the calling thread is returned by opt_last_error().
 *   A failed call leaves the problem as it was, except OPT_EHIP from an enqueued
 *   kernel, after which the problem's device state is undefined.
 * - Device pointers are plain HIP device addresses on the device that is current
 *   when the problem is created.  Host pointers are ordinary host memory.
 * - A field of c channels over n sites is stored as c planes of n values
 *   ("SoA"): element (ch, site) at offset ch*n + site.  On a grid of width W and
 *   height H, site (i, j) is j*W + i, with i along the width (the first grid
 *   dimension in the paper's listings).
 * - Bulk values (unknowns, data arrays, internal vectors) are float64 under
 *   OPT_FP64 and float32 under OPT_MIXED.  Dot products, costs, the PCG scalars
 *   and the LM step test are accumulated in float64 under both (Sec. 7, "Numerical
 *   Precision", offers float and double; the mixed form keeps the reductions in
 *   double).  Masks are uint8.
 * - All work is enqueued on the HIP stream given at creation, in order.  Calls
 *   that return host values synchronise that stream once before returning.
 * - The library allocates no device memory: all of its device state lives in a
 *   caller-owned workspace of opt_workspace_size() bytes.  Data arrays are
 *   referenced, not copied: they must stay valid and unchanged while work that
 *   reads them is in flight, and the caller may edit them between calls (the
 *   multi-pass use of Sec. 7).
 * - A problem handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef OPT_H
#define OPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define OPT_OK 0
#define OPT_EINVAL (-1)       /* invalid argument, size or descriptor field */
#define OPT_ENOMEM (-2)       /* workspace smaller than opt_workspace_size() */
#define OPT_EHIP (-3)         /* a HIP runtime call failed; message names it */
#define OPT_EAGAIN (-4)       /* server: no free slot or arena range; retry later */
#define OPT_ENUMERIC (-5)     /* a cost came out NaN or infinite */
#define OPT_EUNSUPPORTED (-6) /* combination of domain/energy/precision not built */

typedef enum { OPT_GRID2D = 0, OPT_GRAPH = 1, OPT_GRID3D = 2 } opt_domain;

/*
 * Energies.  For each: unknown channels; arrays[] in order; params[] in order.
 *
 * OPT_E_LAPLACIAN (grid or graph; Figs. 3 and 5, the introductory example).  On
 *   a grid: 1 unknown per pixel; residuals w_fit (X - A) and w_reg (X(i,j) -
 *   X(i+1,j)), w_reg (X(i,j) - X(i,j+1)) where the neighbour is on the grid.  On
 *   a graph: 3 unknowns per vertex (a float3); residuals w_fit (X_v - A_v) and
 *   w_reg (X_v0 - X_v1) once per listed edge.  arrays: [0] A (1 plane on a grid,
 *   3 on a graph).  params: w_fit, w_reg.  Linear: one GN step with an exact
 *   inner solve reaches the minimiser (w_fit^2 I + w_reg^2 L) x = w_fit^2 A.
 *   opt_energy_channels reports its grid form (1).
 * OPT_E_ARAP_WARP (grid; Fig. 24, Appendix A.1.1).  Unknowns 3: offset x, offset y,
 *   angle.  arrays: [0] U rest positions (2 planes), [1] C targets (2 planes; a
 *   target is used when both components are >= 0), [2] mask (uint8; pixels with
 *   mask != 0 are excluded from the solve but keep their terms).  params:
 *   w_fit, w_reg (square roots of the energy weights).
 * OPT_E_POISSON (grid; Fig. 27, A.1.4).  Unknowns 4 (RGBA).  arrays: [0] T
 *   (4 planes), [1] mask (uint8; mask != 0 excluded).  params: none.
 * OPT_E_SFS (grid; Fig. 26, A.1.3).  Unknowns 1 (depth).  arrays: [0] D_i input
 *   depth (D_i <= 0 is excluded), [1] Im intensity, [2] edgeMaskR (uint8),
 *   [3] edgeMaskC (uint8).  params: w_p, w_s, w_g (energy weights; their square
 *   roots are applied), f_x, f_y, u_x, u_y, L1..L9.
 * OPT_E_FLOW (grid; Fig. 30, A.2.3).  Unknowns 2 (u, v).  arrays: [0] I,
 *   [1] I_hat, [2] dI_hat/dx, [3] dI_hat/dy.  params: w_fit, w_reg.
 * OPT_E_ARAP_MESH (graph; Fig. 25, A.1.2).  Unknowns 6: offset xyz, Euler angles
 *   xyz with R = Rz Ry Rx.  arrays: [0] U rest positions (3 planes), [1] C targets
 *   (3 planes; a component is used when >= -999999.9).  Each listed undirected
 *   edge {v0, v1} contributes the ARAP residual in both orientations.  params:
 *   w_fit, w_reg.
 * OPT_E_ARAP_VOLUME (3D grid, OPT_GRID3D; Fig. 31, A.2.5).  Unknowns 6 per
 *   voxel as for the mesh; voxel (i, j, k) is (k*height + j)*width + i.  The
 *   voxel lattice is the connectivity: every voxel has the ARAP residual towards
 *   each in-bounds neighbour along +-x, +-y, +-z (so each lattice edge counts in
 *   both orientations).  arrays and params as for OPT_E_ARAP_MESH.
 * OPT_E_LP_SMOOTH (grid; Sec. 7, the IRLS variant of Gauss-Newton).  1 unknown
 *   per pixel.  Data term w_fit (X - A), squared; edge terms f = w_reg (X(i,j) -
 *   X(i+1,j)), w_reg (X(i,j) - X(i,j+1)) where the neighbour is on the grid,
 *   entering as (f^2 + eps^2)^(p/2).  The reported cost is that objective.  Each
 *   outer iteration freezes w = (p/2) (f^2 + eps^2)^((p-2)/2) per edge at the
 *   current unknowns and takes a Gauss-Newton step on the reweighted least
 *   squares sum (w_fit (X - A))^2 + sum w f^2 (iteratively reweighted least
 *   squares).  arrays: [0] A.  params: w_fit, w_reg, p in (0, 2], eps > 0
 *   (OPT_EINVAL otherwise).  OPT_LM is refused (OPT_EUNSUPPORTED).
 * OPT_E_INTRINSIC (grid; A.2.4, Fig. 33, solved by IRLS as Sec. 7 describes).
 *   4 unknowns per pixel: reflectance r (3 channels) and shading s, in the
 *   channel order r0, r1, r2, s.  Residuals at a pixel: the fits w_fit (r_c + s -
 *   I_c), and for each of the four stencil neighbours q on the grid the
 *   reflectance term f = w_a (r - r_q), entering as (|f|^2 + eps^2)^(p/2), and
 *   the shading term w_s (s - s_q) (each edge thus counts at both ends).  The
 *   reported cost is that objective.  Each outer iteration freezes w = (p/2)
 *   (|f|^2 + eps^2)^((p-2)/2) per edge and takes a Gauss-Newton step on the
 *   reweighted least-squares problem.  A uniform shift of r down and s up leaves
 *   everything unchanged (the PCG keeps to the normal equations' range).
 *   arrays: [0] I (3 planes, image in the log domain).  params: w_fit, w_a,
 *   w_s, p in (0, 2], eps > 0 (OPT_EINVAL otherwise).  OPT_LM is refused
 *   (OPT_EUNSUPPORTED).
 */
typedef enum {
  OPT_E_LAPLACIAN = 0,
  OPT_E_ARAP_WARP = 1,
  OPT_E_POISSON = 2,
  OPT_E_SFS = 3,
  OPT_E_FLOW = 4,
  OPT_E_ARAP_MESH = 5,
  OPT_E_ARAP_VOLUME = 6,
  OPT_E_LP_SMOOTH = 7,
  OPT_E_INTRINSIC = 8
} opt_energy;

typedef enum { OPT_FP64 = 0, OPT_MIXED = 1 } opt_precision;
typedef enum { OPT_GN = 0, OPT_LM = 1 } opt_method;

/*
 * Form of the preconditioned CG inner solve (Sec. 4.1).  Both give the same
 * iterates in exact arithmetic and differ only by rounding.
 * OPT_PCG_FUSED: one kernel per iteration, the single-reduction recurrence of
 *   Chronopoulos and Gear (alpha and beta from r.z and (A z).z of the previous
 *   iteration), with A p evaluated exactly; r, p and d each cross HBM once.
 *   Available for the grid energies (ARAP warp, Poisson, flow, the Laplacian;
 *   shape from shading with its own residual-streaming kernel) and, on a
 *   graph, for the ARAP mesh and the Laplacian: there a block stages a chunk
 *   of 256 vertices with its one- and two-ring neighbourhoods, whose lists are
 *   built with the incidence list; a graph whose chunks pass the lists' caps
 *   (one-ring 256, two-ring 320 vertices, 2048 incidence entries of the chunk
 *   and of its one-ring), and every other graph energy, runs the split form
 *   (opt_problem_pcg_form tells which).
 * OPT_PCG_SPLIT: the textbook recurrence (alpha = r.z / p.Ap, then beta), two
 *   kernels per iteration.
 * OPT_PCG_MATERIALIZED: the materialised alternative of Sec. 7 (evalJ): J is
 *   evaluated into the workspace once per outer iteration and each PCG
 *   iteration multiplies by it twice (y = J p, then q = J^T y, J^T read through
 *   per-unknown lists of J's entries), with the textbook recurrence.  Needs a
 *   problem created with desc.materialize = 1 (OPT_EINVAL otherwise); built for
 *   ARAP warping and shape from shading on a grid (for the latter, the fully
 *   materialised strategy of Sec. 8.3: J's rows come from the stored lighting
 *   partials).  For comparing matrix-free and materialised products; a server
 *   runs such requests in the split form.
 * OPT_PCG_RECOMPUTE: the split form with the per-site state an energy stores at
 *   each linearisation recomputed inside every product instead of read: for
 *   shape from shading the lighting term's partials at each pixel the product
 *   reads, from the linearisation point (the fully matrix-free strategy of
 *   Sec. 8.3, Fig. 17; the stored values are reproduced, so the iterates are
 *   the split form's).  Built for shape from shading (OPT_EUNSUPPORTED
 *   otherwise); a server runs such requests in the split form.
 */
typedef enum {
  OPT_PCG_FUSED = 0,
  OPT_PCG_SPLIT = 1,
  OPT_PCG_MATERIALIZED = 2,
  OPT_PCG_RECOMPUTE = 3
} opt_pcg_variant;

typedef struct {
  int32_t domain;     /* opt_domain */
  int32_t energy;     /* opt_energy */
  int32_t precision;  /* opt_precision */
  int32_t width, height;           /* grid size (OPT_GRID2D, OPT_GRID3D), each >= 1 */
  int32_t n_vertices, n_edges;     /* graph size (OPT_GRAPH), V >= 1, E >= 0 */
  const int32_t* edges;            /* device, [E][2] vertex ids (v0, v1); read by
                                      opt_problem_create only */
  const void* arrays[8];           /* device, energy-specific (see opt_energy) */
  double params[16];               /* energy-specific (see opt_energy) */
  int32_t n_params;                /* number of params[] entries supplied */
  int32_t depth;                   /* OPT_GRID3D: third grid size (>= 1); else unused */
  int32_t materialize;             /* 1: the workspace also holds the materialised
                                      Jacobian (OPT_PCG_MATERIALIZED; OPT_EUNSUPPORTED
                                      for an energy without it); 0: not */
} opt_problem_desc;

typedef struct opt_problem opt_problem;

/* Text of the last error on the calling thread ("" if none).  Never NULL. */
const char* opt_last_error(void);

/* Bytes of device workspace the problem needs.  Pure host computation. */
int opt_workspace_size(const opt_problem_desc* desc, size_t* bytes);

/*
 * Create a problem (Fig. 4's define + plan steps; with hand-written energies both
 * collapse into one call).  `workspace` is caller-owned device memory of at least
 * opt_workspace_size() bytes, 256-byte aligned, that must outlive the handle.
 * `hip_stream` is a hipStream_t (NULL = the null stream).  For a graph the edge
 * list is sorted into a per-vertex incidence list inside the workspace, and for
 * an energy whose product stages vertices in LDS (ARAP mesh) each chunk of 256
 * consecutive vertex ids gets a list of its outside neighbours there too; the
 * host builds both in O(V + E) and copies them (this synchronises the stream
 * once).  Results do not depend on the vertex numbering beyond summation order,
 * but neighbours with nearby ids (a spatial ordering) make the products faster.
 * On failure *out is set to NULL.
 */
int opt_problem_create(const opt_problem_desc* desc, void* workspace, size_t workspace_bytes,
                       void* hip_stream, opt_problem** out);

/* Release the handle (not the workspace or arrays).  NULL is accepted. */
int opt_problem_destroy(opt_problem* prob);

typedef struct {
  int32_t method;       /* opt_method */
  int32_t outer_iters;  /* nonlinear iterations K >= 0 (LM: rejected steps count) */
  int32_t pcg_iters;    /* linear iterations L >= 0 per outer iteration */
  int32_t use_precond;  /* 1: Jacobi M = diag(J^T J) (Sec. 4.1); 0: plain CG */
  double lm_radius0;    /* initial trust-region radius; lambda = 1/radius (Sec. 4) */
  double lm_radius_min; /* LM stops once the radius falls below this */
  double lm_radius_max; /* cap on the radius */
  double lm_diag_min, lm_diag_max; /* clamp of the damping diagonal D */
  double lm_min_rel_decrease;      /* step accepted iff model decrease m > 0 and
                                      (E(x) - E(x+d)) / m exceeds this */
  int32_t pcg_variant;  /* opt_pcg_variant */
} opt_solve_params;

typedef struct {
  double cost_initial;   /* E(x) before the first iteration */
  double cost_final;     /* E(x) after the last */
  int32_t outer_done;    /* iterations executed (LM may stop early) */
  int32_t steps_accepted;/* GN: outer_done; LM: accepted steps */
  double* cost_trace;    /* optional host array of outer_iters+1 entries: E at the
                            start of each iteration, then the final E; NULL = skip */
} opt_solve_report;

/* Fill `p` with the defaults: GN, 10 x 50, preconditioned, LM radius 1e4 in
   [1e-32, 1e16], diagonal clamp [1e-6, 1e32], min relative decrease 1e-3,
   OPT_PCG_FUSED. */
void opt_default_params(opt_solve_params* p);

/*
 * Run the solver on `unknowns` (device, channels x sites, in/out), following
 * Sec. 4: GN updates x += d after each PCG solve; LM takes or rejects the step
 * by the gain ratio and updates the radius.  Excluded unknowns never change.
 * If `report` is NULL the call only enqueues work and returns; otherwise it
 * synchronises once and fills the report.  Returns OPT_ENUMERIC (with the report
 * filled) if a cost is NaN or infinite.
 */
int opt_solve(opt_problem* prob, void* unknowns, const opt_solve_params* params,
              opt_solve_report* report);

/*
 * opt_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc): create the
 * problem of `desc` and solve it as opt_problem_create + opt_solve would, with
 * the same kernels, launch shape (the automatic one; no tuning) and results,
 * but with the problem's workspace in the library's static scratch: one
 * OPT_SCRATCH_BYTES device array per GPU, held from the library's first use on
 * that GPU until the process ends.  The call allocates no device memory.
 * `unknowns` (device, channels x sites, in/out) and `report` (may be NULL:
 * enqueue only) are as for opt_solve; `hip_stream` is a hipStream_t (NULL = the
 * null stream) on the current device.  A graph's edges are read as by
 * opt_problem_create (this synchronises the stream).
 * Errors: those of opt_problem_create and opt_solve, and OPT_ENOMEM when the
 * problem's workspace (opt_workspace_size) exceeds OPT_SCRATCH_BYTES.
 * Every call on one GPU uses that GPU's one scratch array and leaves its
 * contents behind: calls whose work may overlap on one GPU (from several host
 * threads, or on different streams while an earlier call's work is still in
 * flight) race and must be serialised by the caller.
 */
#define OPT_SCRATCH_BYTES ((size_t)128 << 20)
int opt_solve_scratch(const opt_problem_desc* desc, void* unknowns, const opt_solve_params* params,
                      opt_solve_report* report, void* hip_stream);

/* E(x) = sum_r f_r(x)^2 in float64 at `unknowns` (device); synchronises. */
int opt_cost(opt_problem* prob, const void* unknowns, double* cost);

/*
 * Step-level entry points.  They expose the stages of one outer iteration so
 * each can be checked and timed on its own; opt_solve chains the same kernels.
 *
 * opt_linearize: evaluate the residuals at `unknowns` and store the per-site
 *   state the matrix-free products need (Sec. 7's precomputed arrays: e.g. the
 *   rotation's cosine and sine, the shading term and its gradient, sampled image
 *   derivatives).  Writes E(x) to *cost if cost != NULL (then synchronises).
 *   The later step calls read `unknowns` again: it must stay valid and unchanged
 *   until the next opt_linearize or opt_solve on this problem.
 * opt_eval_jtf: at the last linearisation point, write b = -J^T F and
 *   diag(J^T J) (device, channels x sites, bulk type; either may be NULL).
 *   Excluded unknowns get 0 in both.
 * opt_apply_jtj: at the last linearisation point, q = (J^T J + lambda D) p with
 *   D = clamp(diag(J^T J), lm_diag_min, lm_diag_max) from `params` (which may be
 *   NULL when lambda == 0).  p, q: device, channels x sites; excluded entries of
 *   p are ignored and of q set to 0.  p and q must not overlap.
 * opt_pcg: at the last linearisation point, run params->pcg_iters PCG iterations
 *   (in the form params->pcg_variant) on (J^T J + lambda D) d = -J^T F from d = 0
 *   and write d (device).
 */
int opt_linearize(opt_problem* prob, const void* unknowns, double* cost);
int opt_eval_jtf(opt_problem* prob, void* b_out, void* diag_out);
int opt_apply_jtj(opt_problem* prob, const void* p, void* q, double lambda,
                  const opt_solve_params* params);
int opt_pcg(opt_problem* prob, const opt_solve_params* params, double lambda, void* delta_out);

/*
 * Timing of the PCG phase.  After opt_profile_enable(prob, 1) every opt_solve
 * records a HIP event pair on the problem's stream around the L PCG iterations of
 * each outer iteration.  opt_profile_read synchronises the stream, adds the
 * elapsed times of all pairs recorded since the last read into *pcg_ms, the
 * number of PCG iterations they cover into *pcg_iters, and clears them.
 */
int opt_profile_enable(opt_problem* prob, int enable);
int opt_profile_read(opt_problem* prob, double* pcg_ms, int64_t* pcg_iters);

/*
 * Launch tuning of a problem (no effect on results beyond the order of a few
 * additions: every choice computes the same iterates up to rounding; only the
 * work split changes).  The fused PCG kernel gives each wavefront a strip of at
 * most 60 columns (58 for shape from shading; the grid's width split evenly)
 * and some rows.
 *   strip_rows > 0: strips of that many rows.
 *   waves_per_simd > 0 (and strip_rows == 0): about that many strips per SIMD,
 *     rows split evenly.
 *   both 0 (automatic): two strips per SIMD, rows split evenly, at least 4
 *     rows.
 * Shorter strips mean more wavefronts in flight but more halo rows read twice.
 *   large_grid_form = 1: run the fused kernel's large-grid form (each strip
 *     addresses its rows from its own first row; the form a grid whose
 *     vectors pass 256 MB always runs) even on a grid that does not need it.
 *     Same iterates up to rounding; for checking and timing that form.  0: the
 *     form is chosen by size.  Ignored by shape from shading, which has no
 *     such form.
 * opt_problem_get_tuning returns the values in force (resolved: the largest
 * strip height and the strips per SIMD, rounded up).
 */
typedef struct {
  int32_t strip_rows;
  int32_t waves_per_simd;
  int32_t large_grid_form;
} opt_tuning;

int opt_problem_set_tuning(opt_problem* prob, const opt_tuning* tuning);
int opt_problem_get_tuning(opt_problem* prob, opt_tuning* tuning);

/*
 * Graph replay of repeated solves (on by default).  The kernels a solve
 * enqueues depend only on the unknowns pointer, the solve parameters and the
 * tuning (every decision of Sec. 4's loop, LM's included, is taken on the
 * device).  When opt_solve is called again with the same three as the call
 * before it, the library records that launch sequence once as a HIP graph (on a
 * private stream of its own) and from then on launches the whole solve as one
 * graph on the problem's stream while they stay the same.  Results are the same
 * bits as without it; only the host's launch cost changes (one graph launch
 * instead of one launch per kernel, which bounds small problems).  Solves with
 * profiling on (opt_profile_enable) are never replayed.  enable = 0 turns it off
 * and frees the recorded graph.  Destroying the problem frees it too.
 */
int opt_problem_set_graph_replay(opt_problem* prob, int enable);

/*
 * The PCG form a solve of this problem runs when it asks for `variant`
 * (opt_pcg_variant): *form = OPT_PCG_FUSED where the fused kernel serves it
 * (the grid energies; on a graph, the ARAP mesh and the Laplacian when every
 * chunk's lists fit their caps), else OPT_PCG_SPLIT; OPT_PCG_MATERIALIZED
 * and OPT_PCG_RECOMPUTE answer themselves (the latter OPT_EUNSUPPORTED for an
 * energy without it).  OPT_EINVAL for a NULL argument or an unknown variant.
 */
int opt_problem_pcg_form(opt_problem* prob, int variant, int* form);

/*
 * Multi-pass optimisation (Sec. 7: between solves the caller may change the
 * problem state; hierarchical, coarse-to-fine solves are the common case).  The
 * steps between passes as kernels, and the hierarchical optical flow of
 * Appendix A.2.3 built from them.  All images are row-major planes (site
 * j*W + i) of the bulk type of `precision` (float64 under OPT_FP64, float32
 * under OPT_MIXED), device memory, work enqueued on `hip_stream` (a
 * hipStream_t; NULL = the null stream) without synchronising.
 *
 * opt_image_downsample2: dst (planes x floor(W/2) x floor(H/2)) = the mean of
 *   each 2 x 2 block of src (planes x W x H); W, H >= 2; 1 <= planes <= 8.
 * opt_image_gradient: the derivative images of img (W x H) along the width
 *   (dx) and the height (dy): central differences (img(i+1) - img(i-1)) / 2
 *   inside, one-sided differences on the first and last column or row, 0 along
 *   a dimension of one pixel.  These are the derivative images the sampled-image
 *   operator of the flow energy reads (Sec. 7).
 * opt_field_upsample: dst(c; i, j) = scale[c] * S(src_c; (i + 1/2) Ws/Wd - 1/2,
 *   (j + 1/2) Hs/Hd - 1/2), S the bilinear clamp-to-edge sample with texel
 *   centres at integer coordinates: the coarse field at the point under each
 *   fine pixel's centre, scaled per plane (a flow measured in coarse pixels is
 *   scaled by the size ratio).  scale: host array of `planes` values.
 *
 * opt_solve_flow_pyramid: the hierarchical dense optical flow of A.2.3 on
 *   frames I and I_hat (W x H): level l of `levels` has floor(W/2^l) x
 *   floor(H/2^l) pixels (the coarsest at least 4 x 4); its images are the 2 x 2
 *   means of the level above (level 0 is I, I_hat themselves) and its
 *   derivative images are opt_image_gradient of its I_hat.  The coarsest level
 *   starts from zero flow; every level is solved as opt_solve would solve the
 *   OPT_E_FLOW problem of its images (params w_fit, w_reg; `params` for every
 *   level) with the automatic launch shape; each finer level starts from the
 *   solution below it, upsampled (opt_field_upsample, scaled by the size
 *   ratios).  `unknowns` (device, 2 planes u, v of W x H) receives the level-0
 *   solution; with levels == 1 it is also the starting point.  `workspace`:
 *   device, 256-byte aligned, at least opt_flow_pyramid_workspace_size bytes,
 *   caller-owned.  `reports` (host, may be NULL) holds `levels` reports,
 *   reports[l] for level l (each as opt_solve fills it; its cost_trace may be
 *   NULL); with reports the call synchronises once per level, without it it
 *   only enqueues work.  Errors: OPT_EINVAL (sizes, levels, precision,
 *   parameters), OPT_ENOMEM (workspace too small), OPT_ENUMERIC (a level's cost
 *   was not finite; later levels are not solved).
 */
int opt_image_downsample2(const void* src, int32_t width, int32_t height, int32_t planes, int32_t precision,
                          void* dst, void* hip_stream);
int opt_image_gradient(const void* img, int32_t width, int32_t height, int32_t precision, void* dx, void* dy,
                       void* hip_stream);
int opt_field_upsample(const void* src, int32_t src_width, int32_t src_height, int32_t planes,
                       const double* scale, int32_t precision, void* dst, int32_t dst_width, int32_t dst_height,
                       void* hip_stream);
int opt_flow_pyramid_workspace_size(int32_t width, int32_t height, int32_t levels, int32_t precision,
                                    size_t* bytes);
int opt_solve_flow_pyramid(const void* I, const void* I_hat, int32_t width, int32_t height, int32_t levels,
                           double w_fit, double w_reg, int32_t precision, const opt_solve_params* params,
                           void* unknowns, void* workspace, size_t workspace_bytes, void* hip_stream,
                           opt_solve_report* reports);

/* Number of unknown channels per site for an energy (0 if unknown). */
int opt_energy_channels(int32_t energy);

/*
 * Serving: many solves at once (continuous batching).
 *
 * Small problems use a GPU poorly (Sec. 8 notes the solver is inefficient below
 * a few thousand unknowns): each kernel launch carries little work.  A server
 * advances every active request by one outer iteration per opt_server_step, and
 * runs each stage of that iteration as one launch per energy kind covering all
 * of its requests; the energy kinds run on streams of their own (forked from
 * and joined back to the server's stream within the step), so they overlap.  Each request keeps the arithmetic and reduction order of
 * opt_solve with the same parameters, so its result is bit-identical to solving
 * it alone, whatever else runs beside it.  One exception: a grid problem whose
 * internal vectors pass 256 MB runs the fused PCG form alone but the split form
 * in a server (the server batches only the regular fused instantiation); its
 * served result then equals opt_solve with OPT_PCG_SPLIT bit for bit.
 *
 * Memory: the caller hands the server one device arena (256-byte aligned).  The
 * first opt_server_reserved_bytes(max_slots) bytes hold the server's argument
 * tables; each admitted request's workspace (opt_workspace_size of its
 * descriptor) is carved from the rest, first fit, and returned when it leaves.
 * The arena size is therefore the memory budget.  The server also allocates a
 * little pinned host memory for staging.
 *
 * opt_server_submit: admit a request: a problem descriptor (arrays referenced as
 *   by opt_problem_create; they and `unknowns` must stay valid until the request
 *   is collected or cancelled) and solve parameters.  Returns OPT_EAGAIN (nothing
 *   admitted) if no slot is free or no free arena range is large enough; the
 *   request may be submitted again after a step has retired others.  A graph's
 *   edge list is copied to the host behind the work already on the server's
 *   stream (the call does not wait for the steps in flight); a later step
 *   builds its incidence lists once that copy has completed, and the request
 *   starts from then on.  An edge naming a vertex outside [0, V) drops the
 *   request: poll then returns OPT_EINVAL for its ticket.  *ticket names the
 *   request.
 * opt_server_step: enqueue one quantum: admitted requests start, in admission
 *   order, while the running set's estimated GPU fill (the share of the device's
 *   wavefront slots its launches occupy, each at most 1) stays within the fill
 *   budget (default 4.0: launches of mid-sized problems are short, and several
 *   run side by side; at least one request always runs); every running
 *   request does one outer iteration (linearise, PCG init, its pcg_iters PCG
 *   iterations, LM decision, update); requests that reach their outer_iters (or
 *   whose LM radius is known to have fallen below the minimum) get their final
 *   cost and leave.  Steps are pipelined: the call returns once the work is
 *   enqueued, with up to 3 steps in flight (it waits for the oldest when 3 are);
 *   completed steps are processed whenever the server is called.  With nothing
 *   to enqueue it waits for the oldest step in flight.  A request's unknowns are
 *   written in place; they are final once poll reports it done.
 * opt_server_wait: wait until every enqueued step has completed.
 * opt_server_set_fill_budget: the fill budget (>= 0; 0 runs one request at a
 *   time, a large value runs every admitted request at once).
 * opt_server_poll: *done = 1 once the request has left; then the report (as
 *   opt_solve's; cost_trace, if not NULL, must hold outer_iters + 1 entries) is
 *   filled and the ticket is forgotten.  Returns OPT_ENUMERIC (report filled) if
 *   a cost was NaN or infinite.  *done = 0 while it runs.  OPT_EINVAL for a
 *   ticket that is unknown or already collected.
 * opt_server_cancel: drop a running request (its unknowns are left part-way;
 *   its arena range is reused once its enqueued work has completed) or an
 *   uncollected result.
 * opt_server_info: requests held (running or admitted) and free arena bytes.
 * opt_server_add_tuning: launch tuning (opt_tuning) applied at admission to
 *   2D-grid requests of that energy and precision whose site count lies in
 *   [min_sites, max_sites]; a later entry overrides an earlier one.
 *
 * A server is not thread-safe: calls on one server must not overlap.  Work the
 * caller puts on the server's stream is ordered with the steps (for example a
 * copy of initial unknowns before their submission).
 */
typedef struct opt_server opt_server;

int opt_server_reserved_bytes(int32_t max_slots, size_t* bytes);
int opt_server_create(void* arena, size_t arena_bytes, int32_t max_slots, void* hip_stream,
                      opt_server** out);
int opt_server_destroy(opt_server* server);
int opt_server_submit(opt_server* server, const opt_problem_desc* desc, void* unknowns,
                      const opt_solve_params* params, int64_t* ticket);
int opt_server_step(opt_server* server);
int opt_server_wait(opt_server* server);
int opt_server_set_fill_budget(opt_server* server, double budget);
int opt_server_poll(opt_server* server, int64_t ticket, int32_t* done, opt_solve_report* report);
int opt_server_cancel(opt_server* server, int64_t ticket);
int opt_server_info(opt_server* server, int32_t* active, size_t* arena_free);
int opt_server_add_tuning(opt_server* server, int32_t energy, int32_t precision, int64_t min_sites,
                          int64_t max_sites, const opt_tuning* tuning);

#ifdef __cplusplus
}
#endif
#endif /* OPT_H */
