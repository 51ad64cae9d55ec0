/*
 * ct.h - C ABI of the MI355X cone-beam CT operator library (libct.so).
 *
 * The library implements the computational core of iterative cone-beam CT reconstruction as
 * organised in Biguri et al., "Arbitrarily large iterative tomographic reconstruction on
 * multiple GPUs using the TIGRE toolbox": the linear model A x = b + e of Section 2, Eq. (1)
 * (A holds the intersection lengths of X-ray paths with image elements), its forward projection
 * A x (Section 2.1), backprojection A^T b (Section 2.2), the out-of-core splitting of the image
 * into axial slabs and of the projections into angle chunks (Algorithms 1 and 2), the iterative
 * algorithms that call them (CGLS and SART, Section 3.2) and the TV steepest-descent regulariser
 * (Section 2.3).
 *
 * Conventions (all entry points):
 *  - Units are millimetres and radians.  The orbit is circular about the z axis: for angle t the
 *    source sits at DSO (cos t, sin t, 0), the detector centre at -(DSD - DSO)(cos t, sin t, 0),
 *    with detector axes e_u = (-sin t, cos t, 0) and e_v = (0, 0, 1).  Pixel (a, b) has its centre
 *    at u_a = (a - (Nu-1)/2) du + offU, v_b = (b - (Nv-1)/2) dv + offV along those axes; one ray
 *    per pixel runs from the source to that centre.
 *  - Voxel (i, j, k) has its centre at offOrigin + ((i-(Nx-1)/2) dx, (j-(Ny-1)/2) dy,
 *    (k-(Nz-1)/2) dz).  The volume is stored vol[k][j][i] (x fastest); projections are stored
 *    proj[angle][b][a] (u fastest).  Arrays are dense, with no padding.
 *  - Every function returns a ct_status: CT_OK (0) or a negative error code, and never throws or
 *    aborts across the ABI.  ct_last_error() returns a message for the calling thread's last
 *    failure.  Argument and geometry validation happen before anything is written; outputs are
 *    untouched after a validation error and unspecified after CT_ERR_HIP.
 *  - Device pointers are HIP device allocations (e.g. torch tensor data_ptr()) on the current
 *    HIP device.  `stream` is a hipStream_t (NULL = the default stream).  Resident calls are
 *    stream-ordered and return after enqueueing; *_host calls are synchronous.
 *  - The caller owns every input and output array.  A plan owns only its per-angle geometry
 *    table (host and device copies); ct_plan_destroy releases it.
 *  - A plan may be used by one host thread at a time.  Distinct plans are independent.
 *  - All kernels are deterministic: identical inputs give bitwise identical outputs, whatever
 *    else runs on the device.
 */
#ifndef CT_H
#define CT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CT_OK = 0,
    CT_ERR_ARG = -1,      /* bad argument (null pointer, bad range, unknown enum) */
    CT_ERR_GEOMETRY = -2, /* geometry fails validation (see ct_plan_create) */
    CT_ERR_DTYPE = -3,    /* unsupported storage type or pairing */
    CT_ERR_OOM = -4,      /* device or pinned-host allocation failed */
    CT_ERR_CAP = -5,      /* device memory cap too small for one slice plus buffers */
    CT_ERR_HIP = -6,      /* a HIP runtime call failed */
    CT_ERR_STATE = -7     /* object in an unusable state */
} ct_status;

/* Storage type of a volume or projection array.  Arithmetic is always FP32 (accumulation along
 * every ray and over every voxel's angles); CGLS inner products and norms are FP64.
 * CT_F64 is not a storage type of the operators or algorithms (they refuse it with CT_ERR_DTYPE):
 * FP64 arrays are accepted by ct_convert, to bring FP64 data to a storage type on the device (to
 * FP32 with one rounding, to FP16/BF16 through FP32), and by ct_dot. */
typedef enum { CT_F32 = 0, CT_F16 = 1, CT_BF16 = 2, CT_F64 = 3 } ct_dtype;

/* Forward projectors (Section 2.1). */
typedef enum {
    CT_SIDDON = 0, /* exact ray/voxel intersection lengths (Siddon 1985) */
    CT_INTERP = 1  /* line integral of the trilinear interpolant, sampled every
                      accuracy * min(dVoxel) mm on a lattice anchored at the source (Chou 2011) */
} ct_projector;

/* Backprojectors (Section 2.2). */
typedef enum {
    CT_BP_FDK = 0,            /* voxel-driven, bilinear, weight (DSO / L)^2, L = voxel depth
                                 along the central ray */
    CT_BP_PSEUDO_MATCHED = 1, /* voxel-driven, bilinear, weight (dx dy dz)/(du dv) DSD^2 |SX| / L^3,
                                 the ray-tube density that approximates the transpose of Siddon */
    CT_BP_ADJOINT = 2         /* the exact transpose of CT_SIDDON */
} ct_backprojector;

/* Scanner and grid description (Section 2 / Section 3.2 scanner distances). */
typedef struct {
    double DSO;             /* source to rotation axis, > 0 */
    double DSD;             /* source to detector plane, > DSO */
    int64_t nVoxel[3];      /* Nx, Ny, Nz, each > 0 */
    double dVoxel[3];       /* voxel size, each > 0 */
    double offOrigin[3];    /* volume centre relative to the rotation axis origin */
    int64_t nDetector[2];   /* Nu, Nv, each > 0 */
    double dDetector[2];    /* pixel size, each > 0 */
    double offDetector[2];  /* detector centre offset along e_u, e_v */
    double accuracy;        /* CT_INTERP sample spacing / min(dVoxel), in (0, 1]; 0 means 0.5 */
} ct_geometry;

typedef struct ct_plan ct_plan;

/* Validate the geometry and build the per-angle table (host FP64).  Validation: DSD > DSO > 0,
 * all sizes and spacings > 0, n_angles > 0, every angle finite, and every corner of the volume
 * box strictly inside the source orbit (x^2 + y^2 < DSO^2), so that every voxel lies in front of
 * the source at every angle.  `angles` (host, n_angles doubles) is copied.  No device work is
 * done here; the device copy of the table is made on first use on each device.
 * Errors: CT_ERR_ARG (null pointers, n_angles <= 0), CT_ERR_GEOMETRY. */
ct_status ct_plan_create(const ct_geometry *geometry, const double *angles, int64_t n_angles,
                         ct_plan **out);
/* A plan over per-view geometry (Section 2.1: the projectors serve circular, C-arm and helical
 * scans).  views (host, n_views x 12 doubles, copied): for each projection the source S, the
 * detector centre C and the detector's unit axes e_u, e_v, in mm in the volume's frame (the frame
 * of offOrigin).  Pixel (a, b) has its centre at C + u_a e_u + v_b e_v with u_a, v_b from nDetector,
 * dDetector and offDetector exactly as in a circular plan; the geometry's DSO and DSD are not used
 * (ct_plan_info reports the largest DSO_v and DSD_v over the views).  The weights of the voxel-driven
 * backprojectors take depths L along the detector normal n = e_u x e_v: FDK (DSO_v / L)^2 with
 * DSO_v = S.n, pseudo-matched (dx dy dz)/(du dv) DSD_v^2 |SX| / L^3 with DSD_v = (S - C).n; a
 * circular orbit written as views reproduces ct_plan_create's operators.
 * Validation: the grid fields as in ct_plan_create; per view: finite entries, |e_u| = |e_v| = 1
 * and e_u.e_v = 0 to 1e-9, DSD_v > 0, and every corner of the volume box at positive depth.
 * Every resident operator and algorithm (ct_forward, ct_backproject, ct_backproject_noalloc,
 * ct_cgls, ct_sart) accepts such a plan; the FDK reconstruction (ct_fdk_filter, ct_fdk, ct_fdk_host)
 * and the out-of-core calls need a circular orbit and return CT_ERR_ARG.
 * Errors: CT_ERR_ARG (null pointers, n_views <= 0), CT_ERR_GEOMETRY. */
ct_status ct_plan_create_views(const ct_geometry *geometry, const double *views, int64_t n_views, ct_plan **out);
/* Release the plan.  All work that uses it must have completed (device copies are released in
 * stream order, without host synchronisation). */
void ct_plan_destroy(ct_plan *plan);
/* Copy of the validated geometry (accuracy resolved) and the angle count. */
ct_status ct_plan_info(const ct_plan *plan, ct_geometry *geometry, int64_t *n_angles);

/* Forward projection proj = A vol (or proj += A vol when accumulate != 0) for the angles
 * [angle_begin, angle_end) of the plan (Section 2.1; one thread per detector pixel).
 * d_vol: device, Nz*Ny*Nx elements of vol_dtype.  d_proj: device, (angle_end - angle_begin)
 * projections of Nv*Nu elements of proj_dtype; projection 0 of d_proj is angle angle_begin.
 * Errors: CT_ERR_ARG (null pointers, empty or out-of-range angle range), CT_ERR_DTYPE, CT_ERR_HIP. */
ct_status ct_forward(ct_plan *plan, ct_projector projector, const void *d_vol, ct_dtype vol_dtype,
                     void *d_proj, ct_dtype proj_dtype, int accumulate, int64_t angle_begin,
                     int64_t angle_end, void *stream);

/* Backprojection vol = B proj (or vol += B proj) over the angles [angle_begin, angle_end)
 * (Section 2.2; one thread per voxel column segment, loops over angles).  Layouts and errors as
 * ct_forward, with the roles of the arrays swapped. */
ct_status ct_backproject(ct_plan *plan, ct_backprojector backprojector, const void *d_proj,
                         ct_dtype proj_dtype, void *d_vol, ct_dtype vol_dtype, int accumulate,
                         int64_t angle_begin, int64_t angle_end, void *stream);

/* ct_backproject for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * ct_backproject (for FP32 volumes bitwise the same), and it allocates nothing: the exact
 * adjoint's transposed copy of the projections goes to a static device array of the library (128
 * MiB, one per device, held from the library's load until the process ends), in sub-chunks of
 * angles that fit it.  That array is shared by every call on a device, so calls that overlap on
 * one device race; callers serialise them (one stream, or events).
 * Extra errors: CT_ERR_ARG when one angle's transposed copy (4 (Nv + 2) Nu bytes) exceeds the
 * array; CT_ERR_STATE when the plan's angle table is not yet on the current device (it is
 * uploaded by the first allocating call with the plan on that device, e.g. ct_backproject). */
ct_status ct_backproject_noalloc(ct_plan *plan, ct_backprojector backprojector, const void *d_proj,
                                 ct_dtype proj_dtype, void *d_vol, ct_dtype vol_dtype, int accumulate,
                                 int64_t angle_begin, int64_t angle_end, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Out-of-core operators: the image and projections live in host memory and the device holds at
 * most `device_cap_bytes` of working buffers (Algorithm 1 for the forward, Algorithm 2 for the
 * backprojection).  The image is split into equal axial slabs, as large as the cap allows, and
 * the projections into chunks of angles; copies run on side streams overlapped with kernels;
 * partial projections from earlier slabs are accumulated inside the projection kernel.
 * Host arrays may be pageable (staged through a pinned ring) or pinned (copied directly).
 * Only rows of the detector that a slab's rays can meet are moved (per-slab row bands).  With the
 * environment variable CT_OOC_SLAB_BUFFERS=2 the backprojections (and ct_fdk_host) hold two slab
 * buffers, each half as tall for the same cap, and copy a finished slab out on a host thread of
 * its own while the next slab accumulates (double-slab buffering); results are the same bit for
 * bit.  The planner (ct_ooc_plan) follows the same setting.
 * Errors: CT_ERR_ARG, CT_ERR_DTYPE, CT_ERR_CAP (cap below one slice plus buffers), CT_ERR_OOM,
 * CT_ERR_HIP.  Stats may be NULL. */
typedef struct {
    int32_t n_slabs;        /* image splits N_sp */
    int32_t slab_slices;    /* slices per slab (last slab may be shorter) */
    int32_t chunk_angles;   /* angles per projection chunk */
    int32_t n_chunks;       /* chunks per slab */
    double bytes_h2d;       /* host to device bytes moved */
    double bytes_d2h;       /* device to host bytes moved */
    double t_total_s;       /* wall time of the call */
    double t_compute_s;     /* time the compute stream was busy (kernels, incl. overlapped copies) */
    double t_stage_s;       /* host time spent copying between caller memory and pinned staging */
    double t_other_mem_s;   /* allocation, freeing and copies not overlapped with kernels */
    double t_pin_s;         /* allocating the pinned staging buffers (hipHostMalloc; part of
                               t_other_mem_s; 0 when the caller's arrays are pinned) */
} ct_ooc_stats;

/* Pure host planner used by the *_host calls: slab height and chunk size for a cap.
 * direction: 0 = forward (3 projection chunk buffers), 1 = FDK or pseudo-matched backprojection
 * (2 buffers), 2 = exact-adjoint backprojection (2 buffers plus the kernel's transposed FP32 copy
 * of one chunk, 8 (Nv + 2) Nu bytes per angle; chunks of up to 128 angles, because each chunk
 * re-reads the slab's accumulators), 3 = FDK reconstruction (ct_fdk_host: 2 buffers plus one
 * filtered FP32 chunk, 4 Nv Nu bytes per angle).  projector matters for direction 0 only.
 * Errors: CT_ERR_ARG, CT_ERR_DTYPE, CT_ERR_CAP. */
ct_status ct_ooc_plan(const ct_plan *plan, int direction, ct_projector projector, ct_dtype vol_dtype,
                      ct_dtype proj_dtype, uint64_t device_cap_bytes, ct_ooc_stats *out);

ct_status ct_forward_host(ct_plan *plan, ct_projector projector, const void *h_vol, ct_dtype vol_dtype,
                          void *h_proj, ct_dtype proj_dtype, uint64_t device_cap_bytes,
                          ct_ooc_stats *stats);
ct_status ct_backproject_host(ct_plan *plan, ct_backprojector backprojector, const void *h_proj,
                              ct_dtype proj_dtype, void *h_vol, ct_dtype vol_dtype,
                              uint64_t device_cap_bytes, ct_ooc_stats *stats);

/* ---------------------------------------------------------------------------------------------
 * Device-resident algorithms.  Each runs entirely on `stream` without host synchronisation
 * (scalars stay in device memory).  `d_workspace` is optional: when NULL the library allocates
 * stream-ordered scratch (hipMallocAsync) and frees it on the same stream; otherwise it must
 * hold at least the number of bytes reported by the matching *_workspace_bytes call and must
 * not be used concurrently by another call. */

/* CGLS (Bjorck) with A = CT_SIDDON and A^T = CT_BP_ADJOINT over all plan angles: from the
 * initial d_x, minimises ||A x - b||.  x is stored in vol_dtype and b in proj_dtype; the
 * recurrence vectors (r, q projection-shaped; s, p volume-shaped) are FP32, because CGLS search
 * directions are unnormalised and overflow FP16's range on realistic problems.  Inner products,
 * step sizes and the residual-norm recurrence rho_{k+1} = rho_k - alpha_k gamma_k are FP64.
 * d_resid (device, niter+1 doubles, may be NULL) receives sqrt(rho_k); if A p = 0 the iteration
 * stops and the last value repeats.  d_b: device projections (all angles).  d_x: device volume,
 * in: x0, out: result.  The workspace also holds the Siddon projector's column-major copy of the
 * projected volume and the exact adjoint's transposed projection copy, so with d_workspace given
 * an iteration allocates nothing (in geometries whose cone angle the column kernels cover). */
ct_status ct_cgls_workspace_bytes(const ct_plan *plan, ct_dtype vol_dtype, ct_dtype proj_dtype,
                                  uint64_t *bytes);
ct_status ct_cgls(ct_plan *plan, const void *d_b, ct_dtype proj_dtype, void *d_x, ct_dtype vol_dtype,
                  int32_t niter, double *d_resid, void *d_workspace, void *stream);

/* Out-of-core CGLS (Section 3.2 runs CGLS on images larger than device memory): the iteration of
 * ct_cgls with every vector in host memory.  Each iteration runs one ct_forward_host (CT_SIDDON)
 * and one ct_backproject_host (CT_BP_ADJOINT) under device_cap_bytes; the vector updates
 * (x += alpha p, r -= alpha q, p = s + beta p: FP32 fused multiply-adds with the scalars rounded
 * to FP32) and the FP64 inner products run on up to 16 host threads over fixed blocks, so the
 * result does not depend on the thread count.  A start x0 that is all zeros skips the projection
 * of x0 (A 0 = 0 exactly).
 * h_b: host projections, FP32, [n_angles][Nv][Nu], read only.  h_x: host volume, FP32, [Nz][Ny][Nx],
 * in: x0, out: result.  h_workspace: caller-owned host memory (pageable or pinned) of at least
 * ct_cgls_host_workspace_bytes bytes, holding r, q, s and p; not to be shared with a concurrent
 * call.  resid: host, niter+1 doubles receiving sqrt(rho_k) (may be NULL); if A p = 0 the
 * iteration stops and the last value repeats.  stats (may be NULL): byte counts and times summed
 * over the operator calls, the split of the forward calls, t_total_s of the whole call, and the
 * host vector work added to t_other_mem_s.  Errors: as ct_forward_host and ct_backproject_host,
 * CT_ERR_ARG for a NULL pointer or niter < 0, CT_ERR_STATE if a host thread cannot start. */
ct_status ct_cgls_host_workspace_bytes(const ct_plan *plan, uint64_t *bytes);
ct_status ct_cgls_host(ct_plan *plan, const float *h_b, float *h_x, int32_t niter, double *resid,
                       void *h_workspace, uint64_t device_cap_bytes, ct_ooc_stats *stats);

/* OS-SART, the ordered-subset SART that Section 3.2 runs (Andersen and Kak's SART when
 * block = 1), with A = CT_SIDDON and B = CT_BP_FDK.  The angles, in natural order, are cut into
 * consecutive subsets of `block` angles (the last one may be shorter); each subset S makes one
 * update with relaxation lambda:
 *   x += lambda B_S(W (b_S - A_S x)) / V
 * with W = 1/(A_S 1) for rays whose chord through the grid exceeds 1e-2 min(dVoxel) (others weigh
 * 0) and V = B_S 1, voxels with V <= 1e-6 left unchanged.  block: 1 .. n_angles (n_angles gives one
 * SIRT step per sweep).  d_b (proj_dtype) and d_x (vol_dtype) as ct_cgls: the sweeps update an FP32
 * copy of x, so a 16-bit x is rounded once, when the result is written back; b is read in its
 * storage type.  The workspace grows with block (two projection-sized buffers per angle of a
 * subset) and does not depend on the dtypes.  Errors: CT_ERR_ARG for a NULL pointer, niter < 0,
 * block outside [1, n_angles] or a non-finite lambda; CT_ERR_DTYPE. */
ct_status ct_sart_workspace_bytes(const ct_plan *plan, int32_t block, uint64_t *bytes);
ct_status ct_sart(ct_plan *plan, const void *d_b, ct_dtype proj_dtype, void *d_x, ct_dtype vol_dtype,
                  int32_t niter, double lambda, int32_t block, void *d_workspace, void *stream);

/* FDK reconstruction (Feldkamp, Davis and Kress 1984, the algorithm that Section 2.2's
 * FDK-weighted backprojector belongs to) for a full circular scan with uniformly spaced angles.
 * ct_fdk_filter weights and filters the projections of the angles [angle_begin, angle_end):
 * every pixel is multiplied by DSD / sqrt(DSD^2 + u^2 + v^2), (u, v) its detector coordinates
 * from the central ray, and every detector row is convolved (linearly, zero-extended, over the
 * whole row) with the band-limited ramp filter sampled at ds = du DSO / DSD: taps 1/(4 ds^2) at
 * offset 0, 0 at even offsets, -1/(pi n ds)^2 at odd offsets n, times ds.  The result is scaled by
 * dtheta / 2 with dtheta = 2 pi / n_angles of the plan.  FP32 arithmetic, taps summed from the
 * centre outwards.
 * d_proj: device, (angle_end - angle_begin) projections of Nv*Nu elements of proj_dtype, projection
 * 0 of d_proj being angle angle_begin (read only).  d_q: device FP32 array of the same shape,
 * written (may not alias d_proj).  Stream-ordered.
 * ct_fdk runs ct_fdk_filter over all angles into d_workspace, then ct_backproject(CT_BP_FDK) of
 * the filtered projections into d_vol (overwritten, vol_dtype).  d_workspace: device memory of at
 * least ct_fdk_workspace_bytes bytes (n_angles*Nv*Nu FP32), or NULL for stream-ordered scratch.
 * Errors: CT_ERR_ARG for a NULL pointer, a bad angle range or detector rows longer than 4096
 * pixels, CT_ERR_DTYPE for an unknown dtype, CT_ERR_HIP for a launch failure. */
ct_status ct_fdk_filter(ct_plan *plan, const void *d_proj, ct_dtype proj_dtype, float *d_q,
                        int64_t angle_begin, int64_t angle_end, void *stream);
ct_status ct_fdk_workspace_bytes(const ct_plan *plan, uint64_t *bytes);
/* Out-of-core FDK reconstruction: Algorithm 2's slab/chunk streaming of ct_backproject_host with
 * CT_BP_FDK, each projection chunk weighted and filtered on the device (as ct_fdk_filter) right
 * after its upload and before its backprojection.  The filter runs once per chunk and slab.
 * h_proj, h_vol, device_cap_bytes and stats as ct_backproject_host; the plan is ct_ooc_plan's
 * direction 3.  Errors: as ct_backproject_host, and CT_ERR_ARG for detector rows longer than
 * 4096 pixels. */
ct_status ct_fdk_host(ct_plan *plan, const void *h_proj, ct_dtype proj_dtype, void *h_vol, ct_dtype vol_dtype,
                      uint64_t device_cap_bytes, ct_ooc_stats *stats);
ct_status ct_fdk(ct_plan *plan, const void *d_proj, ct_dtype proj_dtype, void *d_vol, ct_dtype vol_dtype,
                 void *d_workspace, void *stream);

/* TV steepest descent (Section 2.3, gradient-descent form): nsteps steps of
 * x <- x - alpha g / ||g||_2, g = grad TV_eps(x) with forward differences on a unit grid and zero
 * difference at the last index of each axis, TV_eps(x) = sum_j sqrt(|D x_j|^2 + eps), and
 * alpha = lambda ||x_in||_2 fixed for the call.  Norms are FP64.  d_x: device volume of the
 * geometry's nVoxel shape, stored in dtype; a 16-bit image is stepped in an FP32 copy in the
 * workspace (one more FP32 volume) and rounded once at the end.  d_workspace: at least
 * ct_tv_workspace_bytes(geometry, dtype) bytes, or NULL for stream-ordered scratch.
 * Errors: CT_ERR_ARG (NULL pointer, nsteps < 0, eps <= 0, non-finite lambda), CT_ERR_DTYPE,
 * CT_ERR_GEOMETRY (a voxel count <= 0). */
ct_status ct_tv_workspace_bytes(const ct_geometry *geometry, ct_dtype dtype, uint64_t *bytes);
ct_status ct_tv_steps(const ct_geometry *geometry, void *d_x, ct_dtype dtype, int32_t nsteps, double lambda,
                      double eps, void *d_workspace, void *stream);
/* The same TV steps on an image in host memory (Section 2.3's regularisation of images larger
 * than device memory), under device_cap_bytes.  The image is cut into equal slabs of axial slices;
 * each is uploaded with one halo slice on either side, because the gradient at slice z reads
 * slices z - 1 .. z + 1.  A step makes two passes over the slabs: the first sums ||g||^2 (and, at
 * the first step, ||x_in||^2) in FP64, slab by slab, in slab order; the second recomputes each
 * slab's gradient and applies the update, with the lower halo taken from the slice below as it was
 * before the step.  The result equals ct_tv_steps up to the order of those FP64 sums (bitwise
 * equal with one slab).  h_x: host FP32 volume of the geometry's nVoxel shape, in: x, out: result
 * (pageable or pinned).  stats (may be NULL): n_slabs, slab_slices, bytes moved, t_total_s.
 * halo_depth = 0 selects that exact form.  halo_depth = d >= 1 selects the splitting of Section
 * 2.3 instead: each slab carries d halo slices on either side and takes up to d steps on its own
 * copy before writing back (one upload and one download of the image per d steps); each step's
 * ||g||^2 is the slab's own sum scaled by (Nz / slab slices), the paper's uniform-distribution
 * estimate, so results differ slightly from the exact form (alpha is exact).
 * Synchronous.  Errors: as ct_tv_steps, CT_ERR_ARG for halo_depth outside [0, 4096], and
 * CT_ERR_CAP for a cap below one slice with its halos and buffers (64 MiB reserve). */
ct_status ct_tv_steps_host(const ct_geometry *geometry, float *h_x, int32_t nsteps, double lambda, double eps,
                           int32_t halo_depth, uint64_t device_cap_bytes, ct_ooc_stats *stats);

/* The ROF model (Rudin, Osher and Fatemi; the second TV minimiser of Section 2.3):
 *   min_u ||u - f||^2 / (2 lambda) + sum_j |(grad u)_j|
 * with forward differences on a unit grid, zero at the last index of each axis, solved by
 * Chambolle's projection iteration (2004): from p = 0, niter times
 *   w = div p - f / lambda,   p <- (p + tau grad w) / (1 + tau |grad w|),
 * then u = f - lambda div p, div being minus the adjoint of grad.  tau <= 1/12 converges in 3D.
 * FP32 throughout.  d_x: device FP32 volume of the geometry's nVoxel shape, in: f, out: u.
 * d_workspace: device memory of at least ct_rof_workspace_bytes bytes (p and w: four volumes), or
 * NULL for stream-ordered scratch.  Stream-ordered.  Errors: CT_ERR_ARG for a NULL pointer,
 * niter < 0, lambda or tau not finite and positive, or more than 65535 slices; CT_ERR_GEOMETRY
 * for a non-positive voxel count. */
ct_status ct_rof_workspace_bytes(const ct_geometry *geometry, uint64_t *bytes);
ct_status ct_rof(const ct_geometry *geometry, void *d_x, int32_t niter, double lambda, double tau, void *d_workspace,
                 void *stream);
/* The same ROF iteration on an image in host memory, under device_cap_bytes (Section 2.3: the ROF
 * minimiser holds five image copies, f, the three components of the dual field p and w, and is split
 * through host memory when they do not fit).  The dual field p lives in h_workspace (host, pageable
 * or pinned, at least ct_rof_host_workspace_bytes = 3 images of FP32).  Rounds of up to halo_depth
 * iterations: each axial slab is uploaded with halo_depth halo slices below and halo_depth + 1 above
 * (the forward difference at a slab's top reads the slice above), iterated on the device, and its
 * own slices of p written back; a last pass forms u = f - lambda div p.  Chambolle's step needs no
 * sum over the image, so the result equals ct_rof bit for bit for any slab height and depth.
 * h_x: host FP32 volume of the geometry's nVoxel shape, in: f, out: u.  Synchronous.  stats (may be
 * NULL): n_slabs, slab_slices, bytes moved, t_total_s.  Errors: as ct_rof, CT_ERR_ARG for a NULL
 * workspace or halo_depth outside [1, 4096], CT_ERR_CAP for a cap below one slice with its halos
 * and buffers (64 MiB reserve). */
ct_status ct_rof_host_workspace_bytes(const ct_geometry *geometry, uint64_t *bytes);
ct_status ct_rof_host(const ct_geometry *geometry, float *h_x, int32_t niter, double lambda, double tau,
                      int32_t halo_depth, void *h_workspace, uint64_t device_cap_bytes, ct_ooc_stats *stats);

/* ---------------------------------------------------------------------------------------------
 * Small device utilities used by the algorithms, exported for callers that compose their own. */

/* out[0] = sum_i a[i] * b[i] in FP64 with a fixed reduction order (bitwise repeatable).
 * a, b: device arrays of n elements of dtype (any ct_dtype, CT_F64 included); out: device double. */
ct_status ct_dot(const void *d_a, const void *d_b, ct_dtype dtype, int64_t n, double *d_out,
                 void *stream);
/* Storage conversion: dst[i] = (dst_dtype) src[i] (round to nearest even; from CT_F64 to the 16-bit
 * types through FP32).  Any ct_dtype, CT_F64 included. */
ct_status ct_convert(const void *d_src, ct_dtype src_dtype, void *d_dst, ct_dtype dst_dtype, int64_t n,
                     void *stream);

/* Message for the calling thread's most recent failure ("" if none). */
const char *ct_last_error(void);
/* Library version string. */
const char *ct_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CT_H */
