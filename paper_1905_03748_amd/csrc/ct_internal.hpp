// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ct.h"

namespace ct {

// Per-angle geometry in voxel-index space (voxel (i,j,k) centre at index coordinates (i,j,k)).
// Double precision: the source sits ~DSO/d voxels away from the grid, so rays are set up in FP64
// and traversed in FP32 relative to their entry point.
//
// Every plan fills the general part (e_v, the projective map M, DSO_v, the pseudo-matched constant),
// so the per-view kernels run on circular plans too; c and s are meaningful for circular plans only.
// M's rows are a* L, b* L and L as affine functions of the voxel index (i, j, k, 1), where L (mm) is
// the voxel's depth from the source along the detector normal n = e_u x e_v and (a*, b*) the
// continuous detector indices of the ray from the source through the voxel centre.
struct AngleGeo {
    double c, s;         // cos, sin of the angle (circular plans)
    double S[3];         // source position, index units
    double Dc[3];        // (detector centre - source), index units
    double eu[3];        // e_u / dVoxel (index units per mm along the detector u axis)
    double ev[3];        // e_v / dVoxel
    double M[12];        // projective map, row-major 3 x 4
    double DSOv;         // FDK weight numerator: the world origin's depth (DSO in a circular orbit)
    double pmc;          // pseudo-matched constant dx dy dz / (du dv) * DSD_v^2
    double Smm[3];       // source position, mm
    double DSDv;         // source to detector plane, mm (DSD in a circular orbit)
};
static_assert(sizeof(AngleGeo) == 256, "AngleGeo layout");

void set_error(const std::string &msg);
ct_status fail(ct_status st, const std::string &msg);
ct_status hip_fail(hipError_t e, const char *what);

// Allocation-failure injection for tests of the error paths: with CT_FAULT_ALLOC=n (optionally
// followed by ":tag"), the n-th device or pinned allocation of the library after the variable last
// changed fails as out-of-memory.  Unset, it costs one getenv per allocation.
hipError_t fault_check();
#define CT_MALLOC(p, n) (::ct::fault_check() != hipSuccess ? hipErrorOutOfMemory : hipMalloc((p), (n)))
#define CT_MALLOC_ASYNC(p, n, s) (::ct::fault_check() != hipSuccess ? hipErrorOutOfMemory : hipMallocAsync((p), (n), (s)))
#define CT_HOST_MALLOC(p, n) \
    (::ct::fault_check() != hipSuccess ? hipErrorOutOfMemory : hipHostMalloc((p), (n), hipHostMallocDefault))

#define CT_HIP(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::ct::hip_fail(e_, #call);   \
    } while (0)

size_t dtype_size(ct_dtype t);
bool dtype_ok(int t);      // a storage type of the operators and algorithms (FP32, FP16, BF16)
bool dtype_ok_any(int t);  // also FP64 (conversion and inner products)

}  // namespace ct

struct ct_plan {
    ct_geometry g;
    std::vector<double> angles;  // circular plans; a plan of views holds zeros here
    bool views = false;          // built from per-view vectors: the per-view kernels serve it
    bool vertical = true;        // every view's e_v is +z, e_u horizontal and C at the source's
                                 // height (circular and helical scans): the column walks apply
    std::vector<ct::AngleGeo> tab;
    std::mutex mu;
    int vl_ww = -1, vl_hw = -1;  // LDS window of the per-view backprojection (-1: not computed yet)
    int va_ww = -1, va_hw = -1;  // LDS window of the per-view exact adjoint (-1: not computed yet)
    struct DevTab {
        ct::AngleGeo *ptr;
        hipEvent_t ready;  // recorded after the upload on the stream that first used the plan
    };
    std::map<int, DevTab> dtab;  // device copies, per device id
};

namespace ct {

// Device copy of the per-angle table for the current device.  The first use uploads it in stream
// order on `st` (no host synchronisation); later uses on any stream wait for that upload.
ct_status plan_device_table(ct_plan *p, hipStream_t st, const AngleGeo **out);
// The same without the upload: CT_ERR_STATE when the table is not yet on the current device.
ct_status plan_device_table_existing(ct_plan *p, hipStream_t st, const AngleGeo **out);

// Range of axial slices a launch covers and where its memory starts.
//   own_lo/own_hi: slices whose voxels this launch owns (forward: rays are clipped to them;
//                  backprojection: voxels written).
//   mem_lo: slice stored at the base of the volume pointer; mem_n: slices present in memory.
struct Slab {
    int64_t own_lo, own_hi;
    int64_t mem_lo, mem_n;
    bool first, last;  // the interpolated projector extends ownership to +-inf at the ends
    bool scratch_ok;   // the launch may allocate device scratch (resident calls; not under a cap)
    bool zcol = false; // exact-adjoint backprojection only: the slab is column-major, [y][x][mem_n]
    bool no_alloc = false;  // the launch allocates nothing (the angle table must be on the device)
};

inline Slab full_slab(const ct_geometry &g) {
    Slab s;
    s.own_lo = 0;
    s.own_hi = g.nVoxel[2];
    s.mem_lo = 0;
    s.mem_n = g.nVoxel[2];
    s.first = s.last = true;
    s.scratch_ok = true;
    return s;
}

// Kernel launchers (resident; pointers are device pointers; projection pointer holds the
// angles [a0, a1) starting at projection 0).
// vcopy: optional copy of vol in the layout the projector reads, kept by the caller (then no
// scratch copy is made): for Siddon the column-major slots of launch_zcols (for a slab launch:
// its mem_n slices, mem_n + 2 slots per column), for the interpolated projector the [z][x][y]
// transpose of launch_transpose_xy.
ct_status launch_forward(ct_plan *p, ct_projector kind, const void *vol, ct_dtype vt, void *proj,
                         ct_dtype pt, int accumulate, int64_t a0, int64_t a1, const Slab &slab,
                         hipStream_t st, const void *vcopy = nullptr);
ct_status launch_transpose_xy(const void *vol, ct_dtype vt, void *volT, int64_t nx, int64_t ny, int64_t nz,
                              hipStream_t st);
// [z][y][x] -> [y][x][slot], slot z + 1 holding voxel z, slots 0 and nz + 1 zero
// (nx * ny * (nz + 2) elements)
ct_status launch_zcols(const void *vol, ct_dtype vt, void *vz, int64_t nx, int64_t ny, int64_t nz, hipStream_t st);
// slices [0, nz) of src ([z][y][x]) into slots slot0 + z of columns of nzp slots; pads bit 0 / 1
// zero slot 0 / nzp - 1
ct_status launch_zcols_piece(const void *src, ct_dtype vt, void *vz, int64_t nx, int64_t ny, int64_t nz, int64_t nzp,
                             int64_t slot0, int pads, hipStream_t st);
// the same copy converted to FP32 (vz: FP32), and its inverse back to the volume's type
ct_status launch_zcols_f32(const void *vol, ct_dtype vt, float *vz, int64_t nx, int64_t ny, int64_t nz, hipStream_t st);
ct_status launch_zcols_inv_f32(const float *vz, void *vol, ct_dtype vt, int64_t nx, int64_t ny, int64_t nz,
                               hipStream_t st);
// inverse: column-major slots -> [z][y][x]
ct_status launch_zcols_inv(const void *vz, ct_dtype vt, void *vol, int64_t nx, int64_t ny, int64_t nz, hipStream_t st);
// slots [slot0, slot0 + zn) of column-major columns of nzp slots -> [zn][ny][nx]
ct_status launch_zcols_inv_piece(const void *vz, ct_dtype vt, void *dst, int64_t nx, int64_t ny, int64_t zn,
                                 int64_t nzp, int64_t slot0, hipStream_t st);
// the exact adjoint runs its column kernel (which supports column-major slabs) for this geometry
bool adj_col_ok(const ct_plan *p);
inline int64_t zcol_elems(const ct_geometry &g) { return g.nVoxel[0] * g.nVoxel[1] * (g.nVoxel[2] + 2); }
// whether the column Siddon walk is valid for angles [a0, a1) of the plan
bool zcol_ok(const ct_plan *p, int64_t a0, int64_t a1);
// adj_scratch (optional, adj_bytes): device memory for the exact adjoint's transposed projection
// copy (adj_chunk_bytes_per_angle bytes per angle); without it a launch that may allocate takes
// stream-ordered scratch, and one that may not falls back to the slower gather kernel.
ct_status launch_backproject(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                             ct_dtype vt, int accumulate, int64_t a0, int64_t a1, const Slab &slab,
                             hipStream_t st, void *adj_scratch = nullptr, size_t adj_bytes = 0);
size_t adj_chunk_bytes_per_angle(const ct_geometry &g);
// ct_backproject through the library's static device scratch (no allocation of any kind)
ct_status backproject_noalloc(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                              ct_dtype vt, int accumulate, int64_t a0, int64_t a1, hipStream_t st);

// Algorithm helpers (kern_algos.hip)
ct_status dot_f64(const void *a, const void *b, ct_dtype t, int64_t n, double *out, double *partials,
                  hipStream_t st);
ct_status convert(const void *src, ct_dtype st_, void *dst, ct_dtype dt, int64_t n, hipStream_t st);
size_t dot_partials_count();

ct_status cgls_run(ct_plan *p, const void *b, ct_dtype pt, void *x, ct_dtype vt, int32_t niter,
                   double *resid, void *work, hipStream_t st);
size_t cgls_workspace(const ct_plan *p, ct_dtype vt, ct_dtype pt);
ct_status sart_run(ct_plan *p, const void *b, ct_dtype pt, void *x, ct_dtype vt, int32_t niter, double lambda,
                   int32_t block, void *work, hipStream_t st);
size_t sart_workspace(const ct_plan *p, int32_t block);
ct_status tv_run(const ct_geometry &g, void *x, ct_dtype vt, int32_t nsteps, double lambda, double eps, void *work,
                 hipStream_t st);
size_t tv_workspace(const ct_geometry &g, ct_dtype vt);
ct_status rof_run(const ct_geometry &g, void *x, int32_t niter, double lambda, double tau, void *work, hipStream_t st);
size_t rof_workspace(const ct_geometry &g);
// the same on a host image; hp: host workspace of rof_host_workspace bytes (the dual field)
ct_status rof_host_run(const ct_geometry &g, float *hx, int32_t niter, double lambda, double tau, int32_t depth,
                       float *hp, uint64_t cap, ct_ooc_stats *stats);
size_t rof_host_workspace(const ct_geometry &g);
ct_status tv_host_run(const ct_geometry &g, float *hx, int32_t nsteps, double lambda, double eps, int32_t depth,
                      uint64_t cap, ct_ooc_stats *stats);
// FDK reconstruction (kern_fdk.hip): weighted, ramp-filtered FP32 rows of the angles [a0, a1)
// (proj and q hold those angles from projection 0), and the whole reconstruction through a
// workspace of fdk_workspace bytes (stream-ordered scratch when work is null)
ct_status fdk_filter(ct_plan *p, const void *proj, ct_dtype pt, float *q, int64_t a0, int64_t a1, hipStream_t st);
ct_status fdk_run(ct_plan *p, const void *proj, ct_dtype pt, void *vol, ct_dtype vt, void *work, hipStream_t st);
size_t fdk_workspace(const ct_plan *p);

// Per-view kernels (kern_views.hip): every backprojector and the SART update for plans of views
ct_status launch_backproject_views(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                                   ct_dtype vt, int accumulate, int64_t a0, int64_t a1, const Slab &slab,
                                   const AngleGeo *tab, hipStream_t st);
ct_status launch_sart_update_views(ct_plan *p, const float *r, float *vol, int64_t a0, int64_t a1, float lambda,
                                   const AngleGeo *tab, hipStream_t st);

// SART pieces (kern_backproject.hip / kern_forward.hip)
ct_status launch_ray_chord(ct_plan *p, float *chord, int64_t a0, int64_t a1, hipStream_t st);
// one (OS-)SART update over the angle subset [a0, a1): r holds its weighted residuals [a1-a0][v][u]
ct_status launch_sart_update(ct_plan *p, const float *r, float *vol, int64_t a0, int64_t a1, float lambda,
                             hipStream_t st);
// the same update on the column-major copy (launch_zcols layout), residuals rT in [a1-a0][u][v] layout
ct_status launch_sart_update_col(ct_plan *p, const float *rT, float *vz, int64_t a0, int64_t a1, float lambda,
                                 hipStream_t st);

// Out-of-core (ooc.cpp)
ct_status ooc_plan(const ct_plan *p, int direction, ct_projector proj, ct_dtype vt, ct_dtype pt,
                   uint64_t cap, ct_ooc_stats *out);
ct_status ooc_forward(ct_plan *p, ct_projector kind, const void *h_vol, ct_dtype vt, void *h_proj,
                      ct_dtype pt, uint64_t cap, ct_ooc_stats *stats);
// fdk_filtered: the FDK reconstruction, each projection chunk weighted and ramp-filtered on the
// device before its FDK-weighted backprojection (kind is then CT_BP_FDK)
ct_status ooc_backproject(ct_plan *p, ct_backprojector kind, const void *h_proj, ct_dtype pt, void *h_vol,
                          ct_dtype vt, uint64_t cap, ct_ooc_stats *stats, bool fdk_filtered = false);

// Out-of-core CGLS (ooc_cgls.cpp): host workspace r, q, s, p in FP32
size_t cgls_host_workspace(const ct_plan *p);
ct_status cgls_host_run(ct_plan *p, const float *b, float *x, int32_t niter, double *resid, void *work,
                        uint64_t cap, ct_ooc_stats *stats);

}  // namespace ct
