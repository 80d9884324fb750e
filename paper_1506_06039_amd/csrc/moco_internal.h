// Internal declarations shared by the C ABI (capi.cpp) and the HIP kernels.
// Not installed; the public interface is include/moco.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "moco.h"

namespace moco {

// Geometry of one search: full-resolution m x n, searched grid mg x ng,
// window w (W = 2w-1 shifts per axis).
struct Geom {
    int m, n, mg, ng, w, W, ds;
    moco_dtype dtype;
};

// Resident, prepared template.  All pointers are device memory owned by it.
struct Tmpl {
    Geom g;
    void *raw;        // m x n pixels of g.dtype (full resolution, for the x2 refine)
    double *coarse;   // mg x ng FP64 (box mean when ds)
    double *btab;     // W x W: sum of b'^2 over D_{s,t}, [s+w-1][t+w-1]
    int32_t bmin, bmax;   // range of the integer grid values (uint16 data): box sums or raw
    int8_t *limbs;    // int8 MFMA form: packed template limbs (see corr_int8.hip), or null
    size_t limbs_bytes;
    int nlimb_b;      // number of base-256 limbs the template needs (int8 form)
    int32_t center;   // common integer offset subtracted from frame and template (int8 form)
};

// Per-frame intermediate results of the coarse search (device).
struct CoarseOut {
    int32_t s, t;     // argmin on the searched grid
};

// ---- launchers (kernels_basic.hip) -------------------------------------
// All return hipSuccess or the launch error; they only enqueue.
hipError_t launch_coarse(const void *frames, moco_dtype dt, int C, const Geom &g, double *coarse,
                         hipStream_t st);
hipError_t launch_sat_sq(const double *coarse, int C, const Geom &g, double *sat, hipStream_t st);
hipError_t launch_btab(const double *sat_b, const Geom &g, double *btab, hipStream_t st);
hipError_t launch_corr_fp64(const double *coarse, const double *tcoarse, int C, const Geom &g,
                            double *h, hipStream_t st);
hipError_t launch_combine(const double *sat, const double *btab, const double *h, int C,
                          const Geom &g, double *fsurf, double *fmin, int32_t *coarse_st,
                          int32_t *shifts, double *gaps, double *frefine, hipStream_t st);
hipError_t launch_refine(const void *frames, const void *traw, int C, const Geom &g,
                         const int32_t *coarse_st, int32_t *shifts, double *frefine,
                         double *gaps, hipStream_t st);

}  // namespace moco
