/* drops.h -- C ABI of the drop-size diagnostic of the jet study (the
 * equivalent drop diameter d_e against the Weber number, in the section on
 * liquid jet breakup): connected components of the liquid {phi > thr} of a
 * phase field and, per component, its volume, extent and equivalent
 * diameter.
 *
 * Reading (the paper does not state how drops are identified): the liquid
 * is {phi > thr} with thr = 1/2, the interface level; drops are its
 * connected components under face connectivity (6 neighbours in 3D, 4 in
 * 2D), an axis wrapping where it is periodic; a component's volume V is its
 * node count and d_e = (6 V / pi)^(1/3) (3D) or (4 V / pi)^(1/2) (2D).
 *
 * Fields are device arrays of N = nx * ny * nz values with node index
 * x + nx * (y + ny * z) (x fastest), as lbm_fields writes them.  All device
 * buffers are owned by the caller.  Calls launch on `stream` (hipStream_t,
 * NULL = default) and synchronise it where stated.  Errors return a negative
 * code; dr_last_error() describes the last one (per thread). */
#pragma once
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DR_OK 0
#define DR_EINVAL (-1)     /* bad argument (null buffer, extent, axis, workspace too small) */
#define DR_EDEVICE (-3)    /* a HIP call failed */
#define DR_ECAPACITY (-6)  /* more components than the caller's capacity */
#define DR_EINTERNAL (-7)  /* a union-find iteration bound was exceeded (labels not valid) */

const char* dr_last_error(void);

/* Bytes of device workspace for fields of nx x ny x nz nodes (flags, block
 * counts and offsets, one int per node).  0 for an invalid extent
 * (any extent < 1, or N > 2^30). */
size_t dr_workspace_bytes(int nx, int ny, int nz);

/* Label the liquid of phi_dev[N]:
 *   label_dev[i] = the smallest node index of i's component if phi[i] > thr
 *                  (compared in float), else -1;
 *   periodic: bit d set = axis d (0 x, 1 y, 2 z) wraps.
 * workspace: dr_workspace_bytes() bytes of device memory.  Synchronises the
 * stream (to read the union-find status). */
int dr_label(const float* phi_dev, int nx, int ny, int nz, unsigned periodic, float thr, int* label_dev,
             void* workspace, size_t ws_bytes, void* stream);

/* Components of a labelling made by dr_label, in ascending order of their
 * label, into device arrays of capacity `cap`:
 *   root[k]  the component's label (its smallest node index),
 *   size[k]  its node count,
 *   lo[k], hi[k]  its smallest and largest coordinate along `axis` (0 x, 1 y, 2 z),
 *   deq[k]   its equivalent diameter (sphere when nz > 1, disc when nz == 1).
 * *ncomp (host) receives the number of components.  If it exceeds cap the
 * first cap components are written and DR_ECAPACITY is returned.
 * Synchronises the stream. */
int dr_components(const int* label_dev, int nx, int ny, int nz, int axis, int cap, int* root_dev,
                  int* size_dev, int* lo_dev, int* hi_dev, float* deq_dev, int* ncomp, void* workspace,
                  size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
