/* drops.c -- FP64 CPU oracle of the drop-size diagnostic of the jet study
 * (Sec. on liquid jet breakup: breakup length and equivalent drop diameter
 * d_e against the Weber number).
 *
 * TEST INFRASTRUCTURE ONLY (the tests, the smoke check and the benchmark's
 * CPU-baseline leg).  Shares no code with the HIP implementation.
 *
 * The paper reports d_e / D_j without stating how drops are identified;
 * the reading taken here:
 *   - the liquid is the node set {phi > thr} (thr = 1/2: the interface
 *     level of the phase field);
 *   - drops are its connected components under face (6-neighbour in 3D,
 *     4-neighbour in 2D) connectivity, an axis wrapping where periodic;
 *   - a component's volume is its node count V, its equivalent diameter the
 *     diameter of the sphere (3D) or disc (2D) of that volume:
 *     d_e = (6 V / pi)^(1/3), resp. (4 V / pi)^(1/2).
 * Components are found by breadth-first search from each unlabelled liquid
 * node in ascending node order, so each component is labelled with its
 * smallest node index.  The threshold test is taken on the float phase
 * field in float, as the GPU takes it. */
#include <math.h>
#include <stdlib.h>

static long node_at(const int n[3], const int c[3]) {
  return (long)c[0] + (long)n[0] * ((long)c[1] + (long)n[1] * c[2]);
}

/* label[N]: smallest node index of the node's component, or -1 */
int ora_label(const float* phi, int nx, int ny, int nz, unsigned periodic, float thr, int* label) {
  const int n[3] = {nx, ny, nz};
  const long N = (long)nx * ny * nz;
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  long* queue = (long*)malloc(sizeof(long) * (size_t)N);
  if (!queue) return -2;
  for (long i = 0; i < N; ++i) label[i] = -1;
  for (long s = 0; s < N; ++s) {
    if (!(phi[s] > thr) || label[s] >= 0) continue;
    long head = 0, tail = 0;
    queue[tail++] = s;
    label[s] = (int)s;
    while (head < tail) {
      const long v = queue[head++];
      int c[3] = {(int)(v % nx), (int)((v / nx) % ny), (int)(v / ((long)nx * ny))};
      for (int d = 0; d < 3; ++d) {
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          int m[3] = {c[0], c[1], c[2]};
          m[d] += sgn;
          if (m[d] < 0 || m[d] >= n[d]) {
            if (!((periodic >> d) & 1u)) continue;
            m[d] = (m[d] + n[d]) % n[d];
          }
          const long u = node_at(n, m);
          if (phi[u] > thr && label[u] < 0) {
            label[u] = (int)s;
            queue[tail++] = u;
          }
        }
      }
    }
  }
  free(queue);
  return 0;
}

/* Components of a labelling in ascending order of their label: root,
 * node count, smallest and largest coordinate along `axis`, equivalent
 * diameter.  Returns the number of components (at most cap are written),
 * or -1 on bad arguments. */
int ora_components(const int* label, int nx, int ny, int nz, int axis, int cap, int* root, int* size,
                   int* lo, int* hi, double* deq) {
  const long N = (long)nx * ny * nz;
  if (axis < 0 || axis > 2 || cap < 0) return -1;
  int* cid = (int*)malloc(sizeof(int) * (size_t)N);
  if (!cid) return -1;
  int nc = 0;
  for (long i = 0; i < N; ++i) {
    cid[i] = -1;
    if (label[i] == i) cid[i] = nc++;  /* roots in ascending order */
  }
  for (int k = 0; k < nc && k < cap; ++k) {
    size[k] = 0;
    lo[k] = 1 << 30;
    hi[k] = -1;
  }
  for (long i = 0; i < N; ++i) {
    if (label[i] < 0) continue;
    const int k = cid[label[i]];
    if (k >= cap) continue;
    const int c[3] = {(int)(i % nx), (int)((i / nx) % ny), (int)(i / ((long)nx * ny))};
    if (label[i] == i) root[k] = (int)i;
    size[k] += 1;
    if (c[axis] < lo[k]) lo[k] = c[axis];
    if (c[axis] > hi[k]) hi[k] = c[axis];
  }
  for (int k = 0; k < nc && k < cap; ++k)
    deq[k] = nz > 1 ? cbrt(6.0 * size[k] / M_PI) : sqrt(4.0 * size[k] / M_PI);
  free(cid);
  return nc;
}
