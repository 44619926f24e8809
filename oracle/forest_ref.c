/*
 * forest_ref.c -- oracle side of the heterogeneous forest: point cloud to
 * per-cell forest codes, and the leaf-area density of a coded cell.
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_ref.c).  Shares nothing with the HIP
 * library, which has its own implementation of the same interface.
 *
 * Method (Shao et al., arXiv 2206.15454, Sec. 3, the forest description
 * before Algorithm 1, and the set-up steps of Algorithm 1): every cell that holds at least one
 * point of the forest point cloud is a forest cell.  Its code stores the
 * height h of the forest object it belongs to (vertical extent of the
 * object's bounding box), its own height y above the object's lowest cell
 * and the height y_m of the LAD maximum, packed with a bit mask.  The drag
 * uses the LAD of Eq. (af_theory) evaluated from those three numbers.
 *
 * Readings (the paper names the fields but not their packing or how an
 * object is delimited):
 *   F1  A point (x, y, z), in cell units with the domain origin at 0, lies
 *       in cell (floor x, floor y, floor z); points outside the domain are
 *       an error.
 *   F2  A forest object is a set of forest cells connected through faces
 *       (6-neighbourhood), periodic in x and z like the flow, not in y.
 *   F3  h = number of cell rows the object spans; y = row of the cell minus
 *       the object's lowest row; Eq. (af_theory) is evaluated at the cell
 *       centre y + 1/2 (as for the homogeneous profile).
 *   F4  y_m is given as a fraction of h (the paper's set-ups use 0.7 h) and
 *       stored as q_m = round(4096 * fraction), y_m = h q_m / 4096.
 *   F5  Code bits: h in bits 0-9 (0 = not forest), y in bits 10-19, q_m in
 *       bits 20-31.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* F5 */
static uint32_t pack(uint32_t h, uint32_t y, uint32_t qm) {
    return h | (y << 10) | (qm << 20);
}

void ref_forest_decode(uint32_t code, int *h, int *y, int *qm) {
    *h = (int)(code & 1023u);
    *y = (int)((code >> 10) & 1023u);
    *qm = (int)(code >> 20);
}

/* LAD of one coded cell: a_fm times Eq. (af_theory) at y + 1/2 (F3, F4),
 * or a_fm in every forest cell when constant != 0 (the constant-LAD case
 * of Table tab:forest_cases).  0 for a cell that is not forest. */
double ref_forest_lad(uint32_t code, double afm, int constant) {
    int h, y, qm;
    ref_forest_decode(code, &h, &y, &qm);
    if (h == 0) return 0.0;
    if (constant) return afm;
    double hh = (double)h;
    double ym = hh * (double)qm / 4096.0;
    double yc = (double)y + 0.5;
    double n = (yc < ym) ? 6.0 : 0.5;
    double r = (hh - ym) / (hh - yc);
    return afm * (pow(r, n) * exp(n * (1.0 - r)));
}

/* Point cloud -> codes[nz][ny][nx].  Returns 0, or 1 for a point outside
 * the domain, a bad fraction or an object taller than 1023 rows. */
int ref_forest_codes(const double *pts, int64_t npts, int nx, int ny, int nz, double ym_frac,
                     uint32_t *codes, int64_t *nobjects) {
    if (nx < 1 || ny < 1 || nz < 1 || !(ym_frac >= 0.0)) return 1;
    double qd = floor(ym_frac * 4096.0 + 0.5);
    if (!(qd <= 4095.0)) return 1;
    uint32_t qm = (uint32_t)qd;
    size_t n = (size_t)nx * ny * nz;
    for (size_t x = 0; x < n; ++x) codes[x] = 0;

    /* F1: mark forest cells (temporarily with code 1) */
    for (int64_t p = 0; p < npts; ++p) {
        double fx = floor(pts[3 * p]), fy = floor(pts[3 * p + 1]), fz = floor(pts[3 * p + 2]);
        if (!(fx >= 0.0 && fx < nx && fy >= 0.0 && fy < ny && fz >= 0.0 && fz < nz)) return 1;
        size_t x = ((size_t)fz * ny + (size_t)fy) * nx + (size_t)fx;
        codes[x] = 1;
    }

    /* F2: breadth-first search over face neighbours; label[x] = object id + 1 */
    int64_t *label = (int64_t *)calloc(n, sizeof(int64_t));
    size_t *queue = (size_t *)malloc(n * sizeof(size_t));
    int *lo = NULL, *hi = NULL;
    int64_t nobj = 0, cap = 0;
    int rc = 0;
    if (!label || !queue) rc = 1;
    for (size_t s = 0; s < n && rc == 0; ++s) {
        if (codes[s] == 0 || label[s] != 0) continue;
        if (nobj == cap) {
            cap = cap ? 2 * cap : 64;
            int *l2 = (int *)realloc(lo, cap * sizeof(int));
            if (l2) lo = l2;
            int *h2 = (int *)realloc(hi, cap * sizeof(int));
            if (h2) hi = h2;
            if (!l2 || !h2) { rc = 1; break; }
        }
        nobj += 1;
        lo[nobj - 1] = ny;
        hi[nobj - 1] = -1;
        size_t head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = nobj;
        while (head < tail) {
            size_t x = queue[head++];
            int i = (int)(x % nx), j = (int)((x / nx) % ny), k = (int)(x / ((size_t)nx * ny));
            if (j < lo[nobj - 1]) lo[nobj - 1] = j;
            if (j > hi[nobj - 1]) hi[nobj - 1] = j;
            int nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                            {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
            for (int m = 0; m < 6; ++m) {
                int a = nb[m][0], b = nb[m][1], c = nb[m][2];
                if (b < 0 || b >= ny) continue;
                a = (a + nx) % nx;
                c = (c + nz) % nz;
                size_t y = ((size_t)c * ny + b) * nx + a;
                if (codes[y] != 0 && label[y] == 0) {
                    label[y] = nobj;
                    queue[tail++] = y;
                }
            }
        }
    }

    /* F3-F5: codes from each object's vertical extent */
    for (size_t x = 0; x < n && rc == 0; ++x) {
        if (label[x] == 0) continue;
        int64_t o = label[x] - 1;
        int h = hi[o] - lo[o] + 1;
        int j = (int)((x / nx) % ny);
        if (h > 1023) { rc = 1; break; }
        codes[x] = pack((uint32_t)h, (uint32_t)(j - lo[o]), qm);
    }
    if (rc != 0)
        for (size_t x = 0; x < n; ++x) codes[x] = 0;
    if (nobjects) *nobjects = rc == 0 ? nobj : 0;
    free(label);
    free(queue);
    free(lo);
    free(hi);
    return rc;
}
