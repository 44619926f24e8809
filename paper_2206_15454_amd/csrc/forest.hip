// Heterogeneous forest, host side (Sec. 3, the forest description before
// Algorithm 1, and the set-up steps of Algorithm 1): point cloud -> per-cell forest codes, and
// codes -> the compact form the step kernel reads (a 16-bit index per cell
// into a table of distinct LAD values).
//
// Code bit fields (the interface declared in lbm.h): h bits 0-9, y bits
// 10-19, q_m bits 20-31, y_m = h q_m / 4096.
#include <cmath>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.h"

namespace lbmx {

namespace {

// root of a in the union-find forest, with path halving
int32_t root(std::vector<int32_t> &parent, int32_t a) {
    while (parent[a] != a) {
        parent[a] = parent[parent[a]];
        a = parent[a];
    }
    return a;
}

}  // namespace

// LAD of one code: Eq. (af_theory) at the cell centre, or afm (constant).
double forest_code_lad(uint32_t code, double afm, bool constant) {
    const uint32_t h = code & 1023u;
    if (h == 0) return 0.0;
    if (constant) return afm;
    const double hh = (double)h;
    const double ym = hh * (double)(code >> 20) / 4096.0;
    const double y = (double)((code >> 10) & 1023u) + 0.5;
    const double nexp = y < ym ? 6.0 : 0.5;
    const double r = (hh - ym) / (hh - y);
    return std::exp(nexp * (std::log(r) + 1.0 - r)) * afm;
}

bool forest_table(const uint32_t *codes, long long n, double afm, bool constant,
                  std::vector<uint16_t> &idx, std::vector<double> &table, std::string *why) {
    std::unordered_map<uint32_t, uint16_t> slot;
    table.assign(1, 0.0);  // index 0: not forest
    idx.assign((size_t)n, 0);
    for (long long x = 0; x < n; ++x) {
        const uint32_t c = codes[x];
        if ((c & 1023u) == 0) continue;
        if (((c >> 10) & 1023u) >= (c & 1023u)) {
            *why = "forest code with y >= h";
            return false;
        }
        auto it = slot.find(c);
        if (it == slot.end()) {
            if (table.size() >= (size_t)kForestTable) {
                *why = "more than 65535 distinct forest codes";
                return false;
            }
            it = slot.emplace(c, (uint16_t)table.size()).first;
            table.push_back(forest_code_lad(c, afm, constant));
        }
        idx[(size_t)x] = it->second;
    }
    return true;
}

}  // namespace lbmx

extern "C" {

lbm_status lbm_forest_codes(const double *points, int64_t npoints, int32_t nx, int32_t ny,
                            int32_t nz, double ym_frac, uint32_t *codes, int64_t *nobjects) {
    if (!codes || nx < 1 || ny < 1 || nz < 1 || npoints < 0 || (npoints > 0 && !points))
        return LBM_EINVAL;
    const long long n = (long long)nx * ny * nz;
    if (n >= (1LL << 31)) return LBM_EINVAL;
    const double qd = std::floor(ym_frac * 4096.0 + 0.5);
    if (!(ym_frac >= 0.0) || !(qd <= 4095.0)) return LBM_EINVAL;
    const uint32_t qm = (uint32_t)qd;

    // forest cells: parent = itself; other cells: -1
    std::vector<int32_t> parent((size_t)n, -1);
    for (int64_t p = 0; p < npoints; ++p) {
        const double x = points[3 * p], y = points[3 * p + 1], z = points[3 * p + 2];
        if (!(x >= 0.0 && x < nx && y >= 0.0 && y < ny && z >= 0.0 && z < nz))
            return LBM_EINVAL;
        const long long c = ((long long)z * ny + (long long)y) * nx + (long long)x;
        parent[(size_t)c] = (int32_t)c;
    }
    // join face neighbours in +x, +y, +z (x and z periodic)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int32_t c = (int32_t)(((long long)k * ny + j) * nx + i);
                if (parent[c] < 0) continue;
                const int32_t nb[3] = {
                    (int32_t)(((long long)k * ny + j) * nx + (i + 1) % nx),
                    j + 1 < ny ? (int32_t)(((long long)k * ny + j + 1) * nx + i) : -1,
                    (int32_t)(((long long)((k + 1) % nz) * ny + j) * nx + i)};
                for (int32_t o : nb) {
                    if (o < 0 || parent[o] < 0) continue;
                    const int32_t ra = lbmx::root(parent, c), rb = lbmx::root(parent, o);
                    if (ra != rb) parent[ra > rb ? ra : rb] = ra > rb ? rb : ra;
                }
            }
    // vertical extent of every object (keyed by its root)
    std::unordered_map<int32_t, std::pair<int, int>> extent;
    for (long long c = 0; c < n; ++c) {
        if (parent[(size_t)c] < 0) continue;
        const int j = (int)((c / nx) % ny);
        auto it = extent.emplace(lbmx::root(parent, (int32_t)c), std::make_pair(j, j)).first;
        if (j < it->second.first) it->second.first = j;
        if (j > it->second.second) it->second.second = j;
    }
    for (auto &e : extent)
        if (e.second.second - e.second.first + 1 > 1023) return LBM_EINVAL;
    for (long long c = 0; c < n; ++c) {
        if (parent[(size_t)c] < 0) {
            codes[c] = 0;
            continue;
        }
        const auto &e = extent[lbmx::root(parent, (int32_t)c)];
        const uint32_t h = (uint32_t)(e.second - e.first + 1);
        const uint32_t y = (uint32_t)((c / nx) % ny - e.first);
        codes[c] = h | (y << 10) | (qm << 20);
    }
    if (nobjects) *nobjects = (int64_t)extent.size();
    return LBM_OK;
}

}  // extern "C"
