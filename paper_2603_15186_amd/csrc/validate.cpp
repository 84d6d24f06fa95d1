// Scene validation (host only): the Gaussians' parameters must be finite and
// in range, and the hierarchy must be level-major with contiguous children
// one level down (the tree of Gaussians of NavGSim Sec. III-B as the C ABI
// takes it).
#include "validate.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace hgs {

namespace {

bool finite(float x) { return std::isfinite(x); }

}  // namespace

hgs_status validate_scene(const hgs_gaussians* g, const hgs_hierarchy* h, std::string* why) {
    auto bad = [&](hgs_status s, const std::string& m) {
        *why = m;
        return s;
    };
    if (!g) return bad(HGS_E_INVALID, "gaussians is NULL");
    if (g->n <= 0) return bad(HGS_E_INVALID, "n must be positive");
    if (g->n > (int64_t)0x7fffffff) return bad(HGS_E_UNSUPPORTED, "n exceeds 2^31-1");
    if (g->sh_degree < 0 || g->sh_degree > 3) return bad(HGS_E_INVALID, "sh_degree must be 0..3");
    if (!g->means || !g->scales || !g->quats || !g->opacity || !g->sh)
        return bad(HGS_E_INVALID, "a Gaussian array is NULL");
    const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
    for (int64_t i = 0; i < g->n; ++i) {
        for (int j = 0; j < 3; ++j) {
            if (!finite(g->means[3 * i + j])) return bad(HGS_E_INVALID, "mean of Gaussian " + std::to_string(i) + " is not finite");
            const float s = g->scales[3 * i + j];
            if (!(s > 0.f) || !finite(s)) return bad(HGS_E_INVALID, "scale of Gaussian " + std::to_string(i) + " is not a positive number");
        }
        float qq = 0.f;
        for (int j = 0; j < 4; ++j) {
            const float q = g->quats[4 * i + j];
            if (!finite(q)) return bad(HGS_E_INVALID, "quaternion of Gaussian " + std::to_string(i) + " is not finite");
            qq += q * q;
        }
        if (!(qq > 0.f)) return bad(HGS_E_INVALID, "quaternion of Gaussian " + std::to_string(i) + " is zero");
        const float o = g->opacity[i];
        if (!(o > 0.f && o <= 1.f)) return bad(HGS_E_INVALID, "opacity of Gaussian " + std::to_string(i) + " is outside (0, 1]");
        for (int k = 0; k < 3 * K; ++k)
            if (!finite(g->sh[(int64_t)3 * K * i + k])) return bad(HGS_E_INVALID, "SH of Gaussian " + std::to_string(i) + " is not finite");
    }
    if (!h) return HGS_OK;
    if (h->n_nodes != g->n) return bad(HGS_E_BAD_HIERARCHY, "n_nodes differs from the Gaussian count");
    if (!h->parent || !h->first_child || !h->child_count || !h->bound || !h->level_offset)
        return bad(HGS_E_BAD_HIERARCHY, "a hierarchy array is NULL");
    if (h->n_levels < 1 || h->n_levels > kMaxLevels)
        return bad(HGS_E_BAD_HIERARCHY, "n_levels must be 1.." + std::to_string(kMaxLevels));
    const int64_t n = h->n_nodes;
    if (h->level_offset[0] != 0 || h->level_offset[h->n_levels] != n)
        return bad(HGS_E_BAD_HIERARCHY, "level_offset must start at 0 and end at n_nodes");
    for (int L = 0; L < h->n_levels; ++L)
        if (h->level_offset[L + 1] <= h->level_offset[L]) return bad(HGS_E_BAD_HIERARCHY, "empty or decreasing level");
    for (int64_t k = 0; k < h->level_offset[1]; ++k)
        if (h->parent[k] != -1) return bad(HGS_E_BAD_HIERARCHY, "level 0 must hold only roots (parent -1)");
    int L = 0;
    for (int64_t k = 0; k < n; ++k) {
        while (k >= h->level_offset[L + 1]) ++L;
        const float* b = h->bound + 4 * k;
        if (!finite(b[0]) || !finite(b[1]) || !finite(b[2]) || !(b[3] >= 0.f) || !finite(b[3]))
            return bad(HGS_E_INVALID, "bound of node " + std::to_string(k) + " is invalid");
        if (L > 0) {
            const int32_t p = h->parent[k];
            if (p < h->level_offset[L - 1] || p >= h->level_offset[L])
                return bad(HGS_E_BAD_HIERARCHY, "parent of node " + std::to_string(k) + " is not on the level above");
            const int32_t f = h->first_child[p], c = h->child_count[p];
            if (k < f || k >= (int64_t)f + c)
                return bad(HGS_E_BAD_HIERARCHY, "node " + std::to_string(k) + " is outside its parent's child range");
        }
        const int32_t c = h->child_count[k];
        if (c < 0) return bad(HGS_E_BAD_HIERARCHY, "negative child_count at node " + std::to_string(k));
        if (c > 0) {
            if (L + 1 >= h->n_levels) return bad(HGS_E_BAD_HIERARCHY, "node on the last level has children");
            const int64_t f = h->first_child[k];
            if (f < h->level_offset[L + 1] || f + c > h->level_offset[L + 2])
                return bad(HGS_E_BAD_HIERARCHY, "children of node " + std::to_string(k) + " are not on the next level");
            if (k > h->level_offset[L] && h->child_count[k - 1] > 0 &&
                f != (int64_t)h->first_child[k - 1] + h->child_count[k - 1])
                return bad(HGS_E_BAD_HIERARCHY, "children are not contiguous in parent order at node " + std::to_string(k));
            for (int32_t j = 0; j < c; ++j)
                if (h->parent[f + j] != k) return bad(HGS_E_BAD_HIERARCHY, "child/parent links disagree at node " + std::to_string(k));
        }
    }
    return HGS_OK;
}

}  // namespace hgs

hgs_status hgs_validate_scene(const hgs_gaussians* g, const hgs_hierarchy* h, char* msg, int64_t msg_len) {
    std::string why;
    hgs_status s = hgs::validate_scene(g, h, &why);
    if (msg && msg_len > 0) {
        const size_t n = std::min<size_t>(why.size(), (size_t)msg_len - 1);
        std::memcpy(msg, why.data(), n);
        msg[n] = 0;
    }
    return s;
}
