// Host-only driver of the scene validation, built with the address and
// undefined-behaviour sanitizers: a hand-built three-level hierarchy, every
// malformed case the validation names, and seeded random corruptions of the
// hierarchy arrays (none of which may make the checks read outside the
// arrays they were given).  Prints "validate_driver: ok" and exits 0 when
// every expected status came back.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include "hgs.h"

namespace {

struct Scene {
    int64_t n = 0;
    int deg = 1;
    std::vector<float> means, scales, quats, opacity, sh, bound;
    std::vector<int32_t> parent, first_child, child_count;
    std::vector<int64_t> level_offset;
    int n_levels = 0;

    hgs_gaussians g() const {
        hgs_gaussians x{};
        x.n = n;
        x.sh_degree = deg;
        x.means = means.data();
        x.scales = scales.data();
        x.quats = quats.data();
        x.opacity = opacity.data();
        x.sh = sh.data();
        return x;
    }
    hgs_hierarchy h() const {
        hgs_hierarchy x{};
        x.n_nodes = n;
        x.parent = parent.data();
        x.first_child = first_child.data();
        x.child_count = child_count.data();
        x.bound = bound.data();
        x.n_levels = n_levels;
        x.level_offset = level_offset.data();
        return x;
    }
};

// One root, four children, three leaves under each child: 17 nodes.
Scene make_tree() {
    Scene s;
    s.n = 17;
    s.n_levels = 3;
    s.level_offset = {0, 1, 5, 17};
    const int K = (s.deg + 1) * (s.deg + 1);
    for (int64_t i = 0; i < s.n; ++i) {
        for (int j = 0; j < 3; ++j) {
            s.means.push_back(0.1f * (float)(i + j));
            s.scales.push_back(0.01f * (float)(j + 1));
        }
        s.quats.insert(s.quats.end(), {1.f, 0.f, 0.f, 0.f});
        s.opacity.push_back(0.5f);
        for (int k = 0; k < 3 * K; ++k) s.sh.push_back(0.01f * (float)k);
        s.bound.insert(s.bound.end(), {0.f, 0.f, 0.f, 1.f});
    }
    s.parent = {-1, 0, 0, 0, 0};
    s.first_child = {1, 5, 8, 11, 14};
    s.child_count = {4, 3, 3, 3, 3};
    for (int c = 0; c < 4; ++c)
        for (int j = 0; j < 3; ++j) s.parent.push_back(1 + c);
    for (int i = 5; i < 17; ++i) {
        s.first_child.push_back(0);
        s.child_count.push_back(0);
    }
    return s;
}

int failures = 0;

void expect(const char* what, hgs_status got, hgs_status want) {
    if (got != want) {
        std::printf("validate_driver: %s: status %d, expected %d\n", what, got, want);
        ++failures;
    }
}

hgs_status run(const Scene& s, bool with_h, std::string* msg = nullptr) {
    const hgs_gaussians g = s.g();
    const hgs_hierarchy h = s.h();
    char buf[256];
    const hgs_status st = hgs_validate_scene(&g, with_h ? &h : nullptr, buf, sizeof buf);
    if (msg) *msg = buf;
    return st;
}

}  // namespace

int main() {
    const float nan = std::numeric_limits<float>::quiet_NaN();
    const float inf = std::numeric_limits<float>::infinity();
    const Scene base = make_tree();
    expect("flat scene", run(base, false), HGS_OK);
    expect("hierarchy", run(base, true), HGS_OK);
    expect("null gaussians", hgs_validate_scene(nullptr, nullptr, nullptr, 0), HGS_E_INVALID);
    {
        char tiny[1];
        hgs_gaussians g = base.g();
        g.n = 0;
        expect("n = 0, one-byte message", hgs_validate_scene(&g, nullptr, tiny, 1), HGS_E_INVALID);
        if (tiny[0] != 0) { std::printf("validate_driver: message not terminated\n"); ++failures; }
        g = base.g();
        g.sh_degree = 4;
        expect("sh degree 4", hgs_validate_scene(&g, nullptr, nullptr, 0), HGS_E_INVALID);
        g = base.g();
        g.sh = nullptr;
        expect("null sh", hgs_validate_scene(&g, nullptr, nullptr, 0), HGS_E_INVALID);
    }
    struct FloatCase { const char* what; std::vector<float> Scene::*arr; size_t idx; float v; };
    const FloatCase fc[] = {
        {"scale 0", &Scene::scales, 4, 0.f}, {"scale NaN", &Scene::scales, 5, nan},
        {"mean inf", &Scene::means, 50, inf}, {"opacity 0", &Scene::opacity, 16, 0.f},
        {"opacity > 1", &Scene::opacity, 3, 1.5f}, {"quaternion NaN", &Scene::quats, 9, nan},
        {"sh NaN", &Scene::sh, 12 * 16 - 1, nan}, {"bound radius < 0", &Scene::bound, 4 * 16 + 3, -1.f},
        {"bound NaN", &Scene::bound, 0, nan},
    };
    for (const FloatCase& c : fc) {
        Scene s = base;
        (s.*(c.arr))[c.idx] = c.v;
        const bool bound = c.arr == &Scene::bound;
        expect(c.what, run(s, bound), HGS_E_INVALID);
    }
    {
        Scene s = base;
        for (int j = 0; j < 4; ++j) s.quats[4 * 7 + j] = 0.f;
        expect("zero quaternion", run(s, false), HGS_E_INVALID);
    }
    struct IntCase { const char* what; std::vector<int32_t> Scene::*arr; size_t idx; int32_t v; };
    const IntCase ic[] = {
        {"parent on the wrong level", &Scene::parent, 7, 6}, {"parent of a root", &Scene::parent, 0, 3},
        {"negative child count", &Scene::child_count, 2, -1}, {"first child shifted", &Scene::first_child, 2, 9},
        {"first child far away", &Scene::first_child, 3, 2000000000}, {"parent far away", &Scene::parent, 9, -2000000000},
        {"child count too large", &Scene::child_count, 4, 2000000000}, {"leaf with a child", &Scene::child_count, 16, 1},
        {"parent/child links disagree", &Scene::parent, 6, 2},
    };
    for (const IntCase& c : ic) {
        Scene s = base;
        (s.*(c.arr))[c.idx] = c.v;
        expect(c.what, run(s, true), HGS_E_BAD_HIERARCHY);
    }
    {
        Scene s = base;
        s.level_offset[3] = 16;
        expect("level offsets short of n", run(s, true), HGS_E_BAD_HIERARCHY);
        s = base;
        s.level_offset[2] = 1;
        expect("empty level", run(s, true), HGS_E_BAD_HIERARCHY);
        s = base;
        s.n_levels = 0;
        expect("no levels", run(s, true), HGS_E_BAD_HIERARCHY);
        s = base;
        s.n_levels = 65;
        s.level_offset.resize(66, 17);
        expect("too many levels", run(s, true), HGS_E_BAD_HIERARCHY);
    }
    // seeded random corruptions: any status but a crash or an invalid read
    std::mt19937_64 rng(12345);
    const int32_t picks[] = {-2147483647 - 1, -1, 0, 1, 4, 5, 16, 17, 18, 2147483647};
    int rejected = 0;
    for (int it = 0; it < 20000; ++it) {
        Scene s = base;
        const int nmut = 1 + (int)(rng() % 3);
        for (int m = 0; m < nmut; ++m) {
            std::vector<int32_t>* arrs[] = {&s.parent, &s.first_child, &s.child_count};
            std::vector<int32_t>& a = *arrs[rng() % 3];
            const size_t i = rng() % a.size();
            a[i] = (rng() & 1) ? picks[rng() % 10] : (int32_t)(rng() % 40) - 10;
        }
        const hgs_status st = run(s, true);
        if (st != HGS_OK && st != HGS_E_BAD_HIERARCHY) {
            std::printf("validate_driver: random case %d gave status %d\n", it, st);
            ++failures;
        }
        rejected += st != HGS_OK;
    }
    if (rejected < 10000) {
        std::printf("validate_driver: only %d of 20000 corruptions rejected\n", rejected);
        ++failures;
    }
    if (failures) return 1;
    std::printf("validate_driver: ok (%d of 20000 random corruptions rejected)\n", rejected);
    return 0;
}
