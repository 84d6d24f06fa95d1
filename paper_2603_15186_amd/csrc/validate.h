// Host-side checks of a scene before upload (no device code, no HIP runtime
// calls), kept in a translation unit of their own so that they can also be
// built with the host compiler's address and undefined-behaviour sanitizers.
#pragma once

#include <cstdint>
#include <string>

#include "hgs.h"

namespace hgs {

// Hierarchy levels the scene validation allows.
constexpr int kMaxLevels = 64;

// HGS_OK, or HGS_E_INVALID / HGS_E_BAD_HIERARCHY / HGS_E_UNSUPPORTED with a
// reason in *why.
hgs_status validate_scene(const hgs_gaussians* g, const hgs_hierarchy* h, std::string* why);

}  // namespace hgs
