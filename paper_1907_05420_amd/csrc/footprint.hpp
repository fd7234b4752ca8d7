// Workspace constants shared by the context and the planning query.
#pragma once
#include <cstddef>
#include <cstdint>

#include "../../include/kkt.h"
#include "symbolic.hpp"

namespace kkt {

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// restart length of the flexible GMRES refinement
constexpr int KRYLOV_M = 8;
constexpr int KRYLOV_PART = 512;  // partial sums per Krylov reduction
inline bool uses_krylov(const kkt_options &o) { return o.refine_method == KKT_REFINE_FGMRES && o.refine_max > 0; }

// Device bytes a context with options `o` holds after kkt_analyze of `s` and
// a solve with nrhs right-hand sides: the context's own allocation code run
// without a device (every allocation and upload only counted), so that the
// planning query and kkt_footprint agree byte for byte. Returns a KKT_ status.
int plan_device_bytes(const kkt_structure *s, const kkt_options &o, int64_t nrhs, size_t *bytes);

}  // namespace kkt
