// Element-centric face types (per leaf and face f = 2d + s), shared by the host
// table builder and the kernels.
#pragma once

#include <cstdint>

namespace dgamr {
constexpr int32_t FT_WALL = 0;    // no-flux wall: mirror state
constexpr int32_t FT_CONF = 1;    // same-level neighbour nb[0]
constexpr int32_t FT_FINE = 2;    // this leaf is a fine side: nb[0] = coarse leaf, quadrant in bits 8..9
constexpr int32_t FT_COARSE = 3;  // this leaf is the coarse side: nb[0..3] = fine leaves by quadrant
// flag (bit 16) on a conforming face whose neighbour has a different background at
// the shared nodes: a periodic wrap along z (the background is a function of z, and
// otherwise both leaves compute bitwise-identical z at the face nodes)
constexpr int32_t FT_BG_NB = 1 << 16;
}  // namespace dgamr
