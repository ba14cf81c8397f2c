// Element order of the 3D node-major layout (tiles of 16 elements).
//
// Structured Kuhn-type meshes (every element a translate of one of a few
// shapes, one translate per cell of a regular grid): a tile holds 16
// translates of one shape in 16 consecutive cells, and the tiles of the
// shapes of a block of 16 cells are adjacent.  The neighbours of a tile
// across a local face are then again translates of one shape in consecutive
// cells with one common face-node permutation, so the neighbour-trace
// gathers of a wave touch a few cache lines per row instead of one per lane.
// Other meshes are ordered along a Morton curve of the element centroids.
#pragma once
#include <vector>

#include "mesh.hpp"

namespace dgh {

// slot2elem[slot] = element stored in that slot of the tiled layout, -1 for a
// padding slot; the number of slots is a multiple of 16.
void element_order(const Mesh& m, std::vector<int>& slot2elem, bool* structured);

}  // namespace dgh
