// permute_shape.hpp -- how a permutation out[perm(x)] = in[x] maps onto the
// permute kernels, shared by their launcher and by the planner's time model
// of the TTGT lowering (Section 6, "Optimal permutation for TTGT").  Host
// code only.
#pragma once

#include <cstdint>
#include <vector>

namespace comet {

constexpr int kPermTile = 32;   // edge of the transpose kernel's tile

struct PermDim {
  int64_t ext, si, so;   // extent, stride in the input, stride in the output
};

enum PermKind {
  PERM_EMPTY,    // no element
  PERM_FLAT,     // one run contiguous on both sides (a vector walk when aligned)
  PERM_STREAM,   // both sides share their unit-stride dimension: rows copied along it
  PERM_TILED,    // the unit dimensions differ: 32 x 32 tiles staged through LDS
};

struct PermShape {
  PermKind kind = PERM_EMPTY;
  int64_t total = 0;             // elements
  std::vector<PermDim> d;        // extent-1 dimensions dropped, contiguous pairs fused
  int ui = -1, uo = -1;          // unit-stride dimension of the input, of the output
  // PERM_TILED: the input-contiguous group Gi (grown from ui along input
  // contiguity until it holds kPermTile elements), the output-contiguous
  // group Go, and the rest, each as indices into d
  std::vector<int> gi, go, rest;
  int64_t EI = 0, EO = 0;        // elements of Gi and of Go
};

// `reads` = false for a fill (the input is not read): only the output side
// decides the unit dimension then.
PermShape permute_shape(int ndim, const int64_t *ext, const int64_t *s_in, const int64_t *s_out, bool reads);

// Time model of one permute launch on MI355X, in microseconds: the bytes it
// moves (read and write, plus a read of the output when beta != 0) at the
// rate measured for its kernel class; a transpose whose tile is only partly
// filled (Gi or Go shorter than the tile edge) runs slower.
double permute_time_us(const PermShape &s, int elem_bytes, bool reads_out);

}  // namespace comet
