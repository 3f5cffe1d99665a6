// Host build of the library's pruning bound (prune_bound.h) for the CPU
// tests: the production threshold, and the same formula with its margins
// given by the caller (a margin of 1 removes that safeguard).
#include "../../paper_2606_06255_amd/csrc/prune_bound.h"

extern "C" float shim_prune_threshold(float R, float dv) { return rfps::prune_threshold(R, dv); }

extern "C" float shim_prune_threshold_with(float R, float dv, float inner, float outer)
{
    return rfps::prune_threshold_with(R, dv, inner, outer);
}
