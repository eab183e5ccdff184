// Status bits that the update-step kernels raise in Result::status, and the
// C-ABI status each maps to.  Host-only and free of HIP, so the mapping is
// also compiled and checked on the host by itself.
#pragma once

#include "../../include/hsma.h"

namespace hsma {

enum : int {
    RS_BAD_INPUT = 1,     // non-finite position or charge
    RS_OUT_OF_BOX = 2,    // grounded-cube or slab position on or outside a wall
    RS_NOT_NEUTRAL = 4,   // periodic or slab system with net charge
    RS_COINCIDENT = 8,    // two charges at the same position
    RS_NONFINITE = 16     // energy, a potential or a force came out non-finite
};

// The status of a finished step from its bits: errors in the input first
// (they explain a non-finite result), then a non-finite result.  *msg gets a
// message for the caller's last-error text (nullptr for HSMA_OK).
inline hsma_status status_of_bits(int bits, const char** msg) {
    struct Row { int bit; hsma_status st; const char* text; };
    static const Row rows[] = {
        {RS_BAD_INPUT, HSMA_E_INVALID, "non-finite position or charge"},
        {RS_OUT_OF_BOX, HSMA_E_OUT_OF_BOX, "position on or outside a grounded wall"},
        {RS_NOT_NEUTRAL, HSMA_E_NOT_NEUTRAL, "periodic/slab system is not neutral"},
        {RS_COINCIDENT, HSMA_E_COINCIDENT, "two charges at the same position"},
        {RS_NONFINITE, HSMA_E_NONFINITE,
         "non-finite energy, potential or force (charges closer than the arithmetic resolves)"},
    };
    for (const Row& r : rows)
        if (bits & r.bit) {
            if (msg) *msg = r.text;
            return r.st;
        }
    if (msg) *msg = nullptr;
    return HSMA_OK;
}

}  // namespace hsma
