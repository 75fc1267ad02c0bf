// Lookup tables of the GPU path, built by construction (never copied from the
// CPU oracle, which derives the same mapping from transition counts).
#include "lbpf_internal.h"

namespace lbpf {

// Uniform-59 mapping: the uniform 8-bit patterns are all-zeros, all-ones and
// the eight rotations of every run of L consecutive ones (1 <= L <= 7), 58 in
// all. They take bins 0..57 in increasing numeric order; every other code
// shares bin 58.
void build_uniform59(uint8_t out[256]) {
    bool uniform[256] = {};
    uniform[0] = uniform[255] = true;
    for (int len = 1; len <= 7; ++len) {
        const unsigned run = (1u << len) - 1u;
        for (int r = 0; r < 8; ++r) uniform[((run << r) | (run >> (8 - r))) & 0xFFu] = true;
    }
    int rank = 0;
    for (int c = 0; c < 256; ++c) out[c] = uniform[c] ? (uint8_t)rank++ : (uint8_t)58;
}

// The fast feature kernel produces, per pixel and channel, a byte whose bit p
// is set when neighbour p is BELOW the centre (the complement of the LBP bit
// of Eq. 2). This table maps such a byte straight to the histogram bin.
void build_comparison_lut(const uint8_t bin[256], uint8_t below[256]) {
    for (int i = 0; i < 256; ++i) below[i] = bin[~(unsigned)i & 0xFFu];
}

}  // namespace lbpf
