// checkpoint.h -- header of a checkpoint blob (ij_save_state, ij3_save_state)
// and the hash that ties a blob to its wall mask.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace ij_ckpt {

// 64 bytes, followed by `payload` bytes of the distribution buffer as stored
struct StateHeader {
    char magic[8];
    int64_t nx, ny, nz, pitch, t;
    uint64_t wall_hash, payload;
};
static_assert(sizeof(StateHeader) == 64, "checkpoint header is 64 bytes");

// FNV-1a of a byte array
inline uint64_t fnv1a(const uint8_t* p, size_t n)
{
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
    return h;
}

}  // namespace ij_ckpt
