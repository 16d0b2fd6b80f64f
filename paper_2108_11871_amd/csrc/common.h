// Launch-shape helpers shared by the kernel sources (internal header).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "fft_tile.h"

namespace ips {

constexpr int NT = 256;

inline bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Raise a kernel's dynamic LDS limit above 64 KiB when a launch needs it.
void set_lds(const void *fn, size_t bytes);

// Blocks of a kernel that fit on the device at once (0 if unknown).
int resident_blocks(const void *fn, int nthreads, size_t lds);

// Transforms longer than kLdsTwMaxN run in blocks of NTB threads whose tile
// holds one complex sequence without row padding (W = 2) and whose twiddles
// are read from the global table (the LDS holds only the tile).
constexpr int NTB = 1024;
constexpr int kLdsTwMaxN = 2048;

inline bool big_fft(int N) { return N > kLdsTwMaxN; }

template <typename T>
inline size_t tile_lds(int N, int W)
{
    if (big_fft(N)) return (size_t)N * W * sizeof(T);
    return (size_t)N * sizeof(cx<T>) + (size_t)N * (W + 1) * sizeof(T);
}

// Twiddle table of the transform type: LDS copy (short transforms) or the
// plan's global table (long ones).
template <typename T, bool BIG>
__device__ __forceinline__ const cx<T> *tw_table(unsigned char *smem, const cx<double> *twd,
                                                const cx<float> *twf)
{
    if constexpr (BIG) {
        if constexpr (sizeof(T) == sizeof(float))
            return reinterpret_cast<const cx<T> *>(twf);
        else
            return reinterpret_cast<const cx<T> *>(twd);
    } else {
        return reinterpret_cast<const cx<T> *>(smem);
    }
}

} // namespace ips
