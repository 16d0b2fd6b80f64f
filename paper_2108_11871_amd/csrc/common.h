// Launch-shape helpers shared by the kernel sources (internal header).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fft_tile.h"

namespace ips {

constexpr int NT = 256;

inline bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// The tile helpers address a tile with 32-bit offsets r * rsd + c * csd built
// from 24-bit multiplies (toff): strides below 2^23, extent below 2^31.
inline bool tile_strides_ok(int64_t nrows, int64_t rsd, int64_t ncols, int64_t csd)
{
    const int64_t lim24 = (int64_t)1 << 23, lim31 = ((int64_t)1 << 31) - 1;
    const int64_t ar = rsd < 0 ? -rsd : rsd, ac = csd < 0 ? -csd : csd;
    return ar < lim24 && ac < lim24 && nrows < lim24 && ncols < lim24 && nrows * ar + ncols * ac < lim31;
}

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
