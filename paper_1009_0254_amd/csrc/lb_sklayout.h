// Layout of the structure-factor sampler's row spectra (private to the library).
#pragma once

#include <hip/hip_runtime.h>

namespace lbf {

// One mode's row spectrum of a replica is stored in chunks of SK_KG adjacent kx: [chunk][ky][SK_KG]
// complex values, so that the column pass reads each chunk's rows as one contiguous run (a
// plain [ky][nh] layout puts consecutive ky of one kx a row apart and every read in another
// HBM page).  nh = nx/2 + 1 is padded to a multiple of SK_KG.
constexpr int SK_KG = 16;
__host__ __device__ inline long long sk_nh_padded(int nx) { return (long long)((nx / 2 + SK_KG) / SK_KG) * SK_KG; }
__host__ __device__ inline long long sk_at(int ky, int kx, int ny)
{
    return ((long long)(kx / SK_KG) * ny + ky) * SK_KG + (kx % SK_KG);
}
// the same in 32-bit arithmetic (one replica's mode slot holds fewer than 2^32 elements)
__device__ inline unsigned sk_at32(int ky, int kx, int ny)
{
    return (((unsigned)kx / SK_KG) * (unsigned)ny + (unsigned)ky) * SK_KG + ((unsigned)kx % SK_KG);
}

}  // namespace lbf
