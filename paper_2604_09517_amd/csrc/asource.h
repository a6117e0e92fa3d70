// Where the FP64 matrix of a solve comes from (internal interface).
//
// Memory form: A (column-major, leading dimension lda) in HBM.
// Seeded form: the entries are regenerated from the seeded counter-based
// generator wherever they are needed (Sec. II-B counts scalable generation of
// the input matrix among what HPL-MxP requires):
//   a_ij = u(j n + i) = (mix(key + G (j n + i + 1)) >> 32) 2^-32 - 1/2,
//   key = mix(seed + G (stream + 1)), mix the SplitMix64 finaliser (Steele,
//   Lea & Flood, OOPSLA 2014), G = 0x9E3779B97F4A7C15;
// with, for the diagonally dominant variant, a_ii replaced by diag[i] (the
// sum of |a_ij| over j != i, computed once into a small device array).  The
// same values as mxlu_fill_uniform (+ mxlu_make_diag_dominant) writes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mxlu {

constexpr uint64_t kGenGolden = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t gen_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t gen_key(uint64_t seed, uint64_t stream_id) {
    return gen_mix(seed + kGenGolden * (stream_id + 1ull));
}

// u for the counter value z = key + G (idx + 1)
__host__ __device__ inline double gen_value(uint64_t z) {
    return (double)(gen_mix(z) >> 32) * 0x1p-32 - 0.5;
}

struct ASource {
    const double *A = nullptr;   // memory form when not null
    int64_t lda = 0;
    uint64_t key = 0;            // seeded form
    int64_t n = 0;
    const double *diag = nullptr;   // seeded, diagonally dominant: a_ii

    __host__ __device__ bool seeded() const { return A == nullptr; }

    __device__ __forceinline__ double at(int64_t i, int64_t j) const {
        if (A) return A[(size_t)i + (size_t)j * (size_t)lda];
        if (diag && i == j) return diag[i];
        return gen_value(key + kGenGolden * ((uint64_t)j * (uint64_t)n + (uint64_t)i + 1ull));
    }
};

}  // namespace mxlu
