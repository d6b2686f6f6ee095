// lattice.hpp -- canonical velocity sets of the library (host and device).
//
// D2Q9 and D3Q27 are the tensor products of the three-point Gauss-Hermite rule (nodes 0 and
// +-sqrt(3), weights 2/3 and 1/6) rescaled to c = cs v with cs^2 = 1/3; D3Q19 drops the eight
// body diagonals and keeps the weights 1/3, 1/18, 1/36 fixed by isotropy (App. C).
//
// Canonical order: the rest velocity first, then opposite pairs (c_{2p-1}, c_{2p} = -c_{2p-1})
// for p = 1 .. NP: the three axes, then the face diagonals, then the body diagonals. Kernels
// work pair by pair, so every per-direction quantity that is even in c is stored once per pair.
#pragma once

#include <cstdint>

namespace lbm {

enum LatticeId : int { kD2Q9 = 0, kD3Q19 = 1, kD3Q27 = 2 };

// Positive member of each pair; pair p (1-based) is directions 2p-1 (+c) and 2p (-c).
// Weights are integers over 216 (the common denominator of 4/9, 1/9, 1/36, 8/27, 2/27,
// 1/54, 1/216, 1/3, 1/18).
struct PairRow {
    int8_t cx, cy, cz;
};

template <int LAT> struct Lattice;

template <> struct Lattice<kD2Q9> {
    static constexpr int Q = 9, D = 2, NP = 4;
    static constexpr int w_rest = 96;  // 4/9
    __host__ __device__ static constexpr PairRow pair(int p)
    {
        constexpr PairRow t[4] = {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {1, -1, 0}};
        return t[p];
    }
    __host__ __device__ static constexpr int w_pair(int p)
    {
        constexpr int t[4] = {24, 24, 6, 6};  // 1/9, 1/9, 1/36, 1/36
        return t[p];
    }
};

template <> struct Lattice<kD3Q19> {
    static constexpr int Q = 19, D = 3, NP = 9;
    static constexpr int w_rest = 72;  // 1/3
    __host__ __device__ static constexpr PairRow pair(int p)
    {
        constexpr PairRow t[9] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
                                  {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};
        return t[p];
    }
    __host__ __device__ static constexpr int w_pair(int p)
    {
        constexpr int t[9] = {12, 12, 12, 6, 6, 6, 6, 6, 6};  // 1/18 axes, 1/36 face diagonals
        return t[p];
    }
};

template <> struct Lattice<kD3Q27> {
    static constexpr int Q = 27, D = 3, NP = 13;
    static constexpr int w_rest = 64;  // 8/27
    __host__ __device__ static constexpr PairRow pair(int p)
    {
        constexpr PairRow t[13] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {1, 1, 0}, {1, -1, 0},
                                   {1, 0, 1},  {1, 0, -1}, {0, 1, 1},  {0, 1, -1}, {1, 1, 1},
                                   {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};
        return t[p];
    }
    __host__ __device__ static constexpr int w_pair(int p)
    {
        // 2/27 axes, 1/54 face diagonals, 1/216 body diagonals
        constexpr int t[13] = {16, 16, 16, 4, 4, 4, 4, 4, 4, 1, 1, 1, 1};
        return t[p];
    }
};

constexpr int kWeightDen = 216;
constexpr int kMaxQ = 27;
constexpr int kMaxPairs = 13;

}  // namespace lbm
