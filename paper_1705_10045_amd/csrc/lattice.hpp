// Velocity sets of the thermal multiphase LBM (section 2: D2Q9 and D3Q19, theta = 1/3) and the
// coefficients of the isotropic pseudopotential force (section 3: G = 1 for nearest neighbours,
// 1/4 (D2Q9) or 1/2 (D3Q19) for next-nearest, alpha = 3/2 or 3).
//
// Ordering is chosen for the z-marching kernel: the first nine directions are the in-plane set
// (identical to D2Q9), then the five directions with c_z = +1 (whose pulls read plane z-1),
// then their opposites with c_z = -1 (reading plane z+1).
#pragma once

namespace lbm {

template <int Q>
struct Lattice;

template <>
struct Lattice<9> {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w_rest = 4.0 / 9.0, w_axis = 1.0 / 9.0, w_diag = 1.0 / 36.0;
    static constexpr double G_diag = 0.25;
    static constexpr double alpha = 1.5;
};

template <>
struct Lattice<19> {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 1, -1, 0, 0, 0, -1, 1, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 1, -1, -1, 1, 0, 0, 0, 1, -1, 0, 0, 0, -1, 1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1};
    static constexpr double w_rest = 1.0 / 3.0, w_axis = 1.0 / 18.0, w_diag = 1.0 / 36.0;
    static constexpr double G_diag = 0.5;
    static constexpr double alpha = 3.0;
};

// Weight and force coefficient of direction k from |c_k|^2.
template <int Q>
__host__ __device__ constexpr int norm2(int k)
{
    return Lattice<Q>::cx[k] * Lattice<Q>::cx[k] + Lattice<Q>::cy[k] * Lattice<Q>::cy[k] +
           Lattice<Q>::cz[k] * Lattice<Q>::cz[k];
}

template <int Q>
__host__ __device__ constexpr double weight(int k)
{
    return norm2<Q>(k) == 0 ? Lattice<Q>::w_rest
                            : (norm2<Q>(k) == 1 ? Lattice<Q>::w_axis : Lattice<Q>::w_diag);
}

// Index of the direction opposite to k (c_opp = -c_k).
template <int Q>
__host__ __device__ constexpr int opposite(int k)
{
    for (int j = 0; j < Q; ++j)
        if (Lattice<Q>::cx[j] == -Lattice<Q>::cx[k] && Lattice<Q>::cy[j] == -Lattice<Q>::cy[k] &&
            Lattice<Q>::cz[j] == -Lattice<Q>::cz[k])
            return j;
    return -1;
}

template <int Q>
__host__ __device__ constexpr double force_coef(int k)
{
    return norm2<Q>(k) == 0 ? 0.0 : (norm2<Q>(k) == 1 ? 1.0 : Lattice<Q>::G_diag);
}

}  // namespace lbm
