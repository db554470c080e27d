// Device kernels of the thermal multiphase LBM library and their launchers.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "lattice.hpp"
#include "physics.hpp"
#include "step_launch.hpp"

namespace lbm {

using step_launch::launch_step_t;

namespace {

__device__ __forceinline__ void node_xyz(long long i, int nx, int ny, int& x, int& y, int& z)
{
    x = (int)(i % nx);
    const long long r = i / nx;
    y = (int)(r % ny);
    z = (int)(r / ny);
}

__device__ __forceinline__ long long node_index(int x, int y, int z, int nx, int ny, int nz)
{
    return wrap_index(x, nx) + (long long)nx * (wrap_index(y, ny) + (long long)ny * wrap_index(z, nz));
}

// Element of node (x, y, z) (periodic wrap) in a population plane whose rows have the pitch.
__device__ __forceinline__ long long buf_index(int x, int y, int z, int nx, int ny, int nz, int pitch)
{
    return wrap_index(x, nx) + (long long)pitch * (wrap_index(y, ny) + (long long)ny * wrap_index(z, nz));
}

// Equilibrium initial state N_k = rho0 P_k(u0), g_k = rho0 c_v T0 P_k(u0) (eq:feq, section 4),
// stored in pull form: node y keeps, for direction k, the value belonging to node y + c_k.
template <int Q, class S>
__global__ void k_init(S* __restrict__ buf, const double* __restrict__ rho0,
                       const double* __restrict__ u0, const double* __restrict__ T0, int nx,
                       int ny, int nz, int pitch, long long plane, double c_v, int walls)
{
    using L = Lattice<Q>;
    const long long n = (long long)nx * ny * nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int x, y, z;
    node_xyz(i, nx, ny, x, y, z);
    const long long b = buf_index(x, y, z, nx, ny, nz, pitch);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        // population k stored at node i is pulled by node i + c_k; toward a wall, it is pulled
        // back by node i itself as the opposite direction
        long long j = node_index(x + L::cx[k], y + L::cy[k], z + L::cz[k], nx, ny, nz);
        int kd = k;
        if (walls && (z + L::cz[k] < 0 || z + L::cz[k] >= nz)) {
            j = i;
            kd = opposite<Q>(k);
        }
        const double rho = rho0[j];
        const double ux = u0[j], uy = u0[n + j], uz = u0[2 * n + j];
        const double E = rho * c_v * T0[j];
        const double cu = L::cx[kd] * ux + L::cy[kd] * uy + L::cz[kd] * uz;
        const double P = eq_poly(weight<Q>(kd), cu, ux * ux + uy * uy + uz * uz);
        buf[(long long)k * plane + b] = S(rho * P);
        buf[(long long)(Q + k) * plane + b] = S(E * P);
    }
}

// Moments of the current state in FP64: scratch = [rho | jx | jy | jz | E | T | Phi].
template <int Q, class S>
__global__ void k_moments_a(const S* __restrict__ buf, double* __restrict__ scr, int nx, int ny,
                            int nz, int pitch, long long plane, Phys ph,
                            const double* __restrict__ eos_p, int* err)
{
    using L = Lattice<Q>;
    const long long n = (long long)nx * ny * nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int x, y, z;
    node_xyz(i, nx, ny, x, y, z);
    double rho = 0, jx = 0, jy = 0, jz = 0, E = 0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        long long j = buf_index(x - L::cx[k], y - L::cy[k], z - L::cz[k], nx, ny, nz, pitch);
        int pk = k;
        if (ph.walls && (z - L::cz[k] < 0 || z - L::cz[k] >= nz)) {   // bounce-back at a wall
            pk = opposite<Q>(k);
            j = buf_index(x, y, z, nx, ny, nz, pitch);
        }
        const double nk = double(buf[(long long)pk * plane + j]);
        rho += nk;
        jx += L::cx[k] * nk;
        jy += L::cy[k] * nk;
        jz += L::cz[k] * nk;
        E += double(buf[(long long)(Q + pk) * plane + j]);
    }
    const double T = E / (rho * ph.c_v);
    const double Te = (ph.flags & kBaro) ? ph.T0_baro : T;
    bool inside = true;
    const double p = ph.eos ? ph.p_c * table_pressure(rho * ph.inv_rho_c, Te * ph.inv_T_c, ph, eos_p, inside)
                            : vdw_pressure(rho, Te, ph);
    double phi2 = rho * kTheta - p;
    if (!inside || !(phi2 > 0.0) || !(rho * ph.inv_rho_c < 3.0) || !(rho > 0.0) || !(E == E)) {
        atomicOr(err, 1);
        phi2 = 0.0;
    }
    scr[i] = rho;
    scr[n + i] = jx;
    scr[2 * n + i] = jy;
    scr[3 * n + i] = jz;
    scr[4 * n + i] = E;
    scr[5 * n + i] = T;
    scr[6 * n + i] = sqrt(phi2);
}

// u* = (j + F/2)/rho (eq:ustar) with the force of section 3 from the Phi field (mirrored beyond
// walls) plus the body force rho g; writes the requested output fields (any pointer may be
// null).
template <int Q>
__global__ void k_moments_b(const double* __restrict__ scr, int nx, int ny, int nz, Phys ph,
                            double* __restrict__ rho_o, double* __restrict__ us_o,
                            double* __restrict__ E_o, double* __restrict__ T_o)
{
    using L = Lattice<Q>;
    const long long n = (long long)nx * ny * nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int x, y, z;
    node_xyz(i, nx, ny, x, y, z);
    const double* Phi = scr + 6 * n;
    double s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
#pragma unroll
    for (int k = 1; k < Q; ++k) {
        int zz = z + L::cz[k];
        if (ph.walls) zz = zz < 0 ? -1 - zz : (zz >= nz ? 2 * nz - 1 - zz : zz);
        const double p = Phi[node_index(x + L::cx[k], y + L::cy[k], zz, nx, ny, nz)];
        const double G = force_coef<Q>(k);
        s1[0] += G * p * p * L::cx[k]; s1[1] += G * p * p * L::cy[k]; s1[2] += G * p * p * L::cz[k];
        s2[0] += G * p * L::cx[k]; s2[1] += G * p * L::cy[k]; s2[2] += G * p * L::cz[k];
    }
    const double rho = scr[i];
    if (rho_o) rho_o[i] = rho;
    if (E_o) E_o[i] = scr[4 * n + i];
    if (T_o) T_o[i] = scr[5 * n + i];
    if (us_o) {
        for (int a = 0; a < 3; ++a) {
            const double F = (ph.A * s1[a] + (1.0 - 2.0 * ph.A) * Phi[i] * s2[a]) * ph.inv_alpha +
                             rho * ph.g[a];
            us_o[a * n + i] = (scr[(1 + a) * n + i] + 0.5 * F) / rho;
        }
    }
}

constexpr int kReduceThreads = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block partial sums of mass, momentum and internal energy (FP64): per-thread grid-stride
// sums over 16-byte vectors of consecutive nodes (a population plane's rows are padded to
// whole 128-byte lines, so the plane's element count is a multiple of the vector and every
// plane starts aligned), 64-lane wavefront shuffles, then the waves in order.
template <int Q, class S>
__global__ void __launch_bounds__(kReduceThreads)
k_reduce_partial(const S* __restrict__ buf, long long n, long long plane, double* __restrict__ part)
{
    using L = Lattice<Q>;
    constexpr int VEC = 16 / (int)sizeof(S);
    typedef S V __attribute__((ext_vector_type(VEC)));
    const long long nv = n / VEC;
    double acc[5] = {0, 0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nv;
         i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const V a = *(const V*)(buf + (long long)k * plane + i * VEC);
            const V b = *(const V*)(buf + (long long)(Q + k) * plane + i * VEC);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const double nk = double(a[e]);
                acc[0] += nk;
                if (L::cx[k]) acc[1] += L::cx[k] * nk;
                if (L::cy[k]) acc[2] += L::cy[k] * nk;
                if (L::cz[k]) acc[3] += L::cz[k] * nk;
                acc[4] += double(b[e]);
            }
        }
    }
    __shared__ double wsum[kReduceThreads / 64][5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) wsum[wave][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double s = 0;
        for (int w = 0; w < kReduceThreads / 64; ++w) s += wsum[w][threadIdx.x];
        part[blockIdx.x * 5 + threadIdx.x] = s;
    }
}

// Sum of per-block partial totals (5 per block) in a fixed order: thread t adds the entries
// t, t + 256, ... (independent loads in flight together), then a fixed tree over the threads.
__global__ void __launch_bounds__(kReduceThreads)
k_sum_partials(const double* __restrict__ part, long long nblocks, double* __restrict__ out)
{
    __shared__ double red[5][kReduceThreads];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long b = threadIdx.x; b < nblocks; b += kReduceThreads) {
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q] += part[b * 5 + q];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) out[threadIdx.x] = red[threadIdx.x][0];
}

inline unsigned blocks_for(long long n, int threads)
{
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

// Launch shapes of the fused step.  Variant 0 is the default per (lattice, storage); the
// others are selected for tuning.  Tile shape, thread count and the order of the loads do not
// change the per-node arithmetic, so every variant gives bitwise-identical results.
// `per_cu` is the number of workgroups of the variant resident per compute unit (set by its
// registers and LDS); the automatic z chunk aims at about 256 * per_cu workgroups.
// FP32 variant 5 is the default launch with plain global addressing, which variant 0 falls
// back to for states of 4 GB and more; variant 7 is the same on 64 x 8 tiles (816 moment slots,
// the 48 beyond the 768 threads on threads without collision work), which lbm_init picks for
// such states where 64-wide tiles leave no more x columns idle than 32-wide ones.
struct TileShape { int tx, ty, threads; bool pipe, stash; int per_cu; };
static const TileShape kVariants19f[] = {
    {32, 16, 768, true, true, 1}, {32, 16, 768, false, true, 1}, {32, 16, 768, true, false, 1},
    {32, 16, 768, false, false, 1}, {32, 8, 512, false, false, 2}, {32, 16, 768, true, true, 1},
    {32, 8, 256, false, false, 2}, {64, 8, 768, false, true, 1}};
constexpr int kNumVariants19f = sizeof(kVariants19f) / sizeof(kVariants19f[0]);
// FP64 D3Q19: twice the registers and LDS per node
static const TileShape kVariants19d[] = {
    {32, 8, 512, false, true, 1}, {32, 8, 512, false, false, 1}, {32, 8, 256, false, false, 1},
    {32, 4, 128, false, false, 2}};
constexpr int kNumVariants19d = sizeof(kVariants19d) / sizeof(kVariants19d[0]);
// D2Q9 (one plane, no z march): the moment stage pulls the tile plus a 2-node halo, 1.69x the
// tile's nodes on 32x8 and 1.41x on 32x16
static const TileShape kVariants9[] = {
    {32, 8, 256, true, false, 2}, {32, 16, 512, true, false, 1}, {64, 8, 512, true, false, 1}};
constexpr int kNumVariants9 = sizeof(kVariants9) / sizeof(kVariants9[0]);

int step_variants(int Q, int storage_bytes)
{
    if (Q == 19) return storage_bytes == 4 ? kNumVariants19f : kNumVariants19d;
    return kNumVariants9;
}

void step_tile(int Q, int storage_bytes, int variant, int& tx, int& ty, int& per_cu)
{
    const TileShape* t = nullptr;
    if (Q == 19 && storage_bytes == 4 && variant >= 0 && variant < kNumVariants19f) t = &kVariants19f[variant];
    if (Q == 19 && storage_bytes == 8 && variant >= 0 && variant < kNumVariants19d) t = &kVariants19d[variant];
    if (Q == 9 && variant >= 0 && variant < kNumVariants9) t = &kVariants9[variant];
    if (t) {
        tx = t->tx;
        ty = t->ty;
        per_cu = t->per_cu;
        return;
    }
    tx = 32;
    ty = 8;
    per_cu = 2;
}

hipError_t launch_step(int Q, int storage_bytes, int variant, const void* src, void* dst,
                       const StepGeom& g, const Phys& ph, const StepAux& aux, hipStream_t st)
{
    if (Q == 19 && storage_bytes == 4) {
        switch (variant) {
        case 0: return launch_step_t<19, float, float, 32, 16, 768, true, true>(src, dst, g, ph, aux, st);
        case 1: return launch_step_t<19, float, float, 32, 16, 768, false, true>(src, dst, g, ph, aux, st);
        case 2: return launch_step_t<19, float, float, 32, 16, 768, true>(src, dst, g, ph, aux, st);
        case 3: return launch_step_t<19, float, float, 32, 16, 768, false>(src, dst, g, ph, aux, st);
        case 4: return launch_step_t<19, float, float, 32, 8, 512, false>(src, dst, g, ph, aux, st);
        case 5: return launch_step_t<19, float, float, 32, 16, 768, true, true, true>(src, dst, g, ph, aux, st);
        case 6: return launch_step_t<19, float, float, 32, 8, 256, false>(src, dst, g, ph, aux, st);
        case 7: return launch_step_t<19, float, float, 64, 8, 768, false, true, true>(src, dst, g, ph, aux, st);
        default: return hipErrorInvalidValue;
        }
    }
    if (Q == 19 && storage_bytes == 8) {
        switch (variant) {
        case 0: return launch_step_t<19, double, double, 32, 8, 512, false, true>(src, dst, g, ph, aux, st);
        case 1: return launch_step_t<19, double, double, 32, 8, 512, false>(src, dst, g, ph, aux, st);
        case 2: return launch_step_t<19, double, double, 32, 8, 256, false>(src, dst, g, ph, aux, st);
        case 3: return launch_step_t<19, double, double, 32, 4, 128, false>(src, dst, g, ph, aux, st);
        default: return hipErrorInvalidValue;
        }
    }
    // D2Q9 FP32 populations with FP64 arithmetic: in 2D the registers allow it, and FP32
    // arithmetic tripled the error of the stored-FP32 state alone (u* 9e-6 to 1e-5 against a
    // floor of 3e-6 on a 100-step slab)
    if (Q == 9 && storage_bytes == 4) {
        switch (variant) {
        case 0: return launch_step_t<9, float, double, 32, 8, 256, true>(src, dst, g, ph, aux, st);
        case 1: return launch_step_t<9, float, double, 32, 16, 512, true>(src, dst, g, ph, aux, st);
        case 2: return launch_step_t<9, float, double, 64, 8, 512, true>(src, dst, g, ph, aux, st);
        default: return hipErrorInvalidValue;
        }
    }
    if (Q == 9 && storage_bytes == 8) {
        switch (variant) {
        case 0: return launch_step_t<9, double, double, 32, 8, 256, false>(src, dst, g, ph, aux, st);
        case 1: return launch_step_t<9, double, double, 32, 16, 512, false>(src, dst, g, ph, aux, st);
        case 2: return launch_step_t<9, double, double, 64, 8, 512, false>(src, dst, g, ph, aux, st);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_init(int Q, int storage_bytes, void* buf, const double* rho0, const double* u0,
                       const double* T0, int nx, int ny, int nz, int pitch, long long plane,
                       double c_v, int walls, hipStream_t st)
{
    const long long n = (long long)nx * ny * nz;
    const dim3 grid(blocks_for(n, 256)), block(256);
    if (Q == 19 && storage_bytes == 4) hipLaunchKernelGGL((k_init<19, float>), grid, block, 0, st, (float*)buf, rho0, u0, T0, nx, ny, nz, pitch, plane, c_v, walls);
    else if (Q == 19 && storage_bytes == 8) hipLaunchKernelGGL((k_init<19, double>), grid, block, 0, st, (double*)buf, rho0, u0, T0, nx, ny, nz, pitch, plane, c_v, walls);
    else if (Q == 9 && storage_bytes == 4) hipLaunchKernelGGL((k_init<9, float>), grid, block, 0, st, (float*)buf, rho0, u0, T0, nx, ny, nz, pitch, plane, c_v, 0);
    else if (Q == 9 && storage_bytes == 8) hipLaunchKernelGGL((k_init<9, double>), grid, block, 0, st, (double*)buf, rho0, u0, T0, nx, ny, nz, pitch, plane, c_v, 0);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_moments(int Q, int storage_bytes, const void* buf, double* scratch, int nx, int ny,
                          int nz, int pitch, long long plane, const Phys& ph, const double* eos_p,
                          int* err, double* rho, double* us, double* E, double* T, hipStream_t st)
{
    const long long n = (long long)nx * ny * nz;
    const dim3 grid(blocks_for(n, 256)), block(256);
    if (Q == 19 && storage_bytes == 4) hipLaunchKernelGGL((k_moments_a<19, float>), grid, block, 0, st, (const float*)buf, scratch, nx, ny, nz, pitch, plane, ph, eos_p, err);
    else if (Q == 19 && storage_bytes == 8) hipLaunchKernelGGL((k_moments_a<19, double>), grid, block, 0, st, (const double*)buf, scratch, nx, ny, nz, pitch, plane, ph, eos_p, err);
    else if (Q == 9 && storage_bytes == 4) hipLaunchKernelGGL((k_moments_a<9, float>), grid, block, 0, st, (const float*)buf, scratch, nx, ny, nz, pitch, plane, ph, eos_p, err);
    else if (Q == 9 && storage_bytes == 8) hipLaunchKernelGGL((k_moments_a<9, double>), grid, block, 0, st, (const double*)buf, scratch, nx, ny, nz, pitch, plane, ph, eos_p, err);
    else return hipErrorInvalidValue;
    if (Q == 19) hipLaunchKernelGGL((k_moments_b<19>), grid, block, 0, st, scratch, nx, ny, nz, ph, rho, us, E, T);
    else hipLaunchKernelGGL((k_moments_b<9>), grid, block, 0, st, scratch, nx, ny, nz, ph, rho, us, E, T);
    return hipGetLastError();
}

int reduce_blocks(long long n)
{
    long long b = (n + kReduceThreads * 8 - 1) / (kReduceThreads * 8);
    return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

hipError_t launch_reduce(int Q, int storage_bytes, const void* buf, long long n, long long plane,
                         double* partials, int nblocks, double* out, hipStream_t st)
{
    const dim3 grid(nblocks), block(kReduceThreads);
    if (Q == 19 && storage_bytes == 4) hipLaunchKernelGGL((k_reduce_partial<19, float>), grid, block, 0, st, (const float*)buf, n, plane, partials);
    else if (Q == 19 && storage_bytes == 8) hipLaunchKernelGGL((k_reduce_partial<19, double>), grid, block, 0, st, (const double*)buf, n, plane, partials);
    else if (Q == 9 && storage_bytes == 4) hipLaunchKernelGGL((k_reduce_partial<9, float>), grid, block, 0, st, (const float*)buf, n, plane, partials);
    else if (Q == 9 && storage_bytes == 8) hipLaunchKernelGGL((k_reduce_partial<9, double>), grid, block, 0, st, (const double*)buf, n, plane, partials);
    else return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kReduceThreads), 0, st, (const double*)partials,
                       (long long)nblocks, out);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partials, long long nblocks, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kReduceThreads), 0, st, partials, nblocks, out);
    return hipGetLastError();
}

}  // namespace lbm
