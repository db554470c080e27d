// Fused single-sweep time step of the thermal multiphase LBM (one launch per step).
//
// Storage: structure of arrays, population k of set s (0 = N, 1 = g) at node (x, y, z) is
// buf[(s*Q + k)*plane + i], i = x + pitch*(y + ny*z), with x rows padded to the pitch.  Two
// buffers: a step reads `src` and writes `dst`.  Pull scheme: dst holds post-collision populations at the node where they were
// computed, so the state at time t is N_k(x, t) = src[k][x - c_k].
//
// Dependencies of one node update (sections 3-5): the force at x needs Phi on the 1-ring, the
// pressure work and latent heat need div u* (central differences), i.e. u* and hence F on
// the axis 1-ring, i.e. Phi on a 2-ring; conduction needs rho and T on the axis 1-ring.
//
// Work decomposition: a workgroup owns a TX x TY column of nodes and marches through a chunk
// of z planes (even chunks upward, odd chunks downward).  Per z iteration it runs three
// stages, with a barrier after M and after F (D3Q19's LDS rings are deep enough for the next
// iteration's M to overlap C; D2Q9 also has a barrier after C):
//   M: pull 2Q populations and form rho, j, E, T, p, Phi for plane zm on the tile plus a
//      2-node halo (LDS rings; Phi is kept on the whole region, rho, T and j only on the tile
//      plus a 1-node halo, the part that the force and the energy source read);
//   F: force and u* for the plane one behind zm on the tile plus a 1-node halo (LDS ring);
//   C: energy source, collisions and the store for the plane two behind zm, on the tile.
// D2Q9 runs the same code with a single plane (no z halo, no lag between the stages).
//
// Per-node quantities of the tile's own nodes (rho, j, E, p, F) stay in registers between the
// stages (T comes from its LDS ring); the moving populations of the own node are pulled again
// for the collision, or kept in an LDS stash.
//
// Arithmetic: moments, EOS, Phi and the force in FP64 (the force is a small difference of
// Phi^2 values); u*, the energy source and the collision in R; the rest populations close the
// mass and energy balances of the collision in FP64 over the stored values.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"
#include "lattice.hpp"
#include "node_math.hpp"
#include "physics.hpp"

namespace lbm {

// XCD-aware placement.  Consecutive workgroups are dealt round-robin to the 8 XCDs, and a launch
// larger than what the GPU holds at once runs in rounds of `resident` workgroups (dispatched in
// index order as earlier ones retire).  Workgroup b of round r = b / resident is given logical
// tile r * resident + (b % 8) * (resident / 8) + (b % resident) / 8, so that
//   - each round covers one contiguous run of tiles (x fastest, then y: a band of tile rows),
//     and every tile's neighbours inside the band run at the same time as it;
//   - each XCD owns a contiguous part of that run, and shared halos meet in its own L2.
// A last round shorter than `resident` is split the same way when it is a multiple of 8 and
// left in index order otherwise.  resident <= 0 means one round (the whole launch).
__device__ __forceinline__ int xcd_logical_block(int b, int nblk, int resident = 0)
{
    const int R = (resident > 0 && resident < nblk && (resident & 7) == 0) ? resident : nblk;
    const int base = (b / R) * R;
    const int cnt = min(R, nblk - base);
    if ((cnt & 7) != 0) return b;
    const int l = b - base;
    return base + (l & 7) * (cnt >> 3) + (l >> 3);
}

// Interior-first enumeration of a (W+2h) x (H+2h) region around a W x H tile: slots
// [0, W*H) are the tile row by row, then two full rows top and bottom, then h columns
// left and right of each middle row.  Returns region coordinates (rx, ry).
template <int W, int H, int HALO>
__device__ __forceinline__ void region_slot(int s, int& rx, int& ry)
{
    constexpr int RW = W + 2 * HALO;
    constexpr int RH = H + 2 * HALO;
    if (s < W * H) {
        rx = HALO + s % W;
        ry = HALO + s / W;
        return;
    }
    int r = s - W * H;
    if (r < HALO * RW) {
        rx = r % RW;
        ry = r / RW;
        return;
    }
    r -= HALO * RW;
    if (r < HALO * RW) {
        rx = r % RW;
        ry = RH - HALO + r / RW;
        return;
    }
    r -= HALO * RW;
    const int c = r % (2 * HALO);
    ry = HALO + r / (2 * HALO);
    rx = c < HALO ? c : RW - 2 * HALO + c;
}

// Access to population (set*Q + k) at node i of the two buffers, in one of two address forms
// (ADDR), both with 32-bit per-lane node offsets (a plane is under 4 GB):
//   0 (kAddrGlobal): global pointers with a scalar plane base;
//   1 (kAddrBuf):    one buffer resource per buffer (the state is under 4 GB): the node offset
//                    is the lane's 32-bit offset and the population's plane offset a scalar one.
// Buffer instructions take 32-bit offsets against a scalar base, where global loads carry a
// 64-bit address per lane; at 128^3 and 256^3 the buffer form measured 16-26% faster.  Stores
// are marked non-temporal (nothing in the step reads them back), so they do not displace the
// halo and re-read data the step still needs from L2.
enum AddrMode : int { kAddrGlobal = 0, kAddrBuf = 1 };

// Which extensions of the paper's periodic step an instantiation carries (see step_tile).
enum ExtMode : int { kExtNone = 0, kExtWalls = 1, kExtTable = 2 };

template <class S, int ADDR>
struct PopIO;

template <class S>
struct PopIO<S, kAddrGlobal> {
    const S* __restrict__ src;
    S* __restrict__ dst;
    long long plane;
    __device__ PopIO(const S* s, S* d, long long p, int) : src(s), dst(d), plane(p) {}
    // the plane base is uniform and the node offset a 32-bit unsigned byte offset (a plane is
    // under 4 GB), so a load is one global_load with a scalar base and a 32-bit lane offset
    __device__ __forceinline__ S load(int pk, int i) const
    {
        const char* base = (const char*)(src + (long long)pk * plane);
        return *(const S*)(base + (unsigned)i * (unsigned)sizeof(S));
    }
    __device__ __forceinline__ void store(int pk, int i, S v) const
    {
        char* base = (char*)(dst + (long long)pk * plane);
        __builtin_nontemporal_store(v, (S*)(base + (unsigned)i * (unsigned)sizeof(S)));
    }
};

// Raw buffer access of one FP32 or FP64 value; offsets are formed in unsigned 32-bit arithmetic
// by the callers (the host picks a form only where no offset wraps) and handed over as their
// bit pattern.  Bit 1 of the cache-policy operand is the non-temporal hint.
namespace bufio {
constexpr int kNT = 2;
constexpr int kWord3 = 0x00020000;
template <class S>
__device__ __forceinline__ S load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    const int v = __builtin_bit_cast(int, voff), so = __builtin_bit_cast(int, soff);
    if constexpr (sizeof(S) == 4)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, v, so, 0));
    else
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, v, so, 0));
}
template <class S>
__device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, S x)
{
    const int v = __builtin_bit_cast(int, voff), so = __builtin_bit_cast(int, soff);
    if constexpr (sizeof(S) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, so, kNT);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, x),
                                              r, v, so, kNT);
}
}  // namespace bufio

template <class S>
struct PopIO<S, kAddrBuf> {
    __amdgpu_buffer_rsrc_t rs, rd;
    unsigned plane_bytes;
    __device__ PopIO(const S* s, S* d, long long p, int npk)
    {
        const unsigned bytes = (unsigned)((unsigned long long)p * (unsigned)npk * sizeof(S));
        rs = __builtin_amdgcn_make_buffer_rsrc((void*)s, (short)0, __builtin_bit_cast(int, bytes), bufio::kWord3);
        rd = __builtin_amdgcn_make_buffer_rsrc((void*)d, (short)0, __builtin_bit_cast(int, bytes), bufio::kWord3);
        plane_bytes = (unsigned)((unsigned long long)p * sizeof(S));
    }
    __device__ __forceinline__ S load(int pk, int i) const
    {
        return bufio::load<S>(rs, (unsigned)i * (unsigned)sizeof(S), (unsigned)pk * plane_bytes);
    }
    __device__ __forceinline__ void store(int pk, int i, S v) const
    {
        bufio::store<S>(rd, (unsigned)i * (unsigned)sizeof(S), (unsigned)pk * plane_bytes, v);
    }
};

// How the collision treats the density populations: with tau = 1 the BGK term of N' no longer
// depends on N_k (N' = Neq(rho, u + du) exactly), so they need not be re-read.
enum NMode : int {
    kTauOne = 0,  // caller guarantees tau = 1 and BGK
    kTauAny = 1,  // BGK, re-read N_k
    kMrt = 2      // multiple relaxation times, re-read N_k
};

// LDS of one workgroup's tile: the rings of the three stages and the stash.  The caller owns it
// (one __shared__ object per kernel), so kernels that run several instantiations of the tile
// step share one allocation.
template <int Q, class S, class R, int TX, int TY, bool STASH>
struct TileLds {
    static constexpr int D = Lattice<Q>::D;
    static constexpr int NC = TX * TY;                           // tile
    static constexpr int EX = TX + 4, EY = TY + 4, NE = EX * EY;   // tile + 2-halo
    static constexpr int FX = TX + 2, FY = TY + 2, NF = FX * FY;   // tile + 1-halo
    static constexpr bool kStash = STASH && D == 3;
    // Planes held.  An iteration runs M(zm) | barrier | F(zm-1) | barrier | C(zm-2), and no
    // barrier closes it, so the next iteration's M(zm+1) may overlap a slower wave's C(zm-2):
    //   rho, T: C reads zm-3 .. zm-1 while M writes zm+1                 -> 5 planes
    //   Phi:    F reads zm-2 .. zm; the next write follows a barrier      -> 3 planes
    //   j:      F reads zm-1; M writes zm+1                              -> 2 planes
    //   u*x,y:  F writes zf, C reads zf-1; the next F follows a barrier   -> 2 planes
    //   u*z:    C reads zf-2 and zf                                      -> 3 planes
    // D2Q9 has one plane of each and a barrier closing the iteration.
    static constexpr int RING = (D == 3) ? 5 : 1;
    static constexpr int PR = (D == 3) ? 3 : 1;
    static constexpr int JR = (D == 3) ? 2 : 1;
    static constexpr int UH = (D == 3) ? 2 : 1;
    static constexpr int UZ = (D == 3) ? 3 : 1;

    double phi[PR][NE];          // Phi on the tile + 2-halo
    R rho[RING][NF];             // rho, T, j on the tile + 1-halo
    R T[RING][NF];
    R j[3][JR][NF];
    R uh[2][UH][NF];             // u*x, u*y
    R uz[UZ][NF];                // u*z
    S g[kStash ? 2 : 1][kStash ? Q - 1 : 1][kStash ? NC : 1];   // stash: own energy pulls
};

// One workgroup's share of a step: tile `lb` (x fastest, then y, then z chunk) of the box
// described by g.  Must be called by all NTH threads of the workgroup (NTH >= TX*TY).
//
// Work of a thread: the collision of tile node `tid` (tid < TX*TY); moment slot `tid` of the
// tile + 2-halo region and, when the region has more slots than threads, one of the remaining
// slots if the thread has no collision work (else slots are dealt round-robin); force slot
// `tid` (+ NTH ...) of the tile + 1-halo region.  Slots are numbered interior first, so a
// thread's first moment and force slots are its own collision node and the own node's
// moments and force stay in registers between the stages.
//
// EXT (kExtNone, kExtWalls, kExtTable): walls normal to z (Phys::walls: bounce-back pulls next
// to them, no stages on the planes
// beyond them, mirror values for the stages next to them) and the body force rho g; the
// instantiation without EXT is the periodic step with none of that code; kExtTable adds the
// tabulated equation of state (Phys::eos = 1) to everything kExtWalls has.
//
// PIPE: the pulls of the next plane's first moment slot are issued right after the current
// plane's sums, so they are in flight during the force and collision stages.  STASH (D3Q19):
// the collision does not pull its energy populations again; the moment stage already pulled
// them for the own node, and they wait in an LDS ring of two planes (each thread keeps its
// plane in registers until its collision has read the older plane of the same ring slot, then
// moves it there).  With the stash, the prefetch covers the density populations only (the
// energy pulls already occupy registers until the collision).
//
// RED: the step also forms the FP64 totals of the state it writes (mass, momentum, internal
// energy: what a reduction over the written buffer gives).  Each node sums its stored values
// in FP64 (mass and energy from the collision's own sums of the moving populations), the
// collision wavefronts sum their nodes by a butterfly of shuffles per plane and add that into
// their LDS entry (red_lds: 5 per wavefront), and the workgroup writes the sum of its
// wavefronts' entries to aux.partials[5 lb ...].  The fields are the same as without it.
template <int Q, class S, class R, int TX, int TY, int NTH, bool PIPE, int ADDR, int NMODE,
          bool STASH, int EXT, bool RED = false>
__device__ __forceinline__ void step_tile(TileLds<Q, S, R, TX, TY, STASH>& lds,
                                          const S* __restrict__ src, S* __restrict__ dst,
                                          const StepGeom& g, const Phys& ph, const StepAux& aux,
                                          const int lb, double* red_lds = nullptr)
{
    PopIO<S, ADDR> io(src, dst, g.plane, 2 * Q);
    using L = Lattice<Q>;
    constexpr int D = L::D;
    constexpr int ZH = (D == 3) ? 2 : 0;    // lead of the moment stage over the collision
    constexpr int NC = TX * TY;             // collision threads
    static_assert(NTH >= NC && NTH % 64 == 0, "one collision node per thread");
    using Lds = TileLds<Q, S, R, TX, TY, STASH>;
    constexpr int EX = Lds::EX, EY = Lds::EY, NE = Lds::NE;
    constexpr int FX = Lds::FX, NF = Lds::NF;
    constexpr bool kStash = Lds::kStash;
    // walls and body force exist only in the EXT instantiation (the periodic one has none of
    // their code)
    const bool has_walls = EXT != kExtNone && D == 3 && ph.walls != 0;
    constexpr bool kTable = EXT == kExtTable;
    constexpr bool kFiveRing = D == 3;   // no barrier closes an iteration
    constexpr int RING = Lds::RING, PR = Lds::PR, JR = Lds::JR, UH = Lds::UH, UZ = Lds::UZ;
    // moment slots beyond the first NTH go to threads without collision work when they fit
    constexpr int EXTRA = NE > NTH ? NE - NTH : 0;
    constexpr bool SPARE = EXTRA > 0 && EXTRA <= NTH - NC;
    constexpr int ME = SPARE ? 2 : (NE + NTH - 1) / NTH;
    constexpr int MF = (NF + NTH - 1) / NTH;

    auto& sPhi = lds.phi;
    auto& sRho = lds.rho;
    auto& sT = lds.T;
    auto& sJ = lds.j;
    auto& sUh = lds.uh;
    auto& sUz = lds.uz;
    auto& sG = lds.g;

    auto ring = [](int z) { return (z + 10) % RING; };        // z >= -10
    auto pring = [](int z) { return (z + 9) % PR; };          // z >= -9
    auto jring = [](int z) { return (z + 4) & (JR - 1); };
    auto uhring = [](int z) { return (z + 6) & (UH - 1); };
    auto uzring = [](int z) { return (z + 6) % UZ; };         // z >= -6

    const int tid = threadIdx.x;
    const int tix = lb % g.ntx;
    const int tiy = (lb / g.ntx) % g.nty;
    const int tiz = lb / (g.ntx * g.nty);
    const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * g.chunk;
    const int z1 = min(z0 + g.chunk, g.nz);
    const int nxy = g.pitch * g.ny;   // elements of one z plane (rows padded to the pitch)
    constexpr int kRedWaves = (NC + 63) / 64;   // wavefronts holding collision threads
    double nsum[RED ? 5 : 1];                   // the own node's totals (RED)
    if constexpr (RED) {
        if (tid < 5 * kRedWaves) red_lds[tid] = 0.0;
    }

    // moment-stage slots of this thread: LDS index on the 2-halo region, on the 1-halo region
    // (m_f < 0 outside it) and wrapped x / y*nx of (node - c) for c = +1, 0, -1 (index 1 - c);
    // m_e < 0 marks no slot
    int m_e[ME], m_f[ME];
    int m_x[ME][3], m_y[ME][3];
#pragma unroll
    for (int r = 0; r < ME; ++r) {
        int s = tid + r * NTH;
        if constexpr (SPARE) s = r == 0 ? tid : (tid >= NC ? NTH + (tid - NC) : NE);
        m_e[r] = -1;
        m_f[r] = -1;
        m_x[r][0] = m_x[r][1] = m_x[r][2] = 0;
        m_y[r][0] = m_y[r][1] = m_y[r][2] = 0;
        if (s < NE) {
            int ex, ey;
            region_slot<TX, TY, 2>(s, ex, ey);
            m_e[r] = ex + EX * ey;
            if (ex >= 1 && ex <= EX - 2 && ey >= 1 && ey <= EY - 2)
                m_f[r] = (ex - 1) + FX * (ey - 1);
            const int gx = wrap_index(x0 - 2 + ex, g.nx);
            const int gy = wrap_index(y0 - 2 + ey, g.ny);
            m_x[r][0] = wrap_index(gx - 1, g.nx);
            m_x[r][1] = gx;
            m_x[r][2] = wrap_index(gx + 1, g.nx);
            m_y[r][0] = wrap_index(gy - 1, g.ny) * g.pitch;
            m_y[r][1] = gy * g.pitch;
            m_y[r][2] = wrap_index(gy + 1, g.ny) * g.pitch;
        }
    }
    int f_e[MF], f_f[MF];
#pragma unroll
    for (int r = 0; r < MF; ++r) {
        const int s = tid + r * NTH;
        f_f[r] = -1;
        f_e[r] = 0;
        if (s < NF) {
            int fx, fy;
            region_slot<TX, TY, 1>(s, fx, fy);
            f_f[r] = fx + FX * fy;
            f_e[r] = (fx + 1) + EX * (fy + 1);   // the same node on the 2-halo region
        }
    }
    // this thread's own node (slot 0 of every stage)
    const int otx = tid % TX, oty = tid / TX;
    const int ox = x0 + otx, oy = y0 + oty;
    const bool own_in_xy = tid < NC && ox < g.nx && oy < g.ny;
    const int of = (otx + 1) + FX * (oty + 1);
    const int xs[3] = {m_x[0][0], m_x[0][1], m_x[0][2]};   // slot 0 is the own node
    const int ys[3] = {m_y[0][0], m_y[0][1], m_y[0][2]};

    const R omega_E = R(ph.omega_E);
    const R keepN = R(1.0 - ph.omega), keepG = R(1.0 - ph.omega_E);
    const R cond_half = R(ph.cond_half);
    const unsigned flags = ph.flags;
    const bool pseudo = (flags & kPseudo) != 0;
    // whether the collision re-reads the density populations (not needed with tau = 1)

    // register ring of the own node's moments: [0] newest plane ... [ZH] plane being collided
    // (T of that plane is read from its LDS ring)
    double o_rho[ZH + 1], o_E[ZH + 1];
    R o_jx[ZH + 1], o_jy[ZH + 1], o_jz[ZH + 1], o_p[ZH + 1];
    R fcur[3] = {R(0), R(0), R(0)}, fprev[3] = {R(0), R(0), R(0)};   // force, newest first
#pragma unroll
    for (int q = 0; q <= ZH; ++q) {
        o_rho[q] = 1.0; o_jx[q] = o_jy[q] = o_jz[q] = R(0);
        o_E[q] = 1.0; o_p[q] = R(0);
    }

    // pulls of moment slot r at plane zm: N_k(x, t) = N*_k(x - c_k), g likewise (`sets`: bit 0
    // the density populations, bit 1 the energy populations)
    auto load_slot = [&](int zm, int r, S (&pn)[Q], S (&pe)[Q], auto sets) {
        constexpr int SETS = decltype(sets)::value;
        // next to a wall, a direction pulled from beyond it takes the opposite population
        // leaving the node itself (bounce-back)
        const bool bb_lo = has_walls && zm == 0;
        const bool bb_hi = has_walls && zm == g.nz - 1;
        int zoff[3];
        if constexpr (D == 3) {
            zoff[0] = wrap_index(zm - 1, g.nz) * nxy;
            zoff[1] = wrap_index(zm, g.nz) * nxy;
            zoff[2] = wrap_index(zm + 1, g.nz) * nxy;
        } else {
            zoff[0] = zoff[1] = zoff[2] = 0;
        }
        // the nine (y, z) rows the pulls of this slot read from
        int row[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) row[a][b] = zoff[a] + m_y[r][b];
        auto pulls = [&](auto walled) {
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                int pk = k, off = row[1 - L::cz[k]][1 - L::cy[k]] + m_x[r][1 - L::cx[k]];
                if (decltype(walled)::value && L::cz[k] != 0) {
                    if ((L::cz[k] == 1 && bb_lo) || (L::cz[k] == -1 && bb_hi)) {
                        pk = opposite<Q>(k);
                        off = row[1][1] + m_x[r][1];
                    }
                }
                if constexpr (SETS & 1) pn[k] = io.load(pk, off);
                if constexpr (SETS & 2) pe[k] = io.load(Q + pk, off);
            }
        };
        if (bb_lo || bb_hi) pulls(std::true_type{});
        else pulls(std::false_type{});
    };

    // moments, EOS and Phi of moment slot r (plane in ring slots sm, sp, sj)
    auto moments = [&](int r, const S (&pn)[Q], const S (&pe)[Q], int sm, int sp, int sj) {
        double dr, djx, djy, djz, dE, dT, p, phi2;
        bool ok;
        moment_sums<Q>(pn, pe, dr, djx, djy, djz, dE);
        eos_phi2<kTable>(dr, dE, ph, flags, aux, dT, p, phi2, ok);
        if (!ok) {
            atomicOr(aux.err, 1);
            phi2 = 0.0;
        }
        sPhi[sp][m_e[r]] = sqrt(phi2);
        const int f = m_f[r];
        if (f >= 0) {
            sRho[sm][f] = R(dr);
            sT[sm][f] = R(dT);
            sJ[0][sj][f] = R(djx);
            sJ[1][sj][f] = R(djy);
            sJ[2][sj][f] = R(djz);
        }
        if (r == 0) {
#pragma unroll
            for (int q = ZH; q > 0; --q) {
                o_rho[q] = o_rho[q - 1]; o_jx[q] = o_jx[q - 1]; o_jy[q] = o_jy[q - 1];
                o_jz[q] = o_jz[q - 1]; o_E[q] = o_E[q - 1]; o_p[q] = o_p[q - 1];
            }
            o_rho[0] = dr; o_jx[0] = R(djx); o_jy[0] = R(djy); o_jz[0] = R(djz);
            o_E[0] = dE; o_p[0] = R(p);
        }
    };
    // the register ring advances over a plane beyond a wall too (no moments there)
    auto shift_own = [&]() {
#pragma unroll
        for (int q = ZH; q > 0; --q) {
            o_rho[q] = o_rho[q - 1]; o_jx[q] = o_jx[q - 1]; o_jy[q] = o_jy[q - 1];
            o_jz[q] = o_jz[q - 1]; o_E[q] = o_E[q - 1]; o_p[q] = o_p[q - 1];
        }
        o_rho[0] = 1.0; o_jx[0] = o_jy[0] = o_jz[0] = R(0);
        o_E[0] = 1.0; o_p[0] = R(0);
    };
    // planes beyond a wall: no pulls, moments or force; the stages next to the wall use the
    // mirror values instead
    auto beyond_wall = [&](int z) { return has_walls && (z < 0 || z >= g.nz); };
    const bool has_g = EXT != kExtNone && (ph.g[0] != 0.0 || ph.g[1] != 0.0 || ph.g[2] != 0.0);

    // the own node's pulls for the collision at plane zc (moving directions; the rest ones
    // follow from the balances): the density populations when the collision reads them
    // (with_n), the energy populations (with_e), from the LDS stash when there is one
    R pk_n[Q], pk_e[Q];
    auto load_own = [&](int zc, auto with_n, auto with_e) {
        constexpr bool WN = decltype(with_n)::value;
        constexpr bool WE = decltype(with_e)::value;
        if constexpr (kStash && WE) {
#pragma unroll
            for (int k = 1; k < Q; ++k) {
                pk_e[k] = R(sG[zc & 1][k - 1][tid]);
                if constexpr (NMODE == kTauOne) pk_n[k] = R(0);
            }
        }
        if constexpr (!WN && (kStash || !WE)) return;
        const bool bb_lo = has_walls && zc == 0;
        const bool bb_hi = has_walls && zc == g.nz - 1;
        const int zoc = wrap_index(zc, g.nz) * nxy;
        int zpull[3] = {zoc, zoc, zoc};
        if constexpr (D == 3) {
            zpull[0] = wrap_index(zc - 1, g.nz) * nxy;
            zpull[2] = wrap_index(zc + 1, g.nz) * nxy;
        }
        int row[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) row[a][b] = zpull[a] + ys[b];
        auto pulls = [&](auto walled) {
#pragma unroll
            for (int k = 1; k < Q; ++k) {
                int pk = k, off = row[1 - L::cz[k]][1 - L::cy[k]] + xs[1 - L::cx[k]];
                if (decltype(walled)::value && L::cz[k] != 0) {
                    if ((L::cz[k] == 1 && bb_lo) || (L::cz[k] == -1 && bb_hi)) {
                        pk = opposite<Q>(k);
                        off = row[1][1] + xs[1];
                    }
                }
                if constexpr (!kStash && WE) pk_e[k] = R(io.load(Q + pk, off));
                if constexpr (WN) pk_n[k] = R(io.load(pk, off));
                else pk_n[k] = R(0);
            }
        };
        if (bb_lo || bb_hi) pulls(std::true_type{});
        else pulls(std::false_type{});
    };
    using WithN = std::integral_constant<bool, NMODE != kTauOne>;
    // with the stash and a collision that reads N_k, those pulls are issued before the force
    // stage, whose LDS work then covers their latency (the stash read stays in the collision)
    constexpr bool kEarlyN = kStash && NMODE != kTauOne;

    // energy source and both collisions of the own node at plane zc; stores the result
    auto collide = [&](int zc, auto with_n) {
        constexpr bool WN = decltype(with_n)::value;
        const int sc = ring(zc), scm = ring(zc - 1), scp = ring(zc + 1);
        const int suc = uhring(zc), sucm = uzring(zc - 1), sucp = uzring(zc + 1);
        const int own = wrap_index(zc, g.nz) * nxy + oy * g.pitch + ox;

        const double rho_d = o_rho[ZH], E_d = o_E[ZH];
        const R rho = R(rho_d), E = R(E_d), T = sT[sc][of];
        const R p = o_p[ZH];
        const R inv_rho = R(1) / rho;
        const R ux = o_jx[ZH] * inv_rho, uy = o_jy[ZH] * inv_rho, uz = o_jz[ZH] * inv_rho;
        const R* Fo = (ZH > 0) ? fprev : fcur;

        // z neighbours of the node; beyond a wall: rho mirrored, u*_z mirrored with the
        // opposite sign, T mirrored or 2 T_wall - T (wall face held at T_wall)
        R uzm = R(0), uzp = R(0), rzm = R(0), rzp = R(0), tzm = R(0), tzp = R(0);
        if constexpr (D == 3) {
            uzm = sUz[sucm][of]; uzp = sUz[sucp][of];
            rzm = sRho[scm][of]; rzp = sRho[scp][of];
            tzm = sT[scm][of]; tzp = sT[scp][of];
            if (has_walls) {
                if (zc == 0) {
                    uzm = -sUz[uzring(zc)][of];
                    rzm = sRho[sc][of];
                    tzm = (ph.wall_heat & kWallTBottom) ? R(2.0 * ph.T_bottom) - T : T;
                }
                if (zc == g.nz - 1) {
                    uzp = -sUz[uzring(zc)][of];
                    rzp = sRho[sc][of];
                    tzp = (ph.wall_heat & kWallTTop) ? R(2.0 * ph.T_top) - T : T;
                }
            }
        }
        // div u* by central differences on each axis (section 6.2)
        R div = R(0.5) * (sUh[0][suc][of + 1] - sUh[0][suc][of - 1]) +
                R(0.5) * (sUh[1][suc][of + FX] - sUh[1][suc][of - FX]);
        if constexpr (D == 3) div += R(0.5) * (uzp - uzm);
        const R dE = energy_source<D, R, FX, kTable>(p, div, rho, T, rzm, sRho[sc], rzp, tzm, sT[sc], tzp,
                                             of, cond_half, flags, ph, aux);

        NodeCollision<Q, S, R, WN, NMODE == kMrt> c;
        c.setup(rho, E, ux, uy, uz, Fo[0], Fo[1], Fo[2], inv_rho, dE, keepN, keepG, omega_E,
                pseudo);
        c.mrt_prepare(pk_n, ph);
        if constexpr (RED) {
#pragma unroll
            for (int q = 1; q < 4; ++q) nsum[q] = 0.0;
        }
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int ko = opposite<Q>(k);
            if (ko < k) continue;
            S out[4];
            c.dir_pair(k, pk_n, pk_e, out);
            io.store(k, own, out[0]);
            io.store(Q + k, own, out[1]);
            io.store(ko, own, out[2]);
            io.store(Q + ko, own, out[3]);
            if constexpr (RED) {
                // direction ko = -k: the pair's momentum is c_k (N_k - N_ko)
                const double a = double(out[0]), b = double(out[2]);
                if (L::cx[k] != 0) nsum[1] += L::cx[k] > 0 ? a - b : b - a;
                if (L::cy[k] != 0) nsum[2] += L::cy[k] > 0 ? a - b : b - a;
                if (L::cz[k] != 0) nsum[3] += L::cz[k] > 0 ? a - b : b - a;
            }
        }
        S n0, g0;
        c.rest(rho_d, E_d, dE, n0, g0);
        io.store(0, own, n0);
        io.store(Q, own, g0);
        if constexpr (RED) {
            // the collision's own FP64 sums of the stored moving populations (which close the
            // node's balances through the rest populations), plus the stored rest ones
            nsum[0] = c.sumN + double(n0);
            nsum[4] = c.sumG + double(g0);
        }
    };

    // Chunks march upward and downward alternately, so the two chunks on either side of a
    // chunk boundary pull its halo planes at about the same time and the second pull finds
    // them in the caches.  The per-node arithmetic does not depend on the direction.
    const int niter = (z1 - z0) + 2 * ZH;
    const int dir = (tiz & 1) ? -1 : 1;
    const int zstart = dir > 0 ? z0 - ZH : z1 - 1 + ZH;
    S pn0[Q], pe0[Q];   // pulls of the first moment slot
    S held[kStash ? Q - 1 : 1];   // own node's energy pulls of plane zm, bound for the stash
    // populations prefetched: both sets, or with the stash (which holds the energy pulls in
    // registers until the collision) the density populations only
    using Both = std::integral_constant<int, 3>;
    using Ahead = std::integral_constant<int, kStash ? 1 : 3>;
    using Late = std::integral_constant<int, kStash ? 2 : 0>;
    if constexpr (PIPE) {
        if (m_e[0] >= 0 && !beyond_wall(zstart)) load_slot(zstart, 0, pn0, pe0, Ahead{});
    }
    for (int it = 0; it < niter; ++it) {
        const int zm = zstart + dir * it;   // moment stage; force at zm - dir, collision at zm - 2 dir
        const int zc = zm - dir * ZH;
        const bool collides = it >= 2 * ZH && own_in_xy;
        const int sm = ring(zm);
        const int sp = pring(zm);
        const int sj = jring(zm);

        // ---------------- M: moments, EOS, Phi on the tile + 2-halo of plane zm
        const bool ghost_m = beyond_wall(zm);
        if (m_e[0] >= 0) {
            if (!ghost_m) {
                if constexpr (!PIPE) load_slot(zm, 0, pn0, pe0, Both{});
                if constexpr (PIPE && Late::value != 0) load_slot(zm, 0, pn0, pe0, Late{});
                moments(0, pn0, pe0, sm, sp, sj);
                if constexpr (kStash) {
#pragma unroll
                    for (int k = 1; k < Q; ++k) held[k - 1] = pe0[k];
                }
            } else {
                shift_own();
            }
            if constexpr (PIPE) {
                if (it + 1 < niter && !beyond_wall(zm + dir)) load_slot(zm + dir, 0, pn0, pe0, Ahead{});
            }
        }
        if (!ghost_m) {
#pragma unroll
            for (int r = 1; r < ME; ++r) {
                if (m_e[r] < 0) continue;
                S pn[Q], pe[Q];
                load_slot(zm, r, pn, pe, Both{});
                moments(r, pn, pe, sm, sp, sj);
            }
        }
        __syncthreads();

        if constexpr (kEarlyN) {
            if (collides) load_own(zc, std::true_type{}, std::false_type{});
        }

        // ---------------- F: force and u* on the tile + 1-halo of plane zf = zm - dir ZH/2
        if (it >= ZH && beyond_wall(zm - dir * (ZH / 2))) {
            fprev[0] = fcur[0]; fprev[1] = fcur[1]; fprev[2] = fcur[2];
            fcur[0] = fcur[1] = fcur[2] = R(0);
        } else if (it >= ZH) {
            const int zf = zm - dir * (ZH / 2);
            const int sf = ring(zf), spf = pring(zf), spfm = pring(zf - 1), spfp = pring(zf + 1);
            const int sjf = jring(zf), suhf = uhring(zf), suzf = uzring(zf);
            // Phi beyond a wall is the mirror image: the plane itself
            const double* pm = (has_walls && zf == 0) ? sPhi[spf] : sPhi[spfm];
            const double* pp = (has_walls && zf == g.nz - 1) ? sPhi[spf] : sPhi[spfp];
#pragma unroll
            for (int r = 0; r < MF; ++r) {
                if (f_f[r] < 0) continue;
                const int e = f_e[r];
                const int f = f_f[r];
                double fx, fy, fz;
                force_at<Q, EX>(pm, sPhi[spf], pp, e, ph.A, ph.inv_alpha, fx, fy, fz);
                if (has_g) {   // body force rho g (eq:edm takes any force)
                    const double rf = double(sRho[sf][f]);
                    fx += rf * ph.g[0];
                    fy += rf * ph.g[1];
                    fz += rf * ph.g[2];
                }
                const R Fx = R(fx), Fy = R(fy), Fz = R(fz);
                const R inv_rho = R(1) / sRho[sf][f];
                sUh[0][suhf][f] = (sJ[0][sjf][f] + R(0.5) * Fx) * inv_rho;
                sUh[1][suhf][f] = (sJ[1][sjf][f] + R(0.5) * Fy) * inv_rho;
                if constexpr (D == 3) sUz[suzf][f] = (sJ[2][sjf][f] + R(0.5) * Fz) * inv_rho;
                if (r == 0) {
                    fprev[0] = fcur[0]; fprev[1] = fcur[1]; fprev[2] = fcur[2];
                    fcur[0] = Fx; fcur[1] = Fy; fcur[2] = Fz;
                }
            }
        }
        __syncthreads();

        // ---------------- C: energy source, collisions, store for plane zc = zm - dir ZH
        if constexpr (D == 2) {
            // one plane and no lag: the moment stage's pulls of slot 0 (the own node, the same
            // loads) are still in registers
            if (collides) {
#pragma unroll
                for (int k = 1; k < Q; ++k) {
                    pk_e[k] = R(pe0[k]);
                    pk_n[k] = NMODE != kTauOne ? R(pn0[k]) : R(0);
                }
            }
        } else if constexpr (kEarlyN) {
            if (collides) load_own(zc, std::false_type{}, std::true_type{});
        } else {
            if (collides) load_own(zc, WithN{}, std::true_type{});
        }
        if constexpr (kStash) {
            // plane zm takes the ring slot of plane zm - 2 dir, read just above by this same
            // thread (every thread touches only its own column of the stash)
            if (tid < NC) {
#pragma unroll
                for (int k = 1; k < Q; ++k) sG[zm & 1][k - 1][tid] = held[k - 1];
            }
        }
        if (collides) collide(zc, WithN{});
        if constexpr (RED) {
            // whole collision wavefronts (the condition is uniform over a wavefront)
            if (it >= 2 * ZH && tid < 64 * kRedWaves) {
                double v[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) v[q] = collides ? nsum[q] : 0.0;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) v[q] += __shfl_xor(v[q], off, 64);
                }
                if ((tid & 63) == 0) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) red_lds[(tid >> 6) * 5 + q] += v[q];
                }
            }
        }
        if constexpr (!kFiveRing) __syncthreads();
    }
    // A caller that runs several tiles in one workgroup reuses the LDS rings: the next tile's
    // moment stage must not overwrite planes that a slower wave's last collision still reads.
    if constexpr (kFiveRing) __syncthreads();
    if constexpr (RED) {
        // the barrier above (D3Q19) or the one closing the last iteration (D2Q9) orders the
        // wavefronts' last additions before these reads
        if (tid < 5) {
            double t = 0.0;
            for (int w = 0; w < kRedWaves; ++w) t += red_lds[w * 5 + tid];
            aux.partials[(long long)lb * 5 + tid] = t;
        }
    }
}

template <int Q, class S, class R, int TX, int TY, int NTH, bool PIPE, int ADDR, int NMODE,
          bool STASH, int EXT, bool RED = false>
__global__ void __launch_bounds__(NTH)
k_step(const S* __restrict__ src, S* __restrict__ dst, const StepGeom g, const Phys ph,
       const StepAux aux)
{
    __shared__ TileLds<Q, S, R, TX, TY, STASH> lds;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x, g.resident);
    if constexpr (RED) {
        __shared__ double red_lds[5 * ((TX * TY + 63) / 64)];
        step_tile<Q, S, R, TX, TY, NTH, PIPE, ADDR, NMODE, STASH, EXT, true>(lds, src, dst, g, ph, aux,
                                                                            lb, red_lds);
    } else {
        step_tile<Q, S, R, TX, TY, NTH, PIPE, ADDR, NMODE, STASH, EXT>(lds, src, dst, g, ph, aux, lb);
    }
}

}  // namespace lbm
