// Fused semi-Lagrangian streaming + collision for a compile-time order P.
//
// One thread block owns a tile of TEX x TEY x TEZ whole cells (one node per
// thread).  The 44 moving velocities are processed in rounds of G.  For each
// velocity the departure window of the tile is interpolated in three 1-D
// passes (z, then y, then x: Psi_i = Iz (x) Iy (x) Ix, Eqs. (8)-(9)):
//
//   z-pass  one task per (window column x, window column y, cell along z):
//           reads the column's source points straight from HBM/L2 (rows of x
//           are contiguous, so a wave's loads are coalesced), writes the P
//           interpolated points of the cell to LDS;
//   y-pass  one task per (window x, tile z, cell along y), LDS -> LDS;
//   x-pass  one task per (tile y, tile z, cell along x), LDS -> LDS in node
//           order; the node's thread then picks up its value.
//
// A task always produces the P outputs of one cell, so it reads each source
// point once and uses all P rows of the 1-D table: the table of a velocity
// is wave-uniform (tasks of one velocity are padded to whole waves) and is
// read with scalar loads.  The departure cell offsets of the P rows of a
// velocity and axis take two values o and o+1 (o_l is non-decreasing in l);
// rows l >= lstar use the upper cell.  The rest velocity is a plain copy.
// After the last round the 90 streamed values of the node are collided in
// registers (collision.h) and written once (x fastest, coalesced).
//
// Tiles are assigned so that each of the 8 XCDs (blocks are dealt to XCDs
// round-robin) walks a contiguous range of tiles in x-y-z order, keeping the
// halo of neighbouring tiles in that XCD's L2.
#include <hip/hip_runtime.h>

#include "collision.h"
#include "sllbm_internal.h"
#include "velset.h"

namespace sllbm {

template <int P, int TEX, int TEY, int TEZ>
struct TileShape {
    static constexpr int TX = TEX * P, TY = TEY * P, TZ = TEZ * P;
    static constexpr int NN = TX * TY * TZ;                          // nodes of a tile
    static constexpr int NT = (2 * NN + 63) / 64 * 64;               // two threads per node, whole waves
    static constexpr int WX = TX + P + 1, WY = TY + P + 1, WZ = TZ + P + 1;   // largest window
    static constexpr int round64(int n) { return (n + 63) / 64 * 64; }
    // tasks per (velocity, population), padded to whole waves
    static constexpr int ZT = WX * WY * TEZ, ZP = round64(ZT);
    static constexpr int YT = WX * TZ * TEY, YP = round64(YT);
    static constexpr int XT = TY * TZ * TEX, XP = round64(XT);
    static constexpr int BZ = TZ * WY * WX;                          // LDS slab of one (velocity, population)
    static constexpr int CY = TZ * TY * WX;
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int wrap(int x, int n)
{
    int r = x % n;
    return r < 0 ? r + n : r;
}

// tile index of this block: contiguous ranges of tiles per XCD
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int xcd = b & 7, slot = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// One velocity's P output rows from a column c[0..2P]:
//   out[l] = sum_k W[l][k] c[k + (l >= lstar ? P : 0)]
template <typename S, int P>
__device__ __forceinline__ void interp_cell(const S *__restrict__ W, int lstar, const S (&c)[2 * P + 1],
                                            S (&out)[P])
{
#pragma unroll
    for (int l = 0; l < P; ++l) {
        S acc = 0;
        if (l < lstar) {
#pragma unroll
            for (int k = 0; k <= P; ++k) acc = fma(W[l * (P + 1) + k], c[k], acc);
        } else {
#pragma unroll
            for (int k = 0; k <= P; ++k) acc = fma(W[l * (P + 1) + k], c[P + k], acc);
        }
        out[l] = acc;
    }
}

template <typename S, int P, int TEX, int TEY, int TEZ, int G, bool COLLIDE, int NTH, int MINB>
__global__ void __launch_bounds__(NTH, MINB)
    k_fused(Geometry geo, FusedTables<S> tab, CollisionParams cp, const S *__restrict__ in, S *__restrict__ out,
            S *__restrict__ pre_out)
{
    using TS = TileShape<P, TEX, TEY, TEZ>;
    constexpr int TX = TS::TX, TY = TS::TY, TZ = TS::TZ, NT = TS::NT, NN = TS::NN;
    constexpr int WX = TS::WX, WY = TS::WY, WZ = TS::WZ;
    constexpr int NROUND = (vs::Q - 1 + G - 1) / G;

    __shared__ S bz[G * 2 * TS::BZ];     // z-pass output; reused for the x-pass output
    __shared__ S cy[G * 2 * TS::CY];     // y-pass output
    __shared__ int xo[G][WX], yo[G][WY], zo[G][WZ];
    __shared__ int sh_lstar[G][3], sh_nrow[G][3];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const int64_t N = geo.nodes;

    // tile origin
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tcx = tile % geo.ntile[0];
    const int tcy = (tile / geo.ntile[0]) % geo.ntile[1];
    const int tcz = tile / (geo.ntile[0] * geo.ntile[1]);
    const int X0 = tcx * TX, Y0 = tcy * TY, Z0 = tcz * TZ;
    // node and population of this thread: lanes 2k (f) and 2k+1 (g) share a node
    const int nl = tid >> 1;
    const int pop = tid & 1;
    const int lx = nl % TX, ly = (nl / TX) % TY, lz = nl / (TX * TY);
    const bool valid = nl < NN && (X0 + lx < geo.N[0]) && (Y0 + ly < geo.N[1]) && (Z0 + lz < geo.N[2]);
    const int node = ((Z0 + lz) * geo.N[1] + (Y0 + ly)) * geo.N[0] + (X0 + lx);
    const S *__restrict__ my_in = in + static_cast<int64_t>(pop) * vs::Q * N;

    S v[vs::Q];
    v[0] = my_in[valid ? node : 0];          // the rest velocity does not move

#pragma unroll
    for (int rd = 0; rd < NROUND; ++rd) {
        const int vbase = 1 + rd * G;
        const int gcount = (vs::Q - vbase) < G ? (vs::Q - vbase) : G;

        // (a) global node offsets of the round's windows, per axis
        for (int e = tid; e < G * (WX + WY + WZ); e += NT) {
            const int gg = e / (WX + WY + WZ);
            const int r = e % (WX + WY + WZ);
            if (gg < gcount) {
                const int i = vbase + gg;
                if (r < WX) {
                    xo[gg][r] = wrap(X0 + tab.omin[i * 3 + 0] * P + r, geo.N[0]);
                } else if (r < WX + WY) {
                    const int w = r - WX;
                    yo[gg][w] = wrap(Y0 + tab.omin[i * 3 + 1] * P + w, geo.N[1]) * geo.N[0];
                } else {
                    const int w = r - WX - WY;
                    zo[gg][w] = wrap(Z0 + tab.omin[i * 3 + 2] * P + w, geo.N[2]) * geo.N[0] * geo.N[1];
                }
            }
            if (e < G * 3 && e / 3 < gcount) {
                const int i = vbase + e / 3, a = e % 3;
                const int ls = tab.lstar[i * 3 + a];
                sh_lstar[e / 3][a] = ls;
                sh_nrow[e / 3][a] = ls < P ? 2 * P + 1 : P + 1;
            }
        }
        __syncthreads();

        // (b) z-pass: columns straight from global memory
        for (int b = wave * 64; b < G * 2 * TS::ZP; b += NT) {
            const int gp = b / TS::ZP;                   // wave-uniform (velocity of the round, population)
            const int gg = gp >> 1, pp = gp & 1;
            const int t = b % TS::ZP + lane;
            if (gg < gcount && t < TS::ZT) {
                const int i = vbase + gg;
                const int wx = t % WX, wy = (t / WX) % WY, ez = t / (WX * WY);
                const S *__restrict__ src = in + static_cast<int64_t>(pp * vs::Q + i) * N;
                const int nrow = uniform(sh_nrow[gg][2]);
                const int base = xo[gg][wx] + yo[gg][wy];
                S c[2 * P + 1];
#pragma unroll
                for (int r = 0; r < 2 * P + 1; ++r) c[r] = (r < nrow) ? src[base + zo[gg][ez * P + r]] : S(0);
                S o[P];
                interp_cell<S, P>(tab.w + (i * 3 + 2) * P * (P + 1), uniform(sh_lstar[gg][2]), c, o);
                S *dst = bz + gp * TS::BZ;
#pragma unroll
                for (int l = 0; l < P; ++l) dst[((ez * P + l) * WY + wy) * WX + wx] = o[l];
            }
        }
        __syncthreads();

        // (c) y-pass
        for (int b = wave * 64; b < G * 2 * TS::YP; b += NT) {
            const int gp = b / TS::YP;
            const int gg = gp >> 1;
            const int t = b % TS::YP + lane;
            if (gg < gcount && t < TS::YT) {
                const int i = vbase + gg;
                const int wx = t % WX, tz = (t / WX) % TZ, ey = t / (WX * TZ);
                const int nrow = uniform(sh_nrow[gg][1]);
                const S *src = bz + gp * TS::BZ + (tz * WY + ey * P) * WX + wx;
                S c[2 * P + 1];
#pragma unroll
                for (int r = 0; r < 2 * P + 1; ++r) c[r] = (r < nrow) ? src[r * WX] : S(0);
                S o[P];
                interp_cell<S, P>(tab.w + (i * 3 + 1) * P * (P + 1), uniform(sh_lstar[gg][1]), c, o);
                S *dst = cy + gp * TS::CY + (tz * TY + ey * P) * WX + wx;
#pragma unroll
                for (int l = 0; l < P; ++l) dst[l * WX] = o[l];
            }
        }
        __syncthreads();

        // (d) x-pass, output in node order (into bz, free since the y-pass)
        for (int b = wave * 64; b < G * 2 * TS::XP; b += NT) {
            const int gp = b / TS::XP;
            const int gg = gp >> 1;
            const int t = b % TS::XP + lane;
            if (gg < gcount && t < TS::XT) {
                const int i = vbase + gg;
                const int ty = t % TY, tz = (t / TY) % TZ, ex = t / (TY * TZ);
                const int nrow = uniform(sh_nrow[gg][0]);
                const S *src = cy + gp * TS::CY + (tz * TY + ty) * WX + ex * P;
                S c[2 * P + 1];
#pragma unroll
                for (int r = 0; r < 2 * P + 1; ++r) c[r] = (r < nrow) ? src[r] : S(0);
                S o[P];
                interp_cell<S, P>(tab.w + (i * 3 + 0) * P * (P + 1), uniform(sh_lstar[gg][0]), c, o);
                S *dst = bz + gp * NN + (tz * TY + ty) * TX + ex * P;
#pragma unroll
                for (int l = 0; l < P; ++l) dst[l] = o[l];
            }
        }
        __syncthreads();

        // (e) this thread's streamed values
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
            const int i = 1 + rd * G + gg;
            if (i < vs::Q && nl < NN) v[i] = bz[(gg * 2 + pop) * NN + nl];
        }
        __syncthreads();
    }

    if (!valid) return;
    if (pre_out != nullptr) {
        S *dst = pre_out + static_cast<int64_t>(pop) * vs::Q * N + node;
#pragma unroll
        for (int i = 0; i < vs::Q; ++i) dst[static_cast<int64_t>(i) * N] = v[i];
    }
    if constexpr (COLLIDE) collide_half<S>(v, pop != 0, cp);
    S *dst = out + static_cast<int64_t>(pop) * vs::Q * N + node;
#pragma unroll
    for (int i = 0; i < vs::Q; ++i) dst[static_cast<int64_t>(i) * N] = v[i];
}

// ---------------------------------------------------------------------------
// Launch configuration per order: cells per tile (about 256 nodes), velocity
// rounds of G = 4, and the minimum blocks per CU that bounds registers.
// ---------------------------------------------------------------------------

template <typename S>
struct MinBlocks {
    static constexpr int value = 1;
};

template <typename S, int P, int TEX, int TEY, int TEZ>
static hipError_t launch_fused_t(const Geometry &g, const FusedTables<S> &t, const CollisionParams &cp,
                                 const S *in, S *out, S *pre, bool collide, hipStream_t st)
{
    using TS = TileShape<P, TEX, TEY, TEZ>;
    constexpr int G = 4;
    constexpr int MB = MinBlocks<S>::value;
    const int nb = g.ntile[0] * g.ntile[1] * g.ntile[2];
    if (collide)
        hipLaunchKernelGGL((k_fused<S, P, TEX, TEY, TEZ, G, true, TS::NT, MB>), dim3(nb), dim3(TS::NT), 0, st, g, t, cp, in,
                           out, pre);
    else
        hipLaunchKernelGGL((k_fused<S, P, TEX, TEY, TEZ, G, false, TS::NT, MB>), dim3(nb), dim3(TS::NT), 0, st, g, t, cp,
                           in, out, pre);
    return hipGetLastError();
}

void fused_tile(int p, int te[3])
{
    static const int table[7][3] = {{0, 0, 0}, {8, 8, 4}, {4, 4, 2}, {2, 2, 2}, {2, 2, 1}, {1, 1, 2}, {1, 1, 1}};
    for (int a = 0; a < 3; ++a) te[a] = table[p][a];
}

template <typename S>
hipError_t launch_fused(const Geometry &g, const FusedTables<S> &t, const CollisionParams &cp, const S *in, S *out,
                        S *pre, bool collide, hipStream_t st)
{
    switch (g.p) {
    case 1: return launch_fused_t<S, 1, 8, 8, 4>(g, t, cp, in, out, pre, collide, st);
    case 2: return launch_fused_t<S, 2, 4, 4, 2>(g, t, cp, in, out, pre, collide, st);
    case 3: return launch_fused_t<S, 3, 2, 2, 2>(g, t, cp, in, out, pre, collide, st);
    case 4: return launch_fused_t<S, 4, 2, 2, 1>(g, t, cp, in, out, pre, collide, st);
    case 5: return launch_fused_t<S, 5, 1, 1, 2>(g, t, cp, in, out, pre, collide, st);
    case 6: return launch_fused_t<S, 6, 1, 1, 1>(g, t, cp, in, out, pre, collide, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_fused<double>(const Geometry &, const FusedTables<double> &, const CollisionParams &,
                                         const double *, double *, double *, bool, hipStream_t);
template hipError_t launch_fused<float>(const Geometry &, const FusedTables<float> &, const CollisionParams &,
                                        const float *, float *, float *, bool, hipStream_t);

}  // namespace sllbm
