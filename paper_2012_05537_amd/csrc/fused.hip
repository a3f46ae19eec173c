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

#include <algorithm>
#include <cmath>
#include <type_traits>

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

// walk index of this block: contiguous ranges of the walk per XCD
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int xcd = b & 7, slot = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// Tile coordinates of walk index L.  The walk visits bricks of
// brick[0] x brick[1] x brick[2] tiles (smaller at the far edges) in z-slab,
// y-row, x order, and the tiles of a brick in x-y-z order, so the blocks one
// XCD holds at a time cover a compact brick whose halo is shared in L2.
__device__ __forceinline__ void walk_tile(int L, const Geometry &g, int &tx, int &ty, int &tz)
{
    const int nx = g.ntile[0], ny = g.ntile[1], nz = g.ntile[2];
    const int BX = g.brick[0], BY = g.brick[1], BZ = g.brick[2];
    const int slab = L / (nx * ny * BZ);
    const int z0 = slab * BZ, bzs = min(BZ, nz - z0);
    int r = L - slab * nx * ny * BZ;
    const int row = r / (nx * BY * bzs);
    const int y0 = row * BY, bys = min(BY, ny - y0);
    r -= row * nx * BY * bzs;
    const int bxi = r / (BX * bys * bzs);
    const int x0 = bxi * BX, bxs = min(BX, nx - x0);
    r -= bxi * BX * bys * bzs;
    tx = x0 + r % bxs;
    ty = y0 + (r / bxs) % bys;
    tz = z0 + r / (bxs * bys);
}

// Per-block state of the fused kernel.  A block has 8 waves; in each round
// wave w streams velocity 1 + 4*round + w/2 of population w%2 through its own
// z-, y- and x-passes in wave-private LDS, so waves proceed independently;
// one block barrier per round publishes the node-ordered results
// (double-buffered) to the threads that own the nodes.
//
// Source-cell grouping.  Along an axis, node n of the tile (row l = n mod P)
// reads cell floor(n/P) + o_l, with o_l = omin for l < lstar and omin + 1
// otherwise.  Equivalently the nodes n = g*P + lstar + j, j = 0..P-1, all
// read cell g + omin + 1 with row l = (lstar + j) mod P.  A pass therefore
// works per (column, group g): it loads the P+1 points of one source cell,
// and writes up to P outputs at an offset that is uniform across the wave
// (lstar is a property of the velocity), with no per-lane selection.
template <typename S, int P, int TEX, int TEY, int TEZ>
struct Fused {
    using TS = TileShape<P, TEX, TEY, TEZ>;
    static constexpr int G = 4;                                     // velocities per round
    static constexpr int NT = 512;                                  // 8 waves = G velocities x 2 populations
    static constexpr int TX = TS::TX, TY = TS::TY, TZ = TS::TZ, NN = TS::NN;
    static constexpr int WX = TS::WX, WY = TS::WY, WZ = TS::WZ;
    static_assert(2 * NN <= NT, "tile too large for the block");
    static constexpr int NROUND = (vs::Q - 1) / G;
    static constexpr int ZC = WX * WY, ZK = (ZC + 63) / 64;         // z columns per wave, per lane
    static constexpr int YC = WX * TZ, YK = (YC + 63) / 64;
    static constexpr int XC = TY * TZ, XK = (XC + 63) / 64;
    static constexpr int RS = 2 * TX + 1;                           // padded row of dx (both populations)

    struct Smem {
        S bz[2 * G][TZ * WY * WX];          // wave-private z-pass output
        S cy[2 * G][TZ * TY * WX];          // wave-private y-pass output
        S dx[2][G][TZ * TY * RS];           // node-ordered streamed values, two buffers
        int xo[NROUND][G][WX];              // global node offsets of the windows
        int yo[NROUND][G][WY];
        int zo[NROUND][G][WZ];
    };

    using Col = S[TEZ + 1][ZK][P + 1];

    // loads of this wave's z-columns of round rd: group g reads window rows (g+1)P .. (g+1)P + P
    static __device__ __forceinline__ void prefetch(const Smem &sm, const S *__restrict__ in, int64_t N, int rd,
                                                    int gg, int pp, int lane, Col &col)
    {
        const int i = 1 + rd * G + gg;
        const S *__restrict__ src = in + static_cast<int64_t>(pp * vs::Q + i) * N;
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            int t = lane + 64 * k;
            t = t < ZC ? t : ZC - 1;                          // idle lanes repeat a valid column
            const int wx = t % WX, wy = t / WX;
            const unsigned base = static_cast<unsigned>(sm.xo[rd][gg][wx] + sm.yo[rd][gg][wy]);
            const int *zo = sm.zo[rd][gg];
#pragma unroll
            for (int g = 0; g <= TEZ; ++g)
#pragma unroll
                for (int r = 0; r <= P; ++r) col[g][k][r] = src[base + static_cast<unsigned>(zo[g * P + r])];
        }
    }

    // outputs of group g (g = -1 .. TE-1) along an axis of TE cells: positions
    // g*P + lstar + j inside [0, TE*P); W = this axis' weights [P][P+1]
    template <int TE, typename Src, typename Dst>
    static __device__ __forceinline__ void group_outputs(int g, int lstar, const S *__restrict__ W, const Src &c,
                                                         Dst &&store)
    {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int pos = g * P + lstar + j;
            if (pos >= 0 && pos < TE * P) {                     // wave-uniform
                const int l = (lstar + j) % P;
                const S *w = W + l * (P + 1);
                S acc = 0;
#pragma unroll
                for (int k = 0; k <= P; ++k) acc = fma(w[k], c[k], acc);
                store(pos, acc);
            }
        }
    }
};

template <typename S, int P, int TEX, int TEY, int TEZ, bool COLLIDE, int MINB>
__global__ void __launch_bounds__(512, MINB)
    k_fused(Geometry geo, FusedTables<S> tab, CollisionParams cp, const S *__restrict__ in, S *__restrict__ out,
            S *__restrict__ pre_out)
{
    using F = Fused<S, P, TEX, TEY, TEZ>;
    constexpr int G = F::G, NT = F::NT, NN = F::NN, RS = F::RS;
    constexpr int TX = F::TX, TY = F::TY, TZ = F::TZ;
    constexpr int WX = F::WX, WY = F::WY, WZ = F::WZ;
    __shared__ typename F::Smem sm;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const int gg = wave >> 1, pp = wave & 1;          // this wave's velocity slot and population
    const int64_t N = geo.nodes;

    // tile origin
    int tcx, tcy, tcz;
    walk_tile(uniform(xcd_tile(blockIdx.x, gridDim.x)), geo, tcx, tcy, tcz);
    const int X0 = tcx * TX, Y0 = tcy * TY, Z0 = tcz * TZ;

    // global node offsets of every round's windows
    for (int e = tid; e < F::NROUND * G * (WX + WY + WZ); e += NT) {
        const int rg = e / (WX + WY + WZ);                 // round * G + velocity slot
        const int r = e % (WX + WY + WZ);
        const int i = 1 + rg;
        if (r < WX) {
            (&sm.xo[0][0][0])[rg * WX + r] = wrap(X0 + tab.omin[i * 3 + 0] * P + r, geo.N[0]);
        } else if (r < WX + WY) {
            const int w = r - WX;
            (&sm.yo[0][0][0])[rg * WY + w] = wrap(Y0 + tab.omin[i * 3 + 1] * P + w, geo.N[1]) * geo.N[0];
        } else {
            const int w = r - WX - WY;
            (&sm.zo[0][0][0])[rg * WZ + w] = wrap(Z0 + tab.omin[i * 3 + 2] * P + w, geo.N[2]) * geo.N[0] * geo.N[1];
        }
    }
    __syncthreads();

    // node and population of this thread: lanes 2k (f) and 2k+1 (g) share a node
    const int nl = tid >> 1;
    const int pop = tid & 1;
    const int lx = nl % TX, ly = (nl / TX) % TY, lz = nl / (TX * TY);
    const bool valid = nl < NN && (X0 + lx < geo.N[0]) && (Y0 + ly < geo.N[1]) && (Z0 + lz < geo.N[2]);
    const int node = ((Z0 + lz) * geo.N[1] + (Y0 + ly)) * geo.N[0] + (X0 + lx);
    const int my_dx = (lz * TY + ly) * RS + lx * 2 + pop;

    S v[vs::Q];
    v[0] = in[static_cast<int64_t>(pop) * vs::Q * N + (valid ? node : 0)];   // the rest velocity does not move

    S *bz = sm.bz[wave];
    S *cy = sm.cy[wave];
    for (int rd = 0; rd < F::NROUND; ++rd) {
        const int i = 1 + rd * G + gg;
        const int lsx = tab.lstar[i * 3 + 0], lsy = tab.lstar[i * 3 + 1], lsz = tab.lstar[i * 3 + 2];
        const S *wxw = tab.w + (i * 3 + 0) * P * (P + 1);
        const S *wyw = tab.w + (i * 3 + 1) * P * (P + 1);
        const S *wzw = tab.w + (i * 3 + 2) * P * (P + 1);

        // z-pass: cell columns straight from global memory
        typename F::Col col;
        F::prefetch(sm, in, N, rd, gg, pp, lane, col);
#pragma unroll
        for (int k = 0; k < F::ZK; ++k) {
            const int t = lane + 64 * k;
            if (t < F::ZC) {
                S *dst = bz + t;                                         // (wx, wy) = t
#pragma unroll
                for (int g = 0; g <= TEZ; ++g)
                    F::template group_outputs<TEZ>(g - 1, lsz, wzw, col[g][k],
                                                   [&](int pos, S val) { dst[pos * WY * WX] = val; });
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // y-pass
#pragma unroll
        for (int k = 0; k < F::YK; ++k) {
            const int t = lane + 64 * k;
            if (t < F::YC) {
                const int wx = t % WX, tz = t / WX;
                const S *src = bz + tz * WY * WX + wx;
                S *dst = cy + tz * TY * WX + wx;
#pragma unroll
                for (int g = 0; g <= TEY; ++g) {
                    S c[P + 1];
#pragma unroll
                    for (int r = 0; r <= P; ++r) c[r] = src[(g * P + r) * WX];
                    F::template group_outputs<TEY>(g - 1, lsy, wyw, c, [&](int pos, S val) { dst[pos * WX] = val; });
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // x-pass into the node-ordered buffer (both populations interleaved)
        S *dxw = sm.dx[rd & 1][gg];
#pragma unroll
        for (int k = 0; k < F::XK; ++k) {
            const int t = lane + 64 * k;
            if (t < F::XC) {
                const S *src = cy + t * WX;                              // row (ty, tz) = t
                S *dst = dxw + t * RS + pp;
#pragma unroll
                for (int g = 0; g <= TEX; ++g) {
                    S c[P + 1];
#pragma unroll
                    for (int r = 0; r <= P; ++r) c[r] = src[g * P + r];
                    F::template group_outputs<TEX>(g - 1, lsx, wxw, c, [&](int pos, S val) { dst[pos * 2] = val; });
                }
            }
        }
        __syncthreads();

        // this round's four values move to the top of v, earlier rounds shift down
#pragma unroll
        for (int q = 1; q + G < vs::Q; ++q) v[q] = v[q + G];
#pragma unroll
        for (int g = 0; g < G; ++g) v[vs::Q - G + g] = sm.dx[rd & 1][g][nl < NN ? my_dx : 0];
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
    constexpr int MB = MinBlocks<S>::value;
    const int nb = g.ntile[0] * g.ntile[1] * g.ntile[2];
    if (collide)
        hipLaunchKernelGGL((k_fused<S, P, TEX, TEY, TEZ, true, MB>), dim3(nb), dim3(512), 0, st, g, t, cp, in, out,
                           pre);
    else
        hipLaunchKernelGGL((k_fused<S, P, TEX, TEY, TEZ, false, MB>), dim3(nb), dim3(512), 0, st, g, t, cp, in,
                           out, pre);
    return hipGetLastError();
}

// Brick of about `concurrent` tiles (the blocks one XCD holds at once).  A
// brick spans whole x rows of tiles when they fit, so its rows are read as
// full cache lines and its x halo is its own data (periodic); its y and z
// extents minimise the ratio of the one-cell-wider read window to the
// brick's own cells.
void fused_bricks(Geometry &g, int concurrent)
{
    const int bx = std::min(g.ntile[0], concurrent);
    double best = 1e300;
    int bb[3] = {bx, 1, 1};
    for (int by = 1; by <= g.ntile[1]; ++by)
        for (int bz = 1; bz <= g.ntile[2]; ++bz) {
            if (bx * by * bz > concurrent) break;
            const double cy = by * g.TE[1], cz = bz * g.TE[2];
            const double wy = by == g.ntile[1] ? cy : cy + 1, wz = bz == g.ntile[2] ? cz : cz + 1;
            const double wx = bx == g.ntile[0] ? 1.0 : (bx * g.TE[0] + 1.0) / (bx * g.TE[0]);
            // fewer tiles than the XCD holds leave CUs idle between bricks: weigh by fill
            const double fill = static_cast<double>(bx * by * bz) / concurrent;
            const double ratio = wx * wy * wz / (cy * cz) / std::sqrt(fill);
            if (ratio < best - 1e-12) {
                best = ratio;
                bb[1] = by;
                bb[2] = bz;
            }
        }
    for (int a = 0; a < 3; ++a) g.brick[a] = bb[a];
}

void fused_tile(int p, int te[3])
{
    static const int table[7][3] = {{0, 0, 0}, {8, 8, 4}, {4, 4, 2}, {3, 3, 1}, {2, 2, 1}, {1, 1, 2}, {1, 1, 1}};
    for (int a = 0; a < 3; ++a) te[a] = table[p][a];
}

template <typename S>
hipError_t launch_fused(const Geometry &g, const FusedTables<S> &t, const CollisionParams &cp, const S *in, S *out,
                        S *pre, bool collide, hipStream_t st)
{
    switch (g.p) {
    case 1: return launch_fused_t<S, 1, 8, 8, 4>(g, t, cp, in, out, pre, collide, st);
    case 2: return launch_fused_t<S, 2, 4, 4, 2>(g, t, cp, in, out, pre, collide, st);
    case 3: return launch_fused_t<S, 3, 3, 3, 1>(g, t, cp, in, out, pre, collide, st);
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
