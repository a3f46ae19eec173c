// Semi-Lagrangian streaming (Sec. II A, Eqs. (8)-(9)) as a z-march per
// (velocity, population) plane and x-y tile.
//
// For velocity i the interpolant factorises into three 1-D operators, and
// along an axis output node e*P + l reads source cell e + o_l, o_l = omin for
// l < lstar and omin + 1 otherwise.  A block owns one population plane of one
// velocity over an x-y tile of TX x TY nodes and walks the z axis:
//   * each source z-row of the tile's window (TX + P + 1 by TY + P + 1 nodes)
//     is loaded once (the next row's loads are in flight while the current
//     row is processed), interpolated along x and then y in LDS, which leaves
//     one value A per output (x, y) and source row;
//   * a thread keeps the A values of the two source cells that output cell
//     e reads (2P + 1 rows) in registers and forms the P outputs of the cell
//     along z with the cell's uniform z weights, then slides by one cell.
// Every source value is read from HBM once per plane (x-y halos of
// neighbouring tiles are served by L2: the tiles of one plane are dealt to
// one XCD), and the outputs are written once, x fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "nt.h"
#include "sllbm_internal.h"
#include "xcd.h"

namespace sllbm {

namespace {

__device__ __forceinline__ int wrapi(int x, int n)
{
    int r = x % n;
    return r < 0 ? r + n : r;
}

constexpr int64_t ZCHUNK_TARGET_BLOCKS = 2048;
constexpr int ZCHUNK_MIN_CELLS = 4;
constexpr int ZCHUNK_MAX_CELL_BYTES = 64;   // cells per chunk times the element size (8 x 32-node tiles)
constexpr int ZCHUNK_MAX_CELLS_LARGE = 32;  // cells per chunk with the 32 x 16-node tiles of large grids

// Number of z-chunks of a march over ntiles x-y tiles and 90 planes.  Small
// grids split the march until the grid has a few blocks per CU slot.  Every
// grid caps a chunk at max_cells cells: blocks of one plane start in
// (chunk, tile) order, so neighbouring tiles march through the same z-rows at
// nearly the same time and more of the x-y halo rows that one tile loads are
// still in L2 when its neighbours read them; blocks that marched the whole
// axis drift apart on large grids.  Each chunk re-reads P + 1 rows.
// Measured at 256^3 nodes (FP64) with 32 x 8-node tiles: reads of 1.87x the
// algorithmic bytes with whole-axis marches, 1.31x with 8-cell chunks (1.59x
// and 1.10x at 128^3), hence ZCHUNK_MAX_CELL_BYTES / elem cells (8 in FP64,
// 16 in FP32).  The 32 x 16-node tiles of large grids have half the x-y halo
// per output, and there 32-cell chunks are 2-4 % faster than 8 or 16 cells.
int z_chunks(const Geometry &g, int ntiles, int max_cells)
{
    int nchunk = 1;
    while (nchunk < g.nel[2] && static_cast<int64_t>(ntiles) * 90 * nchunk < ZCHUNK_TARGET_BLOCKS &&
           g.nel[2] / (2 * nchunk) >= ZCHUNK_MIN_CELLS)
        nchunk *= 2;
    nchunk = std::max(nchunk, (g.nel[2] + max_cells - 1) / max_cells);
    const int zcells = (g.nel[2] + nchunk - 1) / nchunk;
    return (g.nel[2] + zcells - 1) / zcells;
}

// V = values per window load (1, or 16 bytes when every window row starts
// on a 16-byte boundary: p * sizeof(S) and N_x * sizeof(S) multiples of 16)
template <int P, int V = 1, int YN_ = 8>
struct ZTile {
    static constexpr int ORDER = P;
    static constexpr int XN = 32, YN = YN_;                   // target tile extent in nodes (long x rows)
    static constexpr int TXC = XN / P > 0 ? XN / P : 1;       // cells per tile along x and y
    static constexpr int TYC = YN / P > 0 ? YN / P : 1;
    static constexpr int TX = TXC * P, TY = TYC * P;          // nodes per tile
    static constexpr int WX = TX + P + 1, WY = TY + P + 1;    // source window
    static constexpr int WXC = (WX + V - 1) / V, WXP = WXC * V;   // loads per window row, padded row
    static constexpr int NT = (TX * TY + 63) / 64 * 64;       // one thread per output column
    static constexpr int LK = (WXC * WY + NT - 1) / NT;       // window loads per thread and row
    static constexpr int NG = TXC + 1;                        // source cells of an x window row
    static constexpr int BS = TX % 2 ? TX : TX + 1;           // odd row stride of the x-pass output (LDS banks)
};

template <typename S, int V>
struct VecOf {
    typedef S T __attribute__((ext_vector_type(V)));
};
template <typename S>
struct VecOf<S, 1> {
    typedef S T;
};

template <typename VT>
__device__ __forceinline__ auto vcomp(const VT &v, int c)
{
    if constexpr (std::is_arithmetic_v<VT>) return v;
    else return v[c];
}

template <typename S, class Z>
constexpr size_t z_lds_bytes()
{
    return static_cast<size_t>(Z::ORDER + 1) * (static_cast<size_t>(Z::WXP) * Z::WY + Z::WY * Z::BS) * sizeof(S);
}

}  // namespace

// Rows of the x-y tile: 16 (32 x 16 nodes, 512 threads) on grids whose state
// exceeds the Infinity Cache, where the y halo rows that a tile loads per
// output column matter (measured at 256^3 nodes: 5 % faster in FP32, 2 % in
// FP64), if its LDS stays within 64 KB; 8 otherwise (at 64^3 nodes the larger
// tile has too few blocks and is 8 % slower).
template <typename S, int P, int V, bool BIG>
constexpr int z_tile_rows()
{
    return BIG && z_lds_bytes<S, ZTile<P, V, 16>>() <= 64 * 1024 ? 16 : 8;
}

template <typename S, int P, int V, bool NTH>
using ZTileOf = ZTile<P, V, z_tile_rows<S, P, V, NTH>()>;

// NTH: non-temporal output stores and the larger tile (states larger than
// the Infinity Cache)
template <typename S, int P, int V, bool NTH>
__global__ void __launch_bounds__((ZTileOf<S, P, V, NTH>::NT)) k_stream_z(Geometry g, CellTables<S> tab,
                                                                        const S *__restrict__ in,
                                                                        S *__restrict__ out, int ntile_x,
                                                                        int ntiles, int zcells, int nchunk)
{
    using Z = ZTileOf<S, P, V, NTH>;
    using VT = typename VecOf<S, V>::T;
    constexpr int TX = Z::TX, TY = Z::TY, WX = Z::WXP, WY = Z::WY, NT = Z::NT, LK = Z::LK;
    constexpr int WP = WX * WY;
    constexpr int NLD = Z::WXC * WY;                       // window loads per row
    // one batch of source rows (P + 1 for the first cell, P afterwards); single
    // buffers suffice with two barriers per batch: a thread stores the next
    // batch only after the barrier that follows every thread's x-pass, and
    // overwrites bx only after the barrier that follows every thread's y-pass
    __shared__ __align__(16) S pl[P + 1][WP];
    constexpr int BS = Z::BS;
    __shared__ S bx[P + 1][WY * BS];

    const int tid = threadIdx.x;
    const int L = __builtin_amdgcn_readfirstlane(xcd_linear(blockIdx.x, gridDim.x));
    const int q = L / (ntiles * nchunk);
    const int rem = L - q * ntiles * nchunk;
    const int chunk = rem / ntiles, tile = rem - chunk * ntiles;
    const int i = q >> 1, pop = q & 1;
    const int X0 = (tile % ntile_x) * TX, Y0 = (tile / ntile_x) * TY;
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    const int64_t N = g.nodes, NP = static_cast<int64_t>(Nx) * Ny;
    const int omx = tab.omin[i * 3 + 0], omy = tab.omin[i * 3 + 1], omz = tab.omin[i * 3 + 2];
    const int lsx = tab.lstar[i * 3 + 0], lsy = tab.lstar[i * 3 + 1], lsz = tab.lstar[i * 3 + 2];
    const S *Wx = tab.w + (i * 3 + 0) * P * (P + 1);
    const S *Wy = tab.w + (i * 3 + 1) * P * (P + 1);
    const S *Wz = tab.w + (i * 3 + 2) * P * (P + 1);
    const S *__restrict__ src = in + static_cast<int64_t>(pop * 45 + i) * N;
    S *__restrict__ dst = out + static_cast<int64_t>(pop * 45 + i) * N;

    // window loads of this thread (V values each): x-y offsets inside a z-plane;
    // load e covers window row e / WXC, columns V * (e % WXC) ...
    int loff[LK];
#pragma unroll
    for (int k = 0; k < LK; ++k) {
        int e = tid + k * NT;
        e = e < NLD ? e : NLD - 1;                         // surplus lanes repeat the last load
        const int wx = (e % Z::WXC) * V, wy = e / Z::WXC;
        loff[k] = wrapi(Y0 + omy * P + wy, Ny) * Nx + wrapi(X0 + omx * P + wx, Nx);
    }
    // x-pass by source cell: window cell c = g + 1 (g = -1 .. TXC - 1) feeds the
    // outputs g*P + lsx + j, j = 0 .. P-1 (those inside the tile), output j
    // with weight row (lsx + j) mod P, the same for every thread
    S xw[P][P + 1];
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
        for (int r = 0; r <= P; ++r) xw[j][r] = Wx[((lsx + j) % P) * (P + 1) + r];
    // y-pass task and output of this thread: node (X0 + tx, Y0 + ty)
    const int tx = tid % TX, ty = tid / TX;
    const bool own = tid < TX * TY && X0 + tx < Nx && Y0 + ty < Ny;
    const int ly = ty % P;
    const int ysrc = (ty / P + (ly >= lsy ? 1 : 0)) * P * Z::BS + (tid < TX * TY ? tx : 0);
    S yw[P + 1];
#pragma unroll
    for (int r = 0; r <= P; ++r) yw[r] = Wy[ly * (P + 1) + r];
    const int64_t oxy = static_cast<int64_t>(Y0 + ty) * Nx + (X0 + tx);
    S wz[P][P + 1];                                        // uniform z weights of this velocity
#pragma unroll
    for (int l = 0; l < P; ++l)
#pragma unroll
        for (int r = 0; r <= P; ++r) wz[l][r] = Wz[l * (P + 1) + r];

    // this block's output cells [ez0, ez1) along z; source rows in march
    // order: z = (ez0 + omz) * P + k (mod Nz), k = 0 .. P + (ez1 - ez0) * P
    const int ez0 = chunk * zcells, ez1 = min(g.nel[2], ez0 + zcells);
    // row k < P + 1 + (ez1 - ez0) P <= Nz + P + 1 and zb < Nz, so two
    // conditional subtractions wrap zb + k (no integer division per row)
    const int zb = wrapi((ez0 + omz) * P, Nz);
    // two register buffers of source rows: the rows of the cell after next are
    // in flight while a cell is processed
    VT rawA[P + 1][LK], rawB[P][LK];
    auto load_rows = [&](auto &raw, int k0, int nr) {
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            if (r < nr && r < static_cast<int>(sizeof(raw) / sizeof(raw[0]))) {
                int z = zb + k0 + r;
                z -= z >= Nz ? Nz : 0;
                z -= z >= Nz ? Nz : 0;
                const int64_t zo = static_cast<int64_t>(z) * NP;
#pragma unroll
                for (int j = 0; j < LK; ++j) raw[r][j] = *reinterpret_cast<const VT *>(src + zo + loff[j]);
            }
        }
    };
    // a batch of NR rows: registers -> LDS, the same registers reloaded with
    // the rows two batches ahead, x-pass, y-pass
    auto batch = [&](auto nr_c, auto &raw, int next_k0, int next_nr, S *res) {
        constexpr int NR = decltype(nr_c)::value;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int j = 0; j < LK; ++j)
                if (tid + j * NT < NLD) *reinterpret_cast<VT *>(&pl[r][V * (tid + j * NT)]) = raw[r][j];
        if (next_nr > 0) load_rows(raw, next_k0, next_nr);
        __syncthreads();
        constexpr int XT = NR * WY * Z::NG;                   // (row, window row, source cell) tasks
#pragma unroll
        for (int k = 0; k < (XT + NT - 1) / NT; ++k) {
            const int e = tid + k * NT;
            if (e < XT) {
                const int r = e / (WY * Z::NG), rem = e - r * (WY * Z::NG);
                const int g = rem / WY - 1, wy = rem - (g + 1) * WY;   // neighbouring lanes: neighbouring rows
                const S *c = &pl[r][wy * WX + (g + 1) * P];
                S v[P + 1];
#pragma unroll
                for (int m = 0; m <= P; ++m) v[m] = c[m];
                S *o = &bx[r][wy * BS];
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int pos = g * P + lsx + j;
                    if (pos >= 0 && pos < TX) {
                        S acc = 0;
#pragma unroll
                        for (int m = 0; m <= P; ++m) acc = fma(xw[j][m], v[m], acc);
                        o[pos] = acc;
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            S acc = 0;
#pragma unroll
            for (int m = 0; m <= P; ++m) acc = fma(yw[m], bx[r][ysrc + m * BS], acc);
            res[r] = acc;
        }
    };
    // P outputs of cell ez along z from the rows in a, then slide by one cell
    S a[2 * P + 1];
    auto emit = [&](int ez) {
        if (own) {
#pragma unroll
            for (int l = 0; l < P; ++l) {
                const bool hi = l >= lsz;
                S acc = 0;
#pragma unroll
                for (int r = 0; r <= P; ++r) acc = fma(wz[l][r], hi ? a[P + r] : a[r], acc);
                store_hint<NTH>(&dst[static_cast<int64_t>(ez * P + l) * NP + oxy], acc);
            }
        }
#pragma unroll
        for (int r = 0; r <= P; ++r) a[r] = a[r + P];
    };

    // rows 0 .. P (first source cell) in rawA, then the rows of cell e
    // (P + 1 + e*P .. 2P + e*P) alternate between rawB (even e) and rawA (odd e)
    const int nel = ez1 - ez0;
    auto rows_of = [&](int e) { return e < nel ? P : 0; };
    load_rows(rawA, 0, P + 1);
    load_rows(rawB, P + 1, rows_of(0));
    batch(std::integral_constant<int, P + 1>(), rawA, 2 * P + 1, rows_of(1), a);
    for (int e = 0; e < nel; e += 2) {
        batch(std::integral_constant<int, P>(), rawB, P + 1 + (e + 2) * P, rows_of(e + 2), a + P + 1);
        emit(ez0 + e);
        if (e + 1 < nel) {
            batch(std::integral_constant<int, P>(), rawA, P + 1 + (e + 3) * P, rows_of(e + 3), a + P + 1);
            emit(ez0 + e + 1);
        }
    }
}

template <typename S, int P, int V, bool NTH>
static hipError_t launch_zvn(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    using Z = ZTileOf<S, P, V, NTH>;
    const int ntx = (g.N[0] + Z::TX - 1) / Z::TX, nty = (g.N[1] + Z::TY - 1) / Z::TY;
    const int ntiles = ntx * nty;
    const int nchunk = z_chunks(g, ntiles, Z::YN == 16 ? ZCHUNK_MAX_CELLS_LARGE
                                                     : ZCHUNK_MAX_CELL_BYTES / static_cast<int>(sizeof(S)));
    const int zcells = (g.nel[2] + nchunk - 1) / nchunk;
    const int64_t nb = static_cast<int64_t>(ntiles) * 90 * nchunk;
    if (nb > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stream_z<S, P, V, NTH>), dim3(static_cast<unsigned>(nb)), dim3(Z::NT), 0, st, g, t, in, out,
                       ntx, ntiles, zcells, nchunk);
    return hipGetLastError();
}

template <typename S, int P, int V>
static hipError_t launch_zv(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    if (use_nontemporal(90 * g.nodes * static_cast<int64_t>(sizeof(S))))
        return launch_zvn<S, P, V, true>(g, t, in, out, st);
    return launch_zvn<S, P, V, false>(g, t, in, out, st);
}

// 16-byte window loads when every window row starts on a 16-byte boundary
template <typename S, int P>
static hipError_t launch_z(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    constexpr int V = 16 / sizeof(S);
    const bool aligned = (P * sizeof(S)) % 16 == 0 && (g.N[0] * sizeof(S)) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(in) % 16 == 0;
    if constexpr ((P * sizeof(S)) % 16 == 0 && ZTile<P, V>::TX % V == 0) {
        if (aligned) return launch_zv<S, P, V>(g, t, in, out, st);
    }
    return launch_zv<S, P, 1>(g, t, in, out, st);
}

// ---------------------------------------------------------------------------
// Transposed streaming S^T (the adjoint of Eqs. (8)-(9)), same z-march.
//
// Along an axis the forward nodes that read source cell c form a group: the
// nodes (c - omin - 1)*P + lstar + j, j = 0 .. P-1, read it with weight row
// (lstar + j) mod P.  Transposing, node k of cell c receives
//   T[c*P + k] = sum_j W[(lstar + j) mod P][k] lam[group(c)_j]
// and node 0 also, as point P of cell c - 1,
//   + sum_j W[(lstar + j) mod P][P] lam[group(c - 1)_j].
// So each output cell gathers two consecutive groups (2P inputs, starting at
// (c - omin - 2)*P + lstar) with the forward weights; this holds for any
// number of cells, wrap-around included.  The kernel is the forward one with
// that gather along x, y (LDS) and z (a register window of 2P rows sliding by
// one cell).
// ---------------------------------------------------------------------------
template <int P, int V = 1, int YN_ = 8>
struct ZTileT {
    static constexpr int ORDER = P;
    static constexpr int XN = 32, YN = YN_;
    static constexpr int TXC = XN / P > 0 ? XN / P : 1, TYC = YN / P > 0 ? YN / P : 1;
    static constexpr int TX = TXC * P, TY = TYC * P;
    static constexpr int WXC = (TX + P + V - 1 + V - 1) / V;  // loads per window row (V-aligned start)
    static constexpr int WX = WXC * V, WY = TY + P;
    static constexpr int NT = (TX * TY + 63) / 64 * 64;
    static constexpr int LK = (WXC * WY + NT - 1) / NT;
    static constexpr int BS = TX % 2 ? TX : TX + 1;
};

// Tile rows of the transposed march, chosen as in the forward one: 16 on
// grids larger than the Infinity Cache if the LDS stays within 64 KB
template <typename S, class Z>
constexpr size_t zt_lds_bytes()
{
    constexpr int WXO = Z::WX % 2 ? Z::WX : Z::WX + 1;
    return static_cast<size_t>(Z::ORDER) * (static_cast<size_t>(WXO) * Z::WY + Z::WY * Z::BS) * sizeof(S);
}

template <typename S, int P, int V, bool BIG>
constexpr int zt_tile_rows()
{
    return BIG && zt_lds_bytes<S, ZTileT<P, V, 16>>() <= 64 * 1024 ? 16 : 8;
}

template <typename S, int P, int V, bool NTH>
using ZTileTOf = ZTileT<P, V, zt_tile_rows<S, P, V, NTH>()>;

// NTH: non-temporal output stores and the larger tile (states larger than
// the Infinity Cache)
template <typename S, int P, int V, bool NTH>
__global__ void __launch_bounds__((ZTileTOf<S, P, V, NTH>::NT))
    k_stream_zt(Geometry g, CellTables<S> tab, const S *__restrict__ in, S *__restrict__ out, int ntile_x,
                int ntiles, int zcells, int nchunk)
{
    using Z = ZTileTOf<S, P, V, NTH>;
    using VT = typename VecOf<S, V>::T;
    constexpr int TX = Z::TX, TY = Z::TY, WY = Z::WY, NT = Z::NT, LK = Z::LK, BS = Z::BS;
    constexpr int WX = Z::WX % 2 ? Z::WX : Z::WX + 1;      // odd LDS row stride
    constexpr int NLD = Z::WXC * WY;
    __shared__ __align__(16) S pl[P][WX * WY];
    __shared__ S bx[P][WY * BS];

    const int tid = threadIdx.x;
    const int L = __builtin_amdgcn_readfirstlane(xcd_linear(blockIdx.x, gridDim.x));
    const int q = L / (ntiles * nchunk);
    const int rem = L - q * ntiles * nchunk;
    const int chunk = rem / ntiles, tile = rem - chunk * ntiles;
    const int i = q >> 1, pop = q & 1;
    const int X0 = (tile % ntile_x) * TX, Y0 = (tile / ntile_x) * TY;
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    const int64_t N = g.nodes, NP = static_cast<int64_t>(Nx) * Ny;
    const int omx = tab.omin[i * 3 + 0], omy = tab.omin[i * 3 + 1], omz = tab.omin[i * 3 + 2];
    const int lsx = tab.lstar[i * 3 + 0], lsy = tab.lstar[i * 3 + 1], lsz = tab.lstar[i * 3 + 2];
    const S *Wx = tab.w + (i * 3 + 0) * P * (P + 1);
    const S *Wy = tab.w + (i * 3 + 1) * P * (P + 1);
    const S *Wz = tab.w + (i * 3 + 2) * P * (P + 1);
    const S *__restrict__ src = in + static_cast<int64_t>(pop * 45 + i) * N;
    S *__restrict__ dst = out + static_cast<int64_t>(pop * 45 + i) * N;

    // input window: x from X0 + (-2 - omx)*P + lsx (rounded down to V: shift sx), y from Y0 + (-2 - omy)*P + lsy
    const int offx = (-2 - omx) * P + lsx;
    const int offxa = offx - ((offx % V) + V) % V, sx = offx - offxa;
    const int offy = (-2 - omy) * P + lsy;
    int loff[LK], soff[LK];                                // HBM and LDS offsets of this thread's loads
#pragma unroll
    for (int k = 0; k < LK; ++k) {
        int e = tid + k * NT;
        e = e < NLD ? e : NLD - 1;
        const int wx = (e % Z::WXC) * V, wy = e / Z::WXC;
        loff[k] = wrapi(Y0 + offy + wy, Ny) * Nx + wrapi(X0 + offxa + wx, Nx);
        soff[k] = wy * WX + wx;
    }
    // x and z weights, the same for every thread: w*[j][k] = W[(ls + j) mod P][k]
    S wxu[P][P + 1], wzu[P][P + 1];
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
        for (int k = 0; k <= P; ++k) {
            wxu[j][k] = Wx[((lsx + j) % P) * (P + 1) + k];
            wzu[j][k] = Wz[((lsz + j) % P) * (P + 1) + k];
        }
    // output node (X0 + tx, Y0 + ty): point ky of tile cell cy along y gathers
    // window rows (cy + 1)*P + j with yw[j], and for ky = 0 rows cy*P + j with yp[j]
    const int tx = tid % TX, ty = tid / TX;
    const bool own = tid < TX * TY && X0 + tx < Nx && Y0 + ty < Ny;
    const int cy = ty / P, ky = ty % P;
    const int ybase = cy * P * BS + (tid < TX * TY ? tx : 0);
    S yw[P], yp[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        yw[j] = Wy[((lsy + j) % P) * (P + 1) + ky];
        yp[j] = ky == 0 ? Wy[((lsy + j) % P) * (P + 1) + P] : S(0);
    }
    const int64_t oxy = static_cast<int64_t>(Y0 + ty) * Nx + (X0 + tx);

    // input rows in march order: z = (ez0 - omz - 2)*P + lsz + k (mod Nz), k = 0 .. P + nel*P - 1
    const int ez0 = chunk * zcells, ez1 = min(g.nel[2], ez0 + zcells);
    // row k < P + (ez1 - ez0) P <= Nz + P and zb < Nz: two conditional
    // subtractions wrap zb + k
    const int zb = wrapi((ez0 - omz - 2) * P + lsz, Nz);
    VT rawA[P][LK], rawB[P][LK];
    auto load_rows = [&](auto &raw, int k0, int nr) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
            if (r < nr) {
                int z = zb + k0 + r;
                z -= z >= Nz ? Nz : 0;
                z -= z >= Nz ? Nz : 0;
                const int64_t zo = static_cast<int64_t>(z) * NP;
#pragma unroll
                for (int j = 0; j < LK; ++j) raw[r][j] = *reinterpret_cast<const VT *>(src + zo + loff[j]);
            }
        }
    };
    // P rows: registers -> LDS, reload with the rows two batches ahead, x-gather, y-gather
    auto batch = [&](auto &raw, int next_k0, int next_nr, S *res) {
#pragma unroll
        for (int r = 0; r < P; ++r)
#pragma unroll
            for (int j = 0; j < LK; ++j)
                if (tid + j * NT < NLD) {
#pragma unroll
                    for (int c = 0; c < V; ++c) pl[r][soff[j] + c] = vcomp(raw[r][j], c);
                }
        if (next_nr > 0) load_rows(raw, next_k0, next_nr);
        __syncthreads();
        // x: task (row, window row, output cell cl) reads groups cl and cl + 1 of the row
        constexpr int XT = P * WY * Z::TXC;
#pragma unroll
        for (int k = 0; k < (XT + NT - 1) / NT; ++k) {
            const int e = tid + k * NT;
            if (e < XT) {
                const int r = e / (WY * Z::TXC), rem2 = e - r * (WY * Z::TXC);
                const int cl = rem2 / WY, wy = rem2 - cl * WY;
                const S *c = &pl[r][wy * WX + sx + cl * P];
                S prev[P], cur[P];
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    prev[j] = c[j];
                    cur[j] = c[P + j];
                }
                S *o = &bx[r][wy * BS + cl * P];
#pragma unroll
                for (int kk = 0; kk < P; ++kk) {
                    S acc = 0;
#pragma unroll
                    for (int j = 0; j < P; ++j) acc = fma(wxu[j][kk], cur[j], acc);
                    if (kk == 0) {
#pragma unroll
                        for (int j = 0; j < P; ++j) acc = fma(wxu[j][P], prev[j], acc);
                    }
                    o[kk] = acc;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < P; ++r) {
            S acc = 0;
#pragma unroll
            for (int j = 0; j < P; ++j) acc = fma(yw[j], bx[r][ybase + (P + j) * BS], acc);
#pragma unroll
            for (int j = 0; j < P; ++j) acc = fma(yp[j], bx[r][ybase + j * BS], acc);
            res[r] = acc;
        }
    };
    S a[2 * P];
    auto emit = [&](int ez) {
        if (own) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                S acc = 0;
#pragma unroll
                for (int j = 0; j < P; ++j) acc = fma(wzu[j][k], a[P + j], acc);
                if (k == 0) {
#pragma unroll
                    for (int j = 0; j < P; ++j) acc = fma(wzu[j][P], a[j], acc);
                }
                store_hint<NTH>(&dst[static_cast<int64_t>(ez * P + k) * NP + oxy], acc);
            }
        }
#pragma unroll
        for (int j = 0; j < P; ++j) a[j] = a[P + j];
    };

    const int nel = ez1 - ez0;
    auto rows_of = [&](int e) { return e < nel ? P : 0; };
    load_rows(rawA, 0, P);
    load_rows(rawB, P, rows_of(0));
    batch(rawA, 2 * P, rows_of(1), a);
    for (int e = 0; e < nel; e += 2) {
        batch(rawB, P + (e + 2) * P, rows_of(e + 2), a + P);
        emit(ez0 + e);
        if (e + 1 < nel) {
            batch(rawA, P + (e + 3) * P, rows_of(e + 3), a + P);
            emit(ez0 + e + 1);
        }
    }
}

template <typename S, int P, int V, bool NTH>
static hipError_t launch_ztvn(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    using Z = ZTileTOf<S, P, V, NTH>;
    const int ntx = (g.N[0] + Z::TX - 1) / Z::TX, nty = (g.N[1] + Z::TY - 1) / Z::TY;
    const int ntiles = ntx * nty;
    // each chunk re-reads P rows
    const int nchunk = z_chunks(g, ntiles, Z::YN == 16 ? ZCHUNK_MAX_CELLS_LARGE
                                                     : ZCHUNK_MAX_CELL_BYTES / static_cast<int>(sizeof(S)));
    const int zcells = (g.nel[2] + nchunk - 1) / nchunk;
    const int64_t nb = static_cast<int64_t>(ntiles) * 90 * nchunk;
    if (nb > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stream_zt<S, P, V, NTH>), dim3(static_cast<unsigned>(nb)), dim3(Z::NT), 0, st, g, t, in,
                       out, ntx, ntiles, zcells, nchunk);
    return hipGetLastError();
}

template <typename S, int P, int V>
static hipError_t launch_ztv(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    if (use_nontemporal(90 * g.nodes * static_cast<int64_t>(sizeof(S))))
        return launch_ztvn<S, P, V, true>(g, t, in, out, st);
    return launch_ztvn<S, P, V, false>(g, t, in, out, st);
}

// 16-byte window loads need V-aligned window starts: tiles and rows of a
// multiple of V nodes and a 16-byte aligned buffer (the start is rounded down)
template <typename S, int P>
static hipError_t launch_zt(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    constexpr int V = 16 / sizeof(S);
    if constexpr (ZTileT<P, V>::TX % V == 0) {
        if ((g.N[0] * sizeof(S)) % 16 == 0 && reinterpret_cast<uintptr_t>(in) % 16 == 0)
            return launch_ztv<S, P, V>(g, t, in, out, st);
    }
    return launch_ztv<S, P, 1>(g, t, in, out, st);
}

template <typename S>
hipError_t launch_stream_zt(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    switch (g.p) {
    case 1: return launch_zt<S, 1>(g, t, in, out, st);
    case 2: return launch_zt<S, 2>(g, t, in, out, st);
    case 3: return launch_zt<S, 3>(g, t, in, out, st);
    case 4: return launch_zt<S, 4>(g, t, in, out, st);
    case 5: return launch_zt<S, 5>(g, t, in, out, st);
    case 6: return launch_zt<S, 6>(g, t, in, out, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stream_zt<double>(const Geometry &, const CellTables<double> &, const double *, double *,
                                             hipStream_t);
template hipError_t launch_stream_zt<float>(const Geometry &, const CellTables<float> &, const float *, float *,
                                            hipStream_t);

template <typename S>
hipError_t launch_stream_z(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    switch (g.p) {
    case 1: return launch_z<S, 1>(g, t, in, out, st);
    case 2: return launch_z<S, 2>(g, t, in, out, st);
    case 3: return launch_z<S, 3>(g, t, in, out, st);
    case 4: return launch_z<S, 4>(g, t, in, out, st);
    case 5: return launch_z<S, 5>(g, t, in, out, st);
    case 6: return launch_z<S, 6>(g, t, in, out, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stream_z<double>(const Geometry &, const CellTables<double> &, const double *, double *,
                                            hipStream_t);
template hipError_t launch_stream_z<float>(const Geometry &, const CellTables<float> &, const float *, float *,
                                           hipStream_t);

}  // namespace sllbm
