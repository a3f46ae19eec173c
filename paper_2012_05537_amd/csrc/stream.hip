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

#include <type_traits>

#include "sllbm_internal.h"

namespace sllbm {

namespace {

__device__ __forceinline__ int wrapi(int x, int n)
{
    int r = x % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ int xcd_linear(int b, int nb)
{
    const int xcd = b & 7, slot = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

constexpr int64_t ZCHUNK_TARGET_BLOCKS = 2048;
constexpr int ZCHUNK_MIN_CELLS = 4;

// V = values per window load (1, or 16 bytes when every window row starts
// on a 16-byte boundary: p * sizeof(S) and N_x * sizeof(S) multiples of 16)
template <int P, int V = 1>
struct ZTile {
    static constexpr int XN = 32, YN = 8;                     // target tile extent in nodes (long x rows)
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

}  // namespace

template <typename S, int P, int V>
__global__ void __launch_bounds__((ZTile<P, V>::NT)) k_stream_z(Geometry g, CellTables<S> tab, const S *__restrict__ in,
                                                     S *__restrict__ out, int ntile_x, int ntiles, int zcells,
                                                     int nchunk)
{
    using Z = ZTile<P, V>;
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
    const int zb = (ez0 + omz) * P;
    // two register buffers of source rows: the rows of the cell after next are
    // in flight while a cell is processed
    VT rawA[P + 1][LK], rawB[P][LK];
    auto load_rows = [&](auto &raw, int k0, int nr) {
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            if (r < nr && r < static_cast<int>(sizeof(raw) / sizeof(raw[0]))) {
                const int64_t zo = static_cast<int64_t>(wrapi(zb + k0 + r, Nz)) * NP;
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
                dst[static_cast<int64_t>(ez * P + l) * NP + oxy] = acc;
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

template <typename S, int P, int V>
static hipError_t launch_zv(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    using Z = ZTile<P, V>;
    const int ntx = (g.N[0] + Z::TX - 1) / Z::TX, nty = (g.N[1] + Z::TY - 1) / Z::TY;
    const int ntiles = ntx * nty;
    // split the z-march into chunks until the grid has a few blocks per CU
    // slot (each chunk re-reads P + 1 source rows)
    int nchunk = 1;
    while (nchunk < g.nel[2] && static_cast<int64_t>(ntiles) * 90 * nchunk < ZCHUNK_TARGET_BLOCKS &&
           g.nel[2] / (2 * nchunk) >= ZCHUNK_MIN_CELLS)
        nchunk *= 2;
    const int zcells = (g.nel[2] + nchunk - 1) / nchunk;
    nchunk = (g.nel[2] + zcells - 1) / zcells;
    const int64_t nb = static_cast<int64_t>(ntiles) * 90 * nchunk;
    if (nb > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stream_z<S, P, V>), dim3(static_cast<unsigned>(nb)), dim3(Z::NT), 0, st, g, t, in, out, ntx,
                       ntiles, zcells, nchunk);
    return hipGetLastError();
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
// Along x and y the transposed 1-D operator is a gather over the transposed
// tables (node m of a cell reads at most 2P nodes at offsets relative to its
// cell start).  Along z it is applied as the scatter of the forward operator:
// input row e*P + l, which the forward step gathers into source rows
// (e + o_l)*P + k, adds W[l][k] times its value to those rows.  A thread
// keeps the 2P + 1 rows of source cells e + omin and e + omin + 1 in
// registers; after input cell e the rows of cell e + omin are complete (the
// next input cell only reaches cells e + omin + 1 and up) and are written.
// Row 0 of source cell c also receives, as row P of cell c - 1, from input
// cells c - omin - 1 and c - omin - 2, so a chunk of input cells [e0, e1)
// first scatters cells e0 - 2 and e0 - 1 without writing; then every written
// row has all its contributions.  Requires at least three cells along z
// (with two, one input cell would reach the same row twice by wrapping).
// ---------------------------------------------------------------------------
template <int P, int V = 1>
struct ZTileT {
    static constexpr int XN = 32, YN = 8;
    static constexpr int TXC = XN / P > 0 ? XN / P : 1, TYC = YN / P > 0 ? YN / P : 1;
    static constexpr int TX = TXC * P, TY = TYC * P;
    static constexpr int K = 2 * P;                           // taps of a transposed row
    static constexpr int SPMAX = 3 * P + 1;                   // largest offset span of a transposed row set
    static constexpr int WXC = (TX + SPMAX - 1 + V - 1 + V - 1) / V;   // loads per window row (V-aligned start)
    static constexpr int WX = WXC * V, WY = TY + SPMAX - 1;
    static constexpr int NT = (TX * TY + 63) / 64 * 64;
    static constexpr int LK = (WXC * WY + NT - 1) / NT;
    static constexpr int XR = NT / TX;                        // window rows per x-gather pass
    static constexpr int XK = (WY + XR - 1) / XR;
    static constexpr int BS = TX % 2 ? TX : TX + 1;
};

template <typename S, int P, int V>
__global__ void __launch_bounds__((ZTileT<P, V>::NT))
    k_stream_zt(Geometry g, CellTables<S> fwd, const int32_t *__restrict__ toff, const S *__restrict__ twt,
                const int32_t *__restrict__ tlo, const int32_t *__restrict__ tspan, const S *__restrict__ in,
                S *__restrict__ out, int ntile_x, int ntiles, int zcells, int nchunk)
{
    using Z = ZTileT<P, V>;
    using VT = typename VecOf<S, V>::T;
    constexpr int TX = Z::TX, TY = Z::TY, NT = Z::NT, LK = Z::LK, XK = Z::XK, K = Z::K, BS = Z::BS;
    __shared__ __align__(16) S pl[P][Z::WX * Z::WY];
    __shared__ S bx[P][Z::WY * BS];

    const int tid = threadIdx.x;
    const int L = __builtin_amdgcn_readfirstlane(xcd_linear(blockIdx.x, gridDim.x));
    const int q = L / (ntiles * nchunk);
    const int rem = L - q * ntiles * nchunk;
    const int chunk = rem / ntiles, tile = rem - chunk * ntiles;
    const int i = q >> 1, pop = q & 1;
    const int X0 = (tile % ntile_x) * TX, Y0 = (tile / ntile_x) * TY;
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    const int64_t N = g.nodes, NP = static_cast<int64_t>(Nx) * Ny;
    const int lox = tlo[i * 3 + 0], loy = tlo[i * 3 + 1];
    const int lxa = lox - ((lox % V) + V) % V;            // window start, rounded down to V
    const int wxc = (TX + tspan[i * 3 + 0] - 1 + (lox - lxa) + V - 1) / V;
    const int wxs = wxc * V, wys = TY + tspan[i * 3 + 1] - 1;   // window of this velocity
    const int nld = wxc * wys;
    const int omz = fwd.omin[i * 3 + 2], lsz = fwd.lstar[i * 3 + 2];
    const S *Wz = fwd.w + (i * 3 + 2) * P * (P + 1);
    const int32_t *ox = toff + (i * 3 + 0) * P * K, *oy = toff + (i * 3 + 1) * P * K;
    const S *wxt = twt + (i * 3 + 0) * P * K, *wyt = twt + (i * 3 + 1) * P * K;
    const S *__restrict__ src = in + static_cast<int64_t>(pop * 45 + i) * N;
    S *__restrict__ dst = out + static_cast<int64_t>(pop * 45 + i) * N;

    int loff[LK];
#pragma unroll
    for (int k = 0; k < LK; ++k) {
        int e = tid + k * NT;
        e = e < nld ? e : nld - 1;
        const int wx = (e % wxc) * V, wy = e / wxc;
        loff[k] = wrapi(Y0 + loy + wy, Ny) * Nx + wrapi(X0 + lxa + wx, Nx);
    }
    // x-gather: thread (xrow, xt) handles column xt of window rows xrow, xrow + XR, ...;
    // its taps (offsets within the row and weights) are fixed
    const int xt = tid % TX, xrow = tid / TX, mx = xt % P;
    const bool xact = xrow < Z::XR;
    int xs[K];
    S xw[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        xs[t] = xt - mx + ox[mx * K + t] - lxa;
        xw[t] = wxt[mx * K + t];
    }
    const int tx = tid % TX, ty = tid / TX;
    const bool own = tid < TX * TY && X0 + tx < Nx && Y0 + ty < Ny;
    const int my = ty % P;
    int ys[K];
    S yw[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        ys[t] = (ty - my + oy[my * K + t] - loy) * BS + (tid < TX * TY ? tx : 0);
        yw[t] = wyt[my * K + t];
    }
    const int64_t oxy = static_cast<int64_t>(Y0 + ty) * Nx + (X0 + tx);
    S wz[P][P + 1];
#pragma unroll
    for (int l = 0; l < P; ++l)
#pragma unroll
        for (int r = 0; r <= P; ++r) wz[l][r] = Wz[l * (P + 1) + r];

    // input cells e0 - 2 .. e1 - 1; row l of cell e is z = e*P + l
    const int e0 = chunk * zcells, e1 = min(g.nel[2], e0 + zcells);
    VT raw[P][LK];
    auto load_cell = [&](int e) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int64_t zo = static_cast<int64_t>(wrapi(e * P + r, Nz)) * NP;
#pragma unroll
            for (int j = 0; j < LK; ++j) raw[r][j] = *reinterpret_cast<const VT *>(src + zo + loff[j]);
        }
    };
    S acc[2 * P + 1];
#pragma unroll
    for (int r = 0; r <= 2 * P; ++r) acc[r] = 0;
    load_cell(e0 - 2);
    for (int e = e0 - 2; e < e1; ++e) {
#pragma unroll
        for (int r = 0; r < P; ++r)
#pragma unroll
            for (int j = 0; j < LK; ++j)
                if (tid + j * NT < nld) *reinterpret_cast<VT *>(&pl[r][V * (tid + j * NT)]) = raw[r][j];
        if (e + 1 < e1) load_cell(e + 1);
        __syncthreads();
        if (xact) {
#pragma unroll
            for (int r = 0; r < P; ++r)
#pragma unroll
                for (int k = 0; k < XK; ++k) {
                    const int wy = xrow + k * Z::XR;
                    if (wy < wys) {
                        const S *rowp = &pl[r][wy * wxs];
                        S v = 0;
#pragma unroll
                        for (int t = 0; t < K; ++t) v = fma(xw[t], rowp[xs[t]], v);
                        bx[r][wy * BS + xt] = v;
                    }
                }
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < P; ++l) {
            S a = 0;
#pragma unroll
            for (int t = 0; t < K; ++t) a = fma(yw[t], bx[l][ys[t]], a);
            const bool hi = l >= lsz;
#pragma unroll
            for (int r = 0; r <= P; ++r) {
                const S c = wz[l][r] * a;
                acc[P + r] += hi ? c : S(0);
                acc[r] += hi ? S(0) : c;
            }
        }
        if (e >= e0 && own) {
#pragma unroll
            for (int r = 0; r < P; ++r)
                dst[static_cast<int64_t>(wrapi((e + omz) * P + r, Nz)) * NP + oxy] = acc[r];
        }
#pragma unroll
        for (int r = 0; r <= P; ++r) acc[r] = acc[r + P];
#pragma unroll
        for (int r = P + 1; r <= 2 * P; ++r) acc[r] = 0;
    }
}

template <typename S, int P, int V>
static hipError_t launch_ztv(const Geometry &g, const CellTables<S> &t, const int32_t *toff, const S *twt,
                             const int32_t *tlo, const int32_t *tspan, const S *in, S *out, hipStream_t st)
{
    using Z = ZTileT<P, V>;
    const int ntx = (g.N[0] + Z::TX - 1) / Z::TX, nty = (g.N[1] + Z::TY - 1) / Z::TY;
    const int ntiles = ntx * nty;
    int nchunk = 1;
    while (nchunk < g.nel[2] && static_cast<int64_t>(ntiles) * 90 * nchunk < ZCHUNK_TARGET_BLOCKS &&
           g.nel[2] / (2 * nchunk) >= ZCHUNK_MIN_CELLS)
        nchunk *= 2;
    const int zcells = (g.nel[2] + nchunk - 1) / nchunk;
    nchunk = (g.nel[2] + zcells - 1) / zcells;
    const int64_t nb = static_cast<int64_t>(ntiles) * 90 * nchunk;
    if (nb > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stream_zt<S, P, V>), dim3(static_cast<unsigned>(nb)), dim3(Z::NT), 0, st, g, t, toff, twt,
                       tlo, tspan, in, out, ntx, ntiles, zcells, nchunk);
    return hipGetLastError();
}

template <typename S, int P>
static hipError_t launch_zt(const Geometry &g, const CellTables<S> &t, const int32_t *toff, const S *twt,
                            const int32_t *tlo, const int32_t *tspan, const S *in, S *out, hipStream_t st)
{
    // 16-byte loads need V-aligned window starts: tiles of a multiple of V
    // nodes, rows of a multiple of V nodes, a 16-byte aligned buffer
    constexpr int V = 16 / sizeof(S);
    if constexpr (ZTileT<P, V>::TX % V == 0) {
        if ((g.N[0] * sizeof(S)) % 16 == 0 && reinterpret_cast<uintptr_t>(in) % 16 == 0)
            return launch_ztv<S, P, V>(g, t, toff, twt, tlo, tspan, in, out, st);
    }
    return launch_ztv<S, P, 1>(g, t, toff, twt, tlo, tspan, in, out, st);
}

template <typename S>
hipError_t launch_stream_zt(const Geometry &g, const CellTables<S> &t, const StreamTables &adj, const S *in, S *out,
                            hipStream_t st)
{
    const S *wt = static_cast<const S *>(adj.wt);
    switch (g.p) {
    case 1: return launch_zt<S, 1>(g, t, adj.off, wt, adj.lo, adj.span, in, out, st);
    case 2: return launch_zt<S, 2>(g, t, adj.off, wt, adj.lo, adj.span, in, out, st);
    case 3: return launch_zt<S, 3>(g, t, adj.off, wt, adj.lo, adj.span, in, out, st);
    case 4: return launch_zt<S, 4>(g, t, adj.off, wt, adj.lo, adj.span, in, out, st);
    case 5: return launch_zt<S, 5>(g, t, adj.off, wt, adj.lo, adj.span, in, out, st);
    case 6: return launch_zt<S, 6>(g, t, adj.off, wt, adj.lo, adj.span, in, out, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stream_zt<double>(const Geometry &, const CellTables<double> &, const StreamTables &,
                                             const double *, double *, hipStream_t);
template hipError_t launch_stream_zt<float>(const Geometry &, const CellTables<float> &, const StreamTables &,
                                            const float *, float *, hipStream_t);

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
