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

template <int P>
struct ZTile {
    static constexpr int XN = 16, YN = 16;                    // target tile extent in nodes
    static constexpr int TXC = XN / P > 0 ? XN / P : 1;       // cells per tile along x and y
    static constexpr int TYC = YN / P > 0 ? YN / P : 1;
    static constexpr int TX = TXC * P, TY = TYC * P;          // nodes per tile
    static constexpr int WX = TX + P + 1, WY = TY + P + 1;    // source window
    static constexpr int NT = (TX * TY + 63) / 64 * 64;       // one thread per output column
    static constexpr int LK = (WX * WY + NT - 1) / NT;        // window loads per thread and row
    static constexpr int XT = WY * TX, XK = (XT + NT - 1) / NT;   // x-pass outputs per thread and row
};

}  // namespace

template <typename S, int P>
__global__ void __launch_bounds__(ZTile<P>::NT) k_stream_z(Geometry g, CellTables<S> tab, const S *__restrict__ in,
                                                  S *__restrict__ out, int ntile_x, int ntiles, int zcells,
                                                  int nchunk)
{
    using Z = ZTile<P>;
    constexpr int TX = Z::TX, TY = Z::TY, WX = Z::WX, WY = Z::WY, NT = Z::NT, LK = Z::LK, XK = Z::XK;
    constexpr int WP = WX * WY;
    // one batch of source rows (P + 1 for the first cell, P afterwards); single
    // buffers suffice with two barriers per batch: a thread stores the next
    // batch only after the barrier that follows every thread's x-pass, and
    // overwrites bx only after the barrier that follows every thread's y-pass
    __shared__ S pl[P + 1][WP];
    __shared__ S bx[P + 1][WY * TX];

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

    // window loads of this thread: x-y offsets inside a z-plane
    int loff[LK];
#pragma unroll
    for (int k = 0; k < LK; ++k) {
        int e = tid + k * NT;
        e = e < WP ? e : WP - 1;                           // surplus lanes repeat the last element
        const int wx = e % WX, wy = e / WX;
        loff[k] = wrapi(Y0 + omy * P + wy, Ny) * Nx + wrapi(X0 + omx * P + wx, Nx);
    }
    // x-pass tasks: output (wy, tx) from window row wy, columns cx .. cx + P
    int xsrc[XK], xdst[XK];
    S xw[XK][P + 1];
#pragma unroll
    for (int k = 0; k < XK; ++k) {
        int e = tid + k * NT;
        e = e < Z::XT ? e : Z::XT - 1;
        const int tx = e % TX, wy = e / TX, l = tx % P;
        xsrc[k] = wy * WX + (tx / P + (l >= lsx ? 1 : 0)) * P;
        xdst[k] = wy * TX + tx;
#pragma unroll
        for (int r = 0; r <= P; ++r) xw[k][r] = Wx[l * (P + 1) + r];
    }
    // y-pass task and output of this thread: node (X0 + tx, Y0 + ty)
    const int tx = tid % TX, ty = tid / TX;
    const bool own = tid < TX * TY && X0 + tx < Nx && Y0 + ty < Ny;
    const int ly = ty % P;
    const int ysrc = (ty / P + (ly >= lsy ? 1 : 0)) * P * TX + (tid < TX * TY ? tx : 0);
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
    S raw[P + 1][LK];
    auto load_rows = [&](int k0, int nr) {
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            if (r < nr) {
                const int64_t zo = static_cast<int64_t>(wrapi(zb + k0 + r, Nz)) * NP;
#pragma unroll
                for (int j = 0; j < LK; ++j) raw[r][j] = src[zo + loff[j]];
            }
        }
    };
    // a batch of NR rows: registers -> LDS, loads of the next batch, x-pass, y-pass
    auto batch = [&](auto nr_c, int next_k0, int next_nr, S *res) {
        constexpr int NR = decltype(nr_c)::value;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int j = 0; j < LK; ++j)
                if (tid + j * NT < WP) pl[r][tid + j * NT] = raw[r][j];
        if (next_nr > 0) load_rows(next_k0, next_nr);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int k = 0; k < XK; ++k) {
                if (tid + k * NT < Z::XT) {
                    S acc = 0;
#pragma unroll
                    for (int m = 0; m <= P; ++m) acc = fma(xw[k][m], pl[r][xsrc[k] + m], acc);
                    bx[r][xdst[k]] = acc;
                }
            }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            S acc = 0;
#pragma unroll
            for (int m = 0; m <= P; ++m) acc = fma(yw[m], bx[r][ysrc + m * TX], acc);
            res[r] = acc;
        }
    };

    const int nel = ez1 - ez0;
    S a[2 * P + 1];
    load_rows(0, P + 1);
    batch(std::integral_constant<int, P + 1>(), P + 1, nel > 0 ? P : 0, a);
    for (int e = 0; e < nel; ++e) {
        const int ez = ez0 + e;
        batch(std::integral_constant<int, P>(), 2 * P + 1 + e * P, e + 1 < nel ? P : 0, a + P + 1);
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
    }
}

template <typename S, int P>
static hipError_t launch_z(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    using Z = ZTile<P>;
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
    hipLaunchKernelGGL((k_stream_z<S, P>), dim3(static_cast<unsigned>(nb)), dim3(Z::NT), 0, st, g, t, in, out, ntx,
                       ntiles, zcells, nchunk);
    return hipGetLastError();
}

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
