// Two-dimensional semi-Lagrangian streaming (Sec. II A, Eqs. (8)-(9) with
// D = 2) on a periodic mesh of equal cells: the D2Q19 counterpart of the
// z-march of stream.hip, marching along y.
//
// For velocity i the interpolant factorises into two 1-D operators; along an
// axis output node e*P + l reads source cell e + o_l (o_l = omin for l <
// lstar, omin + 1 otherwise) with the weight row of l.  A block owns one
// (velocity, population) plane over an x-strip of TX nodes (whole cells) and
// a chunk of cells along y:
//   * each source row of the strip's window (TX + P + 1 nodes, 16-byte loads
//     when the rows allow) is loaded once, the next batch of rows being in
//     flight while the current one is interpolated along x out of LDS (one
//     output column per thread, two LDS buffers, one barrier per batch);
//   * a thread keeps the x-interpolated values of the two source cells that
//     output cell e reads along y (2P + 1 rows) in registers, forms the P
//     outputs of the cell with the velocity's uniform y weights and slides
//     by one cell.
// Rows are 2 KB long (FP64), so every load and store is a long coalesced
// run; the x halo (P + 1 nodes) and the P + 1 rows a y-chunk re-reads are
// the only reads beyond the algorithmic ones.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sllbm_internal.h"
#include "xcd.h"

namespace sllbm {

namespace {

constexpr int Y_TARGET_BLOCKS = 1024;      // 512^2 nodes: 16-cell chunks, 608 blocks (2048: 5 % slower in FP64)
constexpr int Y_MIN_CELLS = 4;

__device__ __forceinline__ int wrap2(int x, int n)
{
    int r = x % n;
    return r < 0 ? r + n : r;
}

template <int P, int V>
struct YStrip {
    static constexpr int NT = 256;                        // threads: one output column each
    static constexpr int TXC = NT / P;                    // cells per strip
    static constexpr int TX = TXC * P;                    // nodes per strip
    static constexpr int WX = TX + P + 1;                 // source window of a row
    static constexpr int WXC = (WX + V - 1) / V;          // loads per row
    static constexpr int WXP = WXC * V;                   // padded LDS row
    static constexpr int LK = (WXC + NT - 1) / NT;        // loads per thread and row
};

template <typename S, int V>
struct Vec2 {
    typedef S T __attribute__((ext_vector_type(V)));
};
template <typename S>
struct Vec2<S, 1> {
    typedef S T;
};

}  // namespace

template <typename S, int P, int V>
__global__ void __launch_bounds__(256) k_stream_y(Geometry g, CellTables<S> tab, const S *__restrict__ in,
                                                  S *__restrict__ out, int nstrip, int ycells, int nchunk)
{
    using Y = YStrip<P, V>;
    using VT = typename Vec2<S, V>::T;
    constexpr int NT = Y::NT, TX = Y::TX, WXP = Y::WXP, WXC = Y::WXC, LK = Y::LK;
    // two buffers of one batch of rows (P + 1 for the first cell, P afterwards)
    __shared__ __align__(16) S pl[2][P + 1][WXP];

    const int tid = threadIdx.x;
    const int L = __builtin_amdgcn_readfirstlane(xcd_linear(blockIdx.x, gridDim.x));
    const int q = L / (nstrip * nchunk);
    const int rem = L - q * nstrip * nchunk;
    const int chunk = rem / nstrip, strip = rem - chunk * nstrip;
    const int i = q % Q2D, pop = q / Q2D;
    const int X0 = strip * TX;
    const int Nx = g.N[0], Ny = g.N[1];
    const int64_t N = g.nodes;
    const int omx = tab.omin[i * 3 + 0], omy = tab.omin[i * 3 + 1];
    const int lsx = tab.lstar[i * 3 + 0], lsy = tab.lstar[i * 3 + 1];
    const S *Wx = tab.w + (i * 3 + 0) * P * (P + 1);
    const S *Wy = tab.w + (i * 3 + 1) * P * (P + 1);
    const S *__restrict__ src = in + static_cast<int64_t>(pop * Q2D + i) * N;
    S *__restrict__ dst = out + static_cast<int64_t>(pop * Q2D + i) * N;

    // window loads of this thread: columns V*e .. V*e + V-1 of the window,
    // which starts at source cell X0/P + omx
    int loff[LK];
#pragma unroll
    for (int k = 0; k < LK; ++k) {
        int e = tid + k * NT;
        e = e < WXC ? e : WXC - 1;                         // surplus lanes repeat the last load
        loff[k] = wrap2(X0 + omx * P + V * e, Nx);
    }
    // x-pass of this thread's output column X0 + tid: LDS offset of its
    // source cell and its weight row
    const int lx = tid % P;
    const int xsrc = tid < TX ? (tid / P + (lx >= lsx ? 1 : 0)) * P : 0;   // surplus lanes read row start
    const bool own = tid < TX && X0 + tid < Nx;
    S xw[P + 1];
#pragma unroll
    for (int r = 0; r <= P; ++r) xw[r] = Wx[lx * (P + 1) + r];
    S wy[P][P + 1];                                       // uniform y weights of this velocity
#pragma unroll
    for (int l = 0; l < P; ++l)
#pragma unroll
        for (int r = 0; r <= P; ++r) wy[l][r] = Wy[l * (P + 1) + r];

    // output cells [ey0, ey1) along y; source rows in march order:
    // y = (ey0 + omy) * P + k (mod Ny), k = 0 .. P + (ey1 - ey0) * P
    const int ey0 = chunk * ycells, ey1 = min(g.nel[1], ey0 + ycells);
    const int yb = (ey0 + omy) * P;
    VT raw[P + 1][LK];
    auto load_rows = [&](int k0, int nr) {
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            if (r < nr) {
                const int64_t yo = static_cast<int64_t>(wrap2(yb + k0 + r, Ny)) * Nx;
#pragma unroll
                for (int j = 0; j < LK; ++j) raw[r][j] = *reinterpret_cast<const VT *>(src + yo + loff[j]);
            }
        }
    };
    // a batch of nr rows: registers -> LDS buffer b, the registers reloaded
    // with the next batch, one barrier, the x-pass of every row
    int b = 0;
    auto batch = [&](auto nr_c, int next_k0, int next_nr, S *res) {
        constexpr int NR = decltype(nr_c)::value;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int j = 0; j < LK; ++j)
                if (tid + j * NT < WXC) *reinterpret_cast<VT *>(&pl[b][r][V * (tid + j * NT)]) = raw[r][j];
        if (next_nr > 0) load_rows(next_k0, next_nr);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const S *c = &pl[b][r][xsrc];
            S acc = 0;
#pragma unroll
            for (int m = 0; m <= P; ++m) acc = fma(xw[m], c[m], acc);
            res[r] = acc;
        }
        b ^= 1;
    };
    // P outputs of cell ey along y from the rows in a, then slide by one cell
    S a[2 * P + 1];
    auto emit = [&](int ey) {
        if (own) {
#pragma unroll
            for (int l = 0; l < P; ++l) {
                const bool hi = l >= lsy;
                S acc = 0;
#pragma unroll
                for (int r = 0; r <= P; ++r) acc = fma(wy[l][r], hi ? a[P + r] : a[r], acc);
                dst[static_cast<int64_t>(ey * P + l) * Nx + X0 + tid] = acc;
            }
        }
#pragma unroll
        for (int r = 0; r <= P; ++r) a[r] = a[r + P];
    };

    const int nel = ey1 - ey0;
    auto rows_of = [&](int e) { return e < nel ? P : 0; };
    load_rows(0, P + 1);
    batch(std::integral_constant<int, P + 1>(), P + 1, rows_of(0), a);
    for (int e = 0; e < nel; ++e) {
        batch(std::integral_constant<int, P>(), P + 1 + (e + 1) * P, rows_of(e + 1), a + P + 1);
        emit(ey0 + e);
    }
}

namespace {

template <typename S, int P, int V>
hipError_t launch_yv(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    using Y = YStrip<P, V>;
    const int nstrip = (g.N[0] + Y::TX - 1) / Y::TX;
    // split the y-march into chunks until the grid has a few blocks per CU
    // slot (each chunk re-reads P + 1 source rows)
    int nchunk = 1;
    while (nchunk < g.nel[1] && static_cast<int64_t>(nstrip) * 2 * Q2D * nchunk < Y_TARGET_BLOCKS &&
           g.nel[1] / (2 * nchunk) >= Y_MIN_CELLS)
        nchunk *= 2;
    const int ycells = (g.nel[1] + nchunk - 1) / nchunk;
    nchunk = (g.nel[1] + ycells - 1) / ycells;
    const int64_t nb = static_cast<int64_t>(nstrip) * 2 * Q2D * nchunk;
    if (nb > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stream_y<S, P, V>), dim3(static_cast<unsigned>(nb)), dim3(Y::NT), 0, st, g, t, in, out,
                       nstrip, ycells, nchunk);
    return hipGetLastError();
}

// 16-byte window loads when every window row starts on a 16-byte boundary
template <typename S, int P>
hipError_t launch_y(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    constexpr int V = 16 / sizeof(S);
    const bool aligned = (g.N[0] * sizeof(S)) % 16 == 0 && reinterpret_cast<uintptr_t>(in) % 16 == 0;
    if constexpr ((P * sizeof(S)) % 16 == 0 && YStrip<P, V>::TX % V == 0) {
        if (aligned) return launch_yv<S, P, V>(g, t, in, out, st);
    }
    return launch_yv<S, P, 1>(g, t, in, out, st);
}

}  // namespace

template <typename S>
hipError_t launch_stream_2d(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st)
{
    switch (g.p) {
    case 1: return launch_y<S, 1>(g, t, in, out, st);
    case 2: return launch_y<S, 2>(g, t, in, out, st);
    case 3: return launch_y<S, 3>(g, t, in, out, st);
    case 4: return launch_y<S, 4>(g, t, in, out, st);
    case 5: return launch_y<S, 5>(g, t, in, out, st);
    case 6: return launch_y<S, 6>(g, t, in, out, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stream_2d<double>(const Geometry &, const CellTables<double> &, const double *, double *,
                                             hipStream_t);
template hipError_t launch_stream_2d<float>(const Geometry &, const CellTables<float> &, const float *, float *,
                                            hipStream_t);

}  // namespace sllbm
