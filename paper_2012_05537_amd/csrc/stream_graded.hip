// Semi-Lagrangian streaming (Sec. II A, Eqs. (8)-(9)) on a graded mesh:
// periodic, axis-aligned cells of unequal width.
//
// The departure point of every node still factorises per axis, but the
// departure cell and the 1-D Lagrange weights now depend on the node, not
// only on its local point: each axis carries per-node tables (first source
// node, p + 1 weights), built once per mesh.  Along an axis the first source
// node is non-decreasing in the output node, so the source window of an x-y
// tile is one contiguous (wrapped) range per axis.
//
// A block owns one (velocity, population) plane over a 32 x 8 x-y tile and a
// range of output z-rows.  It walks the source z-rows in order, two at a
// time: it stores their tile windows (loaded into registers while the
// previous two rows were processed) in LDS, interpolates along x (per-thread
// taps) and then along y, and keeps the results in a per-thread ring of
// source rows, from which each output z-row takes its p + 1 taps.
// Every source row is read once per plane and tile column of the chunk.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sllbm_internal.h"
#include "xcd.h"

namespace sllbm {

namespace {

__device__ __forceinline__ int wrapg(int x, int n)
{
    int r = x % n;
    return r < 0 ? r + n : r;
}

constexpr int GTX = 32, GTY = 8, GNT = GTX * GTY;
constexpr int GRB = 2;                         // source z-rows interpolated per batch
constexpr int64_t GRADED_TARGET_BLOCKS = 2048;

}  // namespace

template <typename S, int V>
struct VecG {
    typedef S T __attribute__((ext_vector_type(V)));
};
template <typename S>
struct VecG<S, 1> {
    typedef S T;
};

template <typename S, int K, int LK, int V>
__global__ void __launch_bounds__(GNT) k_stream_graded(Geometry g, NodeTables<S> tab, const S *__restrict__ in,
                                                        S *__restrict__ out, int ntile_x, int ntiles, int zrows,
                                                        int nchunk)
{
    constexpr int RB = GRB;                                // source rows per batch (two barriers each)
    constexpr int RZ = K - 1 + RB;                         // ring of source rows per thread
    constexpr int AS = GTX + 1;                            // odd row stride of the x-pass result
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wxm = tab.wxm, wym = tab.wym;
    const int WP = wym * wxm, AP = wym * AS;
    S *pl = reinterpret_cast<S *>(smem_raw);               // [RB][wym][wxm] source windows of a batch
    S *A = pl + RB * WP;                                   // [RB][wym][AS] x-interpolated rows
    S *ring = A + RB * AP;                                 // [RZ][GNT]     x-y interpolated source rows

    const int tid = threadIdx.x;
    const int L = __builtin_amdgcn_readfirstlane(xcd_linear(blockIdx.x, gridDim.x));
    const int q = L / (ntiles * nchunk);
    const int rem = L - q * ntiles * nchunk;
    const int chunk = rem / ntiles, tile = rem - chunk * ntiles;
    const int i = q >> 1, pop = q & 1;
    const int X0 = (tile % ntile_x) * GTX, Y0 = (tile / ntile_x) * GTY;
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    const int64_t N = g.nodes, NP = static_cast<int64_t>(Nx) * Ny;
    const int32_t *sx = tab.src[0] + static_cast<int64_t>(i) * Nx;
    const int32_t *sy = tab.src[1] + static_cast<int64_t>(i) * Ny;
    const int32_t *sz = tab.src[2] + static_cast<int64_t>(i) * Nz;
    const S *wxt = tab.w[0] + static_cast<int64_t>(i) * Nx * K;
    const S *wyt = tab.w[1] + static_cast<int64_t>(i) * Ny * K;
    const S *wzt = tab.w[2] + static_cast<int64_t>(i) * Nz * K;
    const S *__restrict__ src = in + static_cast<int64_t>(pop * 45 + i) * N;
    S *__restrict__ dst = out + static_cast<int64_t>(pop * 45 + i) * N;

    // source window of the tile (first source nodes are non-decreasing); its
    // x start is rounded down to V nodes (shift sh) for V-wide loads
    using VT = typename VecG<S, V>::T;
    const int xs = sx[X0], wxb = sx[min(X0 + GTX, Nx) - 1] - xs + K;
    const int sh = ((xs % V) + V) % V, xs0 = xs - sh;
    const int wxv = (wxb + sh + V - 1) / V;                // V-wide loads per window row
    const int ys0 = sy[Y0], wyb = sy[min(Y0 + GTY, Ny) - 1] - ys0 + K;
    const int nwin = wxv * wyb;                            // <= LK * GNT (checked by the launcher)
    // this thread's window loads: offset inside a z-plane and in LDS
    int loff[LK], soff[LK];
#pragma unroll
    for (int k = 0; k < LK; ++k) {
        const int e = min(tid + k * GNT, nwin - 1);
        const int wy_ = e / wxv, wx_ = (e - wy_ * wxv) * V;
        loff[k] = wrapg(ys0 + wy_, Ny) * Nx + wrapg(xs0 + wx_, Nx);
        soff[k] = wy_ * wxm + wx_;
    }

    // taps of this thread's output column (clamped on ragged tiles, not stored)
    const int tx = tid % GTX, ty = tid / GTX;
    const bool own = X0 + tx < Nx && Y0 + ty < Ny;
    const int gx = min(X0 + tx, Nx - 1), gy = min(Y0 + ty, Ny - 1);
    const int ox = sx[gx] - xs0, oy = sy[gy] - ys0;        // ox includes the shift sh
    S wx[K], wy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        wx[k] = wxt[gx * K + k];
        wy[k] = wyt[gy * K + k];
    }
    const int64_t oxy = static_cast<int64_t>(gy) * Nx + gx;

    const int zo0 = chunk * zrows, zo1 = min(Nz, zo0 + zrows);
    const int r0 = sz[zo0];                                // first source row of the chunk (not wrapped)
    // the windows of the next batch of source rows are loaded into registers
    // while the current batch is interpolated
    VT raw[RB][LK];
    auto load_batch = [&](int r) {
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const S *base = src + static_cast<int64_t>(wrapg(r + b, Nz)) * NP;
#pragma unroll
            for (int k = 0; k < LK; ++k) raw[b][k] = *reinterpret_cast<const VT *>(base + loff[k]);
        }
    };
    load_batch(r0);
    int rnext = r0;                                        // first source row not yet in the ring
    for (int zo = zo0; zo < zo1; ++zo) {
        const int s = sz[zo];
        // bring in batches until row s + K - 1 is in the ring; the ring then
        // holds rows s .. s + K - 1 (older rows are no longer needed)
        for (; rnext <= s + K - 1; rnext += RB) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int k = 0; k < LK; ++k)
                    if (tid + k * GNT < nwin) *reinterpret_cast<VT *>(&pl[b * WP + soff[k]]) = raw[b][k];
            load_batch(rnext + RB);                        // in bounds (wrapped); unused past the chunk
            __syncthreads();
#pragma unroll
            for (int b = 0; b < RB; ++b)
                for (int wy_ = ty; wy_ < wyb; wy_ += GTY) {
                    S acc = 0;
#pragma unroll
                    for (int k = 0; k < K; ++k) acc = fma(wx[k], pl[b * WP + wy_ * wxm + ox + k], acc);
                    A[b * AP + wy_ * AS + tx] = acc;
                }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                S acc = 0;
#pragma unroll
                for (int k = 0; k < K; ++k) acc = fma(wy[k], A[b * AP + (oy + k) * AS + tx], acc);
                ring[((rnext + b - r0) % RZ) * GNT + tid] = acc;
            }
        }
        S acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            acc = fma(wzt[zo * K + k], ring[((s + k - r0) % RZ) * GNT + tid], acc);
        if (own) dst[static_cast<int64_t>(zo) * NP + oxy] = acc;
    }
}

size_t graded_smem_bytes(int taps, int wxm, int wym, size_t elem)
{
    return (GRB * (static_cast<size_t>(wym) * wxm + static_cast<size_t>(wym) * (GTX + 1)) +
            static_cast<size_t>(taps - 1 + GRB) * GNT) * elem;
}

// largest source window of a 32 x 8 tile along an axis (tile extent T)
int graded_window(const int32_t *src, int N, int taps, int T)
{
    int w = 0;
    for (int t0 = 0; t0 < N; t0 += T) w = std::max(w, src[std::min(t0 + T, N) - 1] - src[t0] + taps);
    return w;
}

int graded_taps_supported(int taps)
{
    static const int ks[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24};
    for (int k : ks)
        if (k >= taps) return k;
    return 0;
}

int graded_tile_x() { return GTX; }
int graded_window_pad(size_t elem) { return static_cast<int>(16 / elem); }
int graded_max_window() { return 16 * GNT; }
int graded_tile_y() { return GTY; }

template <typename S, int K, int LK, int V>
static hipError_t launch_gk(const Geometry &g, const NodeTables<S> &t, const S *in, S *out, hipStream_t st)
{
    const int ntx = (g.N[0] + GTX - 1) / GTX, nty = (g.N[1] + GTY - 1) / GTY;
    const int ntiles = ntx * nty;
    // split the z-march into chunks (each re-reads p source rows) until the
    // grid has a few blocks per CU slot
    int nchunk = 1;
    while (static_cast<int64_t>(ntiles) * 90 * nchunk < GRADED_TARGET_BLOCKS && g.N[2] / (2 * nchunk) >= 4 * K)
        nchunk *= 2;
    const int zrows = (g.N[2] + nchunk - 1) / nchunk;
    nchunk = (g.N[2] + zrows - 1) / zrows;
    const int64_t nb = static_cast<int64_t>(ntiles) * 90 * nchunk;
    if (nb > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    const size_t smem = graded_smem_bytes(K, t.wxm, t.wym, sizeof(S));
    if (smem > 160 * 1024) return hipErrorInvalidValue;
    if (smem > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_stream_graded<S, K, LK, V>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_stream_graded<S, K, LK, V>), dim3(static_cast<unsigned>(nb)), dim3(GNT), smem, st, g, t, in,
                       out, ntx, ntiles, zrows, nchunk);
    return hipGetLastError();
}

// window loads per thread: the smallest LK with LK * 256 >= the largest window
template <typename S, int K, int V>
static hipError_t launch_gv(const Geometry &g, const NodeTables<S> &t, const S *in, S *out, hipStream_t st)
{
    const int nw = (t.wxm / V) * t.wym;                    // V-wide loads of the largest window
    if (nw <= 1 * GNT) return launch_gk<S, K, 1, V>(g, t, in, out, st);
    if (nw <= 2 * GNT) return launch_gk<S, K, 2, V>(g, t, in, out, st);
    if (nw <= 4 * GNT) return launch_gk<S, K, 4, V>(g, t, in, out, st);
    if (nw <= 8 * GNT) return launch_gk<S, K, 8, V>(g, t, in, out, st);
    if (nw <= 16 * GNT) return launch_gk<S, K, 16, V>(g, t, in, out, st);
    return hipErrorInvalidValue;
}

// 16-byte window loads when x rows hold a multiple of 16 bytes and the
// buffer is 16-byte aligned (the window start is rounded down)
template <typename S, int K>
static hipError_t launch_g(const Geometry &g, const NodeTables<S> &t, const S *in, S *out, hipStream_t st)
{
    constexpr int V = 16 / sizeof(S);
    if ((g.N[0] * sizeof(S)) % 16 == 0 && reinterpret_cast<uintptr_t>(in) % 16 == 0 && t.wxm % V == 0)
        return launch_gv<S, K, V>(g, t, in, out, st);
    return launch_gv<S, K, 1>(g, t, in, out, st);
}

// taps per output: p + 1 for the forward tables, the padded band width of
// the transposed ones (graded_taps_supported)
template <typename S>
hipError_t launch_stream_graded(const Geometry &g, const NodeTables<S> &t, const S *in, S *out, hipStream_t st)
{
    switch (t.k) {
    case 2: return launch_g<S, 2>(g, t, in, out, st);
    case 3: return launch_g<S, 3>(g, t, in, out, st);
    case 4: return launch_g<S, 4>(g, t, in, out, st);
    case 5: return launch_g<S, 5>(g, t, in, out, st);
    case 6: return launch_g<S, 6>(g, t, in, out, st);
    case 7: return launch_g<S, 7>(g, t, in, out, st);
    case 8: return launch_g<S, 8>(g, t, in, out, st);
    case 10: return launch_g<S, 10>(g, t, in, out, st);
    case 12: return launch_g<S, 12>(g, t, in, out, st);
    case 14: return launch_g<S, 14>(g, t, in, out, st);
    case 16: return launch_g<S, 16>(g, t, in, out, st);
    case 20: return launch_g<S, 20>(g, t, in, out, st);
    case 24: return launch_g<S, 24>(g, t, in, out, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stream_graded<double>(const Geometry &, const NodeTables<double> &, const double *,
                                                 double *, hipStream_t);
template hipError_t launch_stream_graded<float>(const Geometry &, const NodeTables<float> &, const float *, float *,
                                                hipStream_t);

}  // namespace sllbm
