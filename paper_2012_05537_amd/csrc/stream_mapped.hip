// Semi-Lagrangian streaming on a distorted mesh (Sec. II A: departure points
// traced once through the cells; with distorted cells the interpolation does
// not factorise per axis and the paper's subsection "Numerical efficiency"
// expects a memory-bound kernel), and its transpose.
//
// The cells are the isoparametric images of the equal-cell reference grid
// (node displacements, build_mapped_tables); populations are interpolated in
// reference coordinates.  The host stores, per velocity and node, the
// departure cell and the three local coordinates (28 bytes in FP64, 16 in
// FP32); the weights are formed here ("matrix-free": 3 (P+1) Lagrange values
// instead of (P+1)^3 stored coefficients).  Three kernels:
//   * k_stream_mapped_win (the forward streaming): a block per velocity and
//     node tile stages the tile's source window in LDS and gathers from it;
//   * k_stream_mapped: the same gather straight from global memory, one
//     thread per (velocity, node) (the blocks of k_stream_mapped_win whose
//     window does not fit use the same summation);
//   * k_stream_mapped_t_cells / _nodes: the transpose in a fixed order.
// In k_stream_mapped, x-runs of P + 1 values are contiguous and neighbouring
// threads read neighbouring runs, so the gathers are served by L1/L2.  When
// rows and planes start on 16-byte boundaries and P is a multiple of the
// vector width V, the first P values of a run (never wrapped: the cell's
// first node plus P - 1 stays inside the row) are read as 16-byte vectors
// and only the last one, which wraps at the periodic end, on its own.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sllbm_internal.h"
#include "xcd.h"

namespace sllbm {

template <typename S, int V>
struct MVec {
    typedef S T __attribute__((ext_vector_type(V)));
};

template <typename S, int P, int V>
__global__ void __launch_bounds__(256) k_stream_mapped(Geometry g, GlcBasis gb, const int32_t *__restrict__ cell,
                                                       const S *__restrict__ tloc, const S *__restrict__ in,
                                                       S *__restrict__ out)
{
    const int i = blockIdx.y;
    const int64_t N = g.nodes;
    const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (n >= N) return;
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    const int c = cell[static_cast<int64_t>(i) * N + n];
    const int ex = c % g.nel[0], rest = c / g.nel[0];
    const int ey = rest % g.nel[1], ez = rest / g.nel[1];
    // Lagrange weights on the GLC points at the local coordinates
    S w[3][P + 1];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double t = static_cast<double>(tloc[(static_cast<int64_t>(a) * Q + i) * N + n]);
#pragma unroll
        for (int k = 0; k <= P; ++k) {
            double v = gb.inv_den[k];
#pragma unroll
            for (int m = 0; m <= P; ++m)
                if (m != k) v *= t - gb.t[m];
            w[a][k] = static_cast<S>(v);
        }
    }
    const S *fi = in + static_cast<int64_t>(i) * N;
    const S *gi = in + static_cast<int64_t>(Q + i) * N;
    S sf = 0, sg = 0;
#pragma unroll
    for (int kz = 0; kz <= P; ++kz) {
        int zz = ez * P + kz;
        zz = zz >= Nz ? zz - Nz : zz;
#pragma unroll
        for (int ky = 0; ky <= P; ++ky) {
            int yy = ey * P + ky;
            yy = yy >= Ny ? yy - Ny : yy;
            const int64_t row = (static_cast<int64_t>(zz) * Ny + yy) * Nx;
            S af = 0, ag = 0;
            if constexpr (V > 1) {
                using VT = typename MVec<S, V>::T;
                const int64_t x0 = row + ex * P;
#pragma unroll
                for (int k0 = 0; k0 < P; k0 += V) {
                    const VT vf = *reinterpret_cast<const VT *>(fi + x0 + k0);
                    const VT vg = *reinterpret_cast<const VT *>(gi + x0 + k0);
#pragma unroll
                    for (int c = 0; c < V; ++c) {
                        af = fma(w[0][k0 + c], vf[c], af);
                        ag = fma(w[0][k0 + c], vg[c], ag);
                    }
                }
                int xx = ex * P + P;
                xx = xx >= Nx ? xx - Nx : xx;
                af = fma(w[0][P], fi[row + xx], af);
                ag = fma(w[0][P], gi[row + xx], ag);
            } else {
#pragma unroll
                for (int kx = 0; kx <= P; ++kx) {
                    int xx = ex * P + kx;
                    xx = xx >= Nx ? xx - Nx : xx;
                    af = fma(w[0][kx], fi[row + xx], af);
                    ag = fma(w[0][kx], gi[row + xx], ag);
                }
            }
            const S wyz = w[1][ky] * w[2][kz];
            sf = fma(wyz, af, sf);
            sg = fma(wyz, ag, sg);
        }
    }
    out[static_cast<int64_t>(i) * N + n] = sf;
    out[static_cast<int64_t>(Q + i) * N + n] = sg;
}

// The same streaming with the source values staged in LDS: a block owns one
// velocity and a tile of MAPPED_TX x MAPPED_TY x MAPPED_TZ nodes; the host
// has found the box of cells that holds the departure cells of all of them
// (build_mapped_windows), the block loads that window once (coalesced rows,
// each value once from L2 instead of once per reading thread through L1),
// f and g of a node side by side so that one LDS read returns both, and every
// thread gathers its (P+1)^3 support pairs from LDS.  The blocks run in
// XCD-aware order (consecutive tiles of a velocity on one XCD, where their
// overlapping windows and the table lines they share meet in one L2).  A
// block whose window exceeds the LDS budget gathers from global memory
// instead; both paths sum in the same order, so they give the same bits.
template <typename S, int P>
__global__ void __launch_bounds__(256, MAPPED_MIN_WAVES) k_stream_mapped_win(
    Geometry g, GlcBasis gb, const int32_t *__restrict__ cell, const S *__restrict__ tloc,
    const int32_t *__restrict__ win, int ntiles, int ntx, int nty, const S *__restrict__ in, S *__restrict__ out)
{
    using S2 = typename MVec<S, 2>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = __builtin_amdgcn_readfirstlane(xcd_linear(blockIdx.x, gridDim.x));
    const int i = L / ntiles;
    const int t = L - i * ntiles;
    const int64_t N = g.nodes;
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    const int32_t *w = win + (static_cast<int64_t>(i) * ntiles + t) * 4;
    const int ocx = w[0], ocy = w[1], ocz = w[2], dims = w[3];
    const int gx = (t % ntx) * MAPPED_TX + (threadIdx.x % MAPPED_TX);
    const int gy = ((t / ntx) % nty) * MAPPED_TY + (threadIdx.x / MAPPED_TX) % MAPPED_TY;
    const int gz = (t / (ntx * nty)) * MAPPED_TZ + threadIdx.x / (MAPPED_TX * MAPPED_TY);
    const bool own = gx < Nx && gy < Ny && gz < Nz;
    const S *fi = in + static_cast<int64_t>(i) * N;
    const S *gi = in + static_cast<int64_t>(Q + i) * N;
    const int wx = dims & 1023, wy = (dims >> 10) & 1023, wz = dims >> 20;
    S2 *lw = reinterpret_cast<S2 *>(smem);
    if (dims != 0) {
        const int wt = wx * wy * wz;
        const int ox = ocx * P, oy = ocy * P, oz = ocz * P;
        const float rx = 1.0f / static_cast<float>(wx), ry = 1.0f / static_cast<float>(wy);
        for (int k = threadIdx.x; k < wt; k += blockDim.x) {
            // k = (z wy + y) wx + x.  The quotients in single precision are
            // exact: (k + 1/2)/wx lies at least 1/(2 wx) from an integer, and
            // the two roundings move it by less than that while k < 2^21
            // (a window holds at most a few thousand nodes).
            const int r = static_cast<int>((static_cast<float>(k) + 0.5f) * rx);
            const int z = static_cast<int>((static_cast<float>(r) + 0.5f) * ry);
            const int x = k - r * wx, y = r - z * wy;
            // origin node < N and window extent <= N + 1 along every axis
            int xx = ox + x, yy = oy + y, zz = oz + z;
            xx -= xx >= Nx ? Nx : 0;
            yy -= yy >= Ny ? Ny : 0;
            zz -= zz >= Nz ? Nz : 0;
            const int64_t node = (static_cast<int64_t>(zz) * Ny + yy) * Nx + xx;
            S2 v;
            v.x = fi[node];
            v.y = gi[node];
            lw[k] = v;
        }
        __syncthreads();
    }
    if (!own) return;
    const int64_t n = (static_cast<int64_t>(gz) * Ny + gy) * Nx + gx;
    const int c = cell[static_cast<int64_t>(i) * N + n];
    const int ex = c % g.nel[0], rest = c / g.nel[0];
    const int ey = rest % g.nel[1], ez = rest / g.nel[1];
    S wt3[3][P + 1];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double tt = static_cast<double>(tloc[(static_cast<int64_t>(a) * Q + i) * N + n]);
#pragma unroll
        for (int k = 0; k <= P; ++k) {
            double v = gb.inv_den[k];
#pragma unroll
            for (int m = 0; m <= P; ++m)
                if (m != k) v *= tt - gb.t[m];
            wt3[a][k] = static_cast<S>(v);
        }
    }
    S sf = 0, sg = 0;
    if (dims != 0) {
        int bx = ex - ocx, by = ey - ocy, bz = ez - ocz;       // the departure cell inside the window
        bx += bx < 0 ? g.nel[0] : 0;
        by += by < 0 ? g.nel[1] : 0;
        bz += bz < 0 ? g.nel[2] : 0;
#pragma unroll
        for (int kz = 0; kz <= P; ++kz)
#pragma unroll
            for (int ky = 0; ky <= P; ++ky) {
                const int base = ((bz * P + kz) * wy + by * P + ky) * wx + bx * P;
                S af = 0, ag = 0;
#pragma unroll
                for (int kx = 0; kx <= P; ++kx) {
                    const S2 v = lw[base + kx];
                    af = fma(wt3[0][kx], v.x, af);
                    ag = fma(wt3[0][kx], v.y, ag);
                }
                const S wyz = wt3[1][ky] * wt3[2][kz];
                sf = fma(wyz, af, sf);
                sg = fma(wyz, ag, sg);
            }
    } else {
#pragma unroll
        for (int kz = 0; kz <= P; ++kz) {
            int zz = ez * P + kz;
            zz = zz >= Nz ? zz - Nz : zz;
#pragma unroll
            for (int ky = 0; ky <= P; ++ky) {
                int yy = ey * P + ky;
                yy = yy >= Ny ? yy - Ny : yy;
                const int64_t row = (static_cast<int64_t>(zz) * Ny + yy) * Nx;
                S af = 0, ag = 0;
#pragma unroll
                for (int kx = 0; kx <= P; ++kx) {
                    int xx = ex * P + kx;
                    xx = xx >= Nx ? xx - Nx : xx;
                    af = fma(wt3[0][kx], fi[row + xx], af);
                    ag = fma(wt3[0][kx], gi[row + xx], ag);
                }
                const S wyz = wt3[1][ky] * wt3[2][kz];
                sf = fma(wyz, af, sf);
                sg = fma(wyz, ag, sg);
            }
        }
    }
    out[static_cast<int64_t>(i) * N + n] = sf;
    out[static_cast<int64_t>(Q + i) * N + n] = sg;
}

// Transposed streaming S^T on a distorted mesh, summed in a fixed order.
// Output n of velocity i read the (P+1)^3 support values of its departure
// cell c with the weights l_a(t_x) l_b(t_y) l_c(t_z); transposed, support
// point (a, b, c) of cell c receives the sum, over the nodes n departing into
// c, of the same weight times the adjoint of n.
//   Pass 1 (k_stream_mapped_t_cells): one block per (cell, velocity) forms
//   these (P+1)^3 partial sums for f and g, walking the cell's inverse list
//   (build_mapped_inverse) in increasing node order.
//   Pass 2 (k_stream_mapped_t_nodes): every node adds the partial sums of the
//   1, 2, 4 or 8 cells that share it, in a fixed order.
// No atomics: the result is the same bit for bit on every run.
template <int P>
constexpr int mt_threads()
{
    return ((P + 1) * (P + 1) * (P + 1) + 63) / 64 * 64;
}

template <typename S, int P>
__global__ void __launch_bounds__(mt_threads<P>()) k_stream_mapped_t_cells(
    Geometry g, GlcBasis gb, const int32_t *__restrict__ order, const int32_t *__restrict__ start,
    const S *__restrict__ tloc, const S *__restrict__ in, S *__restrict__ partial, int i0)
{
    constexpr int K = P + 1, K3 = K * K * K;
    constexpr int CH = 64;                                 // list entries staged per round
    __shared__ S lw[CH][3][K];
    __shared__ S ly[CH][2];
    const int c = blockIdx.x;
    const int C = static_cast<int>(gridDim.x);
    const int i = i0 + static_cast<int>(blockIdx.y);
    const int64_t N = g.nodes;
    const int32_t *st = start + static_cast<int64_t>(i) * (C + 1);
    const int b0 = st[c], b1 = st[c + 1];
    const int tid = threadIdx.x;
    const int a = tid % K, b = (tid / K) % K, e = tid / (K * K);   // this thread's support point
    S accf = 0, accg = 0;
    for (int base = b0; base < b1; base += CH) {
        const int nb = min(CH, b1 - base);
        if (tid < nb) {
            const int64_t n = order[static_cast<int64_t>(i) * N + base + tid];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const double tt = static_cast<double>(tloc[(static_cast<int64_t>(ax) * Q + i) * N + n]);
#pragma unroll
                for (int k = 0; k <= P; ++k) {
                    double v = gb.inv_den[k];
#pragma unroll
                    for (int m = 0; m <= P; ++m)
                        if (m != k) v *= tt - gb.t[m];
                    lw[tid][ax][k] = static_cast<S>(v);
                }
            }
            ly[tid][0] = in[static_cast<int64_t>(i) * N + n];
            ly[tid][1] = in[static_cast<int64_t>(Q + i) * N + n];
        }
        __syncthreads();
        if (tid < K3) {
            for (int k = 0; k < nb; ++k) {
                const S w = lw[k][0][a] * (lw[k][1][b] * lw[k][2][e]);
                accf = fma(w, ly[k][0], accf);
                accg = fma(w, ly[k][1], accg);
            }
        }
        __syncthreads();
    }
    if (tid < K3) {
        S *pp = partial + (static_cast<int64_t>(blockIdx.y) * C + c) * 2 * K3;
        pp[tid] = accf;
        pp[K3 + tid] = accg;
    }
}

template <typename S, int P>
__global__ void __launch_bounds__(256) k_stream_mapped_t_nodes(Geometry g, const S *__restrict__ partial,
                                                               S *__restrict__ out, int i0)
{
    constexpr int K = P + 1, K3 = K * K * K;
    const int i = i0 + static_cast<int>(blockIdx.y);
    const int64_t N = g.nodes;
    const int64_t m = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (m >= N) return;
    const int Nx = g.N[0], Ny = g.N[1];
    const int64_t NP = static_cast<int64_t>(Nx) * Ny;
    const int gz = static_cast<int>(m / NP), gy = static_cast<int>((m / Nx) % Ny), gx = static_cast<int>(m % Nx);
    const int C = g.nel[0] * g.nel[1] * g.nel[2];
    // along an axis node q lies in cell q / P at local point q % P, and when
    // q % P == 0 also in the previous cell (wrapped) at local point P
    int cs[3][2], ls[3][2], nc[3];
    const int gq[3] = {gx, gy, gz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int e = gq[ax] / P, l = gq[ax] - e * P;
        nc[ax] = 1;
        cs[ax][0] = e;
        ls[ax][0] = l;
        if (l == 0) {
            cs[ax][1] = e == 0 ? g.nel[ax] - 1 : e - 1;
            ls[ax][1] = P;
            nc[ax] = 2;
        }
    }
    const S *pb = partial + static_cast<int64_t>(blockIdx.y) * C * 2 * K3;
    S sf = 0, sg = 0;
    for (int z = 0; z < nc[2]; ++z)
        for (int y = 0; y < nc[1]; ++y)
            for (int x = 0; x < nc[0]; ++x) {
                const int c = (cs[2][z] * g.nel[1] + cs[1][y]) * g.nel[0] + cs[0][x];
                const int k = (ls[2][z] * K + ls[1][y]) * K + ls[0][x];
                const S *pp = pb + static_cast<int64_t>(c) * 2 * K3;
                sf += pp[k];
                sg += pp[K3 + k];
            }
    out[static_cast<int64_t>(i) * N + m] = sf;
    out[static_cast<int64_t>(Q + i) * N + m] = sg;
}

namespace {

template <typename S, int P>
hipError_t launch_mt(const Geometry &g, const MappedTables &t, const S *in, S *out, hipStream_t st)
{
    const int64_t cells = static_cast<int64_t>(g.nel[0]) * g.nel[1] * g.nel[2];
    const int64_t bx = (g.nodes + 255) / 256;
    if (bx > (int64_t(1) << 31) - 1 || cells > (int64_t(1) << 31) - 1 || !t.inv_order || !t.partial)
        return hipErrorInvalidValue;
    for (int i0 = 0; i0 < Q; i0 += t.qchunk) {
        const int qc = std::min(t.qchunk, Q - i0);
        hipLaunchKernelGGL((k_stream_mapped_t_cells<S, P>), dim3(static_cast<unsigned>(cells), qc),
                           dim3(mt_threads<P>()), 0, st, g, t.basis, t.inv_order, t.inv_start,
                           static_cast<const S *>(t.tloc), in, static_cast<S *>(t.partial), i0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_stream_mapped_t_nodes<S, P>), dim3(static_cast<unsigned>(bx), qc), dim3(256), 0, st, g,
                           static_cast<const S *>(t.partial), out, i0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename S, int P>
hipError_t launch_m(const Geometry &g, const MappedTables &t, const S *in, S *out, hipStream_t st)
{
    if (t.win) {
        const int ntx = (g.N[0] + MAPPED_TX - 1) / MAPPED_TX, nty = (g.N[1] + MAPPED_TY - 1) / MAPPED_TY,
                  ntz = (g.N[2] + MAPPED_TZ - 1) / MAPPED_TZ;
        const int64_t ntiles = static_cast<int64_t>(ntx) * nty * ntz;
        if (ntiles * Q > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
        const size_t lds = 2 * static_cast<size_t>(t.win_nodes) * sizeof(S);
        hipLaunchKernelGGL((k_stream_mapped_win<S, P>), dim3(static_cast<unsigned>(ntiles * Q)), dim3(256), lds, st,
                           g, t.basis, t.cell, static_cast<const S *>(t.tloc), t.win, static_cast<int>(ntiles), ntx,
                           nty, in, out);
        return hipGetLastError();
    }
    const int64_t bx = (g.nodes + 255) / 256;
    if (bx > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    constexpr int V = 16 / sizeof(S);
    // 16-byte loads: every plane (N values) and row (N_x values) starts on a
    // 16-byte boundary, and a cell's first node is a multiple of V
    const bool aligned = (g.nodes * sizeof(S)) % 16 == 0 && (g.N[0] * sizeof(S)) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(in) % 16 == 0;
    if constexpr (P % V == 0) {
        if (aligned) {
            hipLaunchKernelGGL((k_stream_mapped<S, P, V>), dim3(static_cast<unsigned>(bx), Q), dim3(256), 0, st, g,
                               t.basis, t.cell, static_cast<const S *>(t.tloc), in, out);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_stream_mapped<S, P, 1>), dim3(static_cast<unsigned>(bx), Q), dim3(256), 0, st, g, t.basis,
                       t.cell, static_cast<const S *>(t.tloc), in, out);
    return hipGetLastError();
}

}  // namespace

template <typename S>
hipError_t launch_stream_mapped(const Geometry &g, const MappedTables &t, const S *in, S *out, hipStream_t st)
{
    switch (g.p) {
    case 1: return launch_m<S, 1>(g, t, in, out, st);
    case 2: return launch_m<S, 2>(g, t, in, out, st);
    case 3: return launch_m<S, 3>(g, t, in, out, st);
    case 4: return launch_m<S, 4>(g, t, in, out, st);
    case 5: return launch_m<S, 5>(g, t, in, out, st);
    case 6: return launch_m<S, 6>(g, t, in, out, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename S>
hipError_t launch_stream_mapped_t(const Geometry &g, const MappedTables &t, const S *in, S *out, hipStream_t st)
{
    switch (g.p) {
    case 1: return launch_mt<S, 1>(g, t, in, out, st);
    case 2: return launch_mt<S, 2>(g, t, in, out, st);
    case 3: return launch_mt<S, 3>(g, t, in, out, st);
    case 4: return launch_mt<S, 4>(g, t, in, out, st);
    case 5: return launch_mt<S, 5>(g, t, in, out, st);
    case 6: return launch_mt<S, 6>(g, t, in, out, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stream_mapped_t<double>(const Geometry &, const MappedTables &, const double *, double *,
                                                   hipStream_t);
template hipError_t launch_stream_mapped_t<float>(const Geometry &, const MappedTables &, const float *, float *,
                                                  hipStream_t);
template hipError_t launch_stream_mapped<double>(const Geometry &, const MappedTables &, const double *, double *,
                                                 hipStream_t);
template hipError_t launch_stream_mapped<float>(const Geometry &, const MappedTables &, const float *, float *,
                                                hipStream_t);

}  // namespace sllbm
