// Band Fast Hough Transform for mostly vertical lines (Section 2.1).
//
// Every band of n = 2^p rows is zero-extended to the right by n columns and
// transformed with the dyadic shift-and-add recursion: stage j merges pairs of
// row blocks of 2^(j-1) rows into blocks of 2^j rows,
//
//   T_j(b, c, s) = T_{j-1}(2b, c, s/2) + T_{j-1}(2b+1, c + ceil(s/2), s/2)   (s/2 rounded down),
//
// so after p stages T_p(0, c, s) is the sum along the dyadic line that starts
// at column c and is displaced by s over the band.  Left-leaning lines are the
// same recursion on the band mirrored about its (cyclic) width, so both
// directions share one code path ("c-space": c = x for right-leaning lines,
// c = W-1-x for left-leaning ones).  Work per band and direction is p*n*W
// additions, the O((w + h/k) * (h/k) * log(h/k)) cost of Section 2.1.
//
// Layout on gfx950: one thread owns one c-space column and keeps the n running
// sums of that column in VGPRs through all p stages; the operand that comes
// from another column (c + ceil(s/2)) is exchanged through LDS once per
// stage.  A workgroup of NT threads covers NT columns and produces the
// NT - (n-1) leftmost of them (the rest are its halo).  Global loads and table
// stores are coalesced along x.  Bands taller than 2^7 rows run the same kernel
// on 128-row sub-blocks, then a second kernel adds the sub-blocks along the
// coarse levels of the recursion.
#include "fhtp_internal.h"

namespace fhtp {
namespace {

// Column offset of row y on the dyadic line of shift s over 2^p rows: bit
// (p-1-j) of y contributes ceil((s >> j) / 2).
__device__ __forceinline__ int dyadic_offset(int p, int s, int y) {
    int off = 0;
    for (int j = 0; j < p; ++j)
        if ((y >> (p - 1 - j)) & 1) off += (s >> (j + 1)) + ((s >> j) & 1);
    return off;
}

template <int P>
struct RegCfg {
    static constexpr int N = 1 << P;
    static constexpr int NT = (P >= 7) ? 512 : 256;
    static constexpr int T = NT - (N - 1);             // columns produced per workgroup
    static constexpr int HALF = (N >= 2) ? N / 2 : 1;
    static constexpr int LW = NT + HALF;               // LDS row width (halo reads stay inside)
    static constexpr int LDS_WORDS = (N >= 2) ? (N / 2) * LW : 1;
};

// One stage of the recursion on the column held in v.
template <int N, int J, int LW>
__device__ __forceinline__ void fht_stage(int32_t (&v)[N], int32_t* lds, int tid) {
    constexpr int half = 1 << (J - 1);
    constexpr int blocks = N >> J;
    __syncthreads();  // the previous stage's LDS reads are complete
#pragma unroll
    for (int b = 0; b < blocks; ++b)
#pragma unroll
        for (int t = 0; t < half; ++t) lds[(b * half + t) * LW + tid] = v[b * 2 * half + half + t];
    __syncthreads();
    int32_t nv[N];
#pragma unroll
    for (int b = 0; b < blocks; ++b) {
#pragma unroll
        for (int t = 0; t < half; ++t) {
            const int32_t a = v[b * 2 * half + t];
            const int32_t* row = lds + (b * half + t) * LW + tid + t;
            nv[b * 2 * half + 2 * t] = a + row[0];
            nv[b * 2 * half + 2 * t + 1] = a + row[1];
        }
    }
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = nv[q];
}

template <int N, int J, int P, int LW>
__device__ __forceinline__ void fht_stages(int32_t (&v)[N], int32_t* lds, int tid) {
    if constexpr (J <= P) {
        fht_stage<N, J, LW>(v, lds, tid);
        fht_stages<N, J + 1, P, LW>(v, lds, tid);
    }
}

// Grid: x = block * tiles + tile over row blocks of 2^P rows, y = direction
// (0 right-leaning, 1 left-leaning).  Output modes:
//   to_table: tables[blk][n-1 +- s][x] of a band of n = 2^P rows (d = 0 only from y = 0);
//   else:     scratch[(blk*2 + dir)*2^P + s][c] in c-space (pass 1 of tall bands).
template <int P, typename PixT>
__global__ __launch_bounds__(RegCfg<P>::NT) void fht_reg_kernel(const PixT* __restrict__ img,
                                                                int w, int W, int tiles,
                                                                int32_t* __restrict__ out,
                                                                int to_table) {
    using C = RegCfg<P>;
    constexpr int N = C::N;
    __shared__ int32_t lds[C::LDS_WORDS];

    const int tid = threadIdx.x;
    const int tile = blockIdx.x % tiles;
    const int blk = blockIdx.x / tiles;
    const int dir = blockIdx.y;
    const int c = tile * C::T + tid;
    const int cm = c % W;
    const int ximg = dir == 0 ? cm : (W - 1 - cm);

    int32_t v[N];
    const PixT* src = img + (size_t)blk * N * (size_t)w;
    const bool inside = ximg < w;
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = inside ? (int32_t)src[(size_t)y * w + ximg] : 0;

    fht_stages<N, 1, P, C::LW>(v, lds, tid);

    if (tid >= C::T || c >= W) return;
    if (to_table) {
        constexpr int D = 2 * N - 1;
        const int xo = dir == 0 ? c : (W - 1 - c);
        int32_t* base = out + (size_t)blk * D * (size_t)W + xo;
#pragma unroll
        for (int s = 0; s < N; ++s) {
            if (dir == 0) {
                base[(size_t)(N - 1 + s) * W] = v[s];
            } else if (s > 0) {
                base[(size_t)(N - 1 - s) * W] = v[s];
            }
        }
    } else {
        int32_t* base = out + (size_t)(blk * 2 + dir) * N * (size_t)W + c;
#pragma unroll
        for (int s = 0; s < N; ++s) base[(size_t)s * W] = v[s];
    }
}

// Pass 2 for bands of n = 2^p > 2^7 rows: the band is M = n/128 sub-blocks whose
// FHTs (fine shift sf = s >> (p-7)) sit in `sub`; the line of shift s starts in
// sub-block m at c + D_s(m*128), so T(c, s) = sum_m sub[m][sf][(c + D_s(128 m)) mod W].
__global__ __launch_bounds__(256) void fht_combine_kernel(const int32_t* __restrict__ sub,
                                                          int p, int W, int tiles_x,
                                                          int32_t* __restrict__ tables) {
    const int n = 1 << p;
    const int D = 2 * n - 1;
    const int M = n >> kRegMaxP;
    const int sh = p - kRegMaxP;
    const int tile = blockIdx.x % tiles_x;
    const int s = blockIdx.x / tiles_x;
    const int dir = blockIdx.y;
    const int band = blockIdx.z;
    const int c = tile * 256 + threadIdx.x;
    if (c >= W || (dir == 1 && s == 0)) return;
    const int sf = s >> sh;
    int32_t acc = 0;
    for (int m = 0; m < M; ++m) {
        int cc = c + dyadic_offset(p, s, m << kRegMaxP);
        cc %= W;
        acc += sub[((size_t)((band * M + m) * 2 + dir) * (1 << kRegMaxP) + sf) * W + cc];
    }
    const int xo = dir == 0 ? c : (W - 1 - c);
    const int r = dir == 0 ? (n - 1 + s) : (n - 1 - s);
    tables[((size_t)band * D + r) * W + xo] = acc;
}

template <int P, typename PixT>
hipError_t launch_reg(const PixT* img, int w, int W, int blocks, int32_t* out, int to_table,
                      hipStream_t stream) {
    using C = RegCfg<P>;
    const int tiles = (W + C::T - 1) / C::T;
    const long long gx = (long long)tiles * blocks;
    if (gx > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)gx, (P == 0) ? 1 : 2, 1);
    hipLaunchKernelGGL((fht_reg_kernel<P, PixT>), grid, dim3(C::NT), 0, stream, img, w, W, tiles,
                       out, to_table);
    return hipGetLastError();
}

template <typename PixT>
hipError_t launch_reg_p(int p, const PixT* img, int w, int W, int blocks, int32_t* out,
                        int to_table, hipStream_t stream) {
    switch (p) {
        case 0: return launch_reg<0>(img, w, W, blocks, out, to_table, stream);
        case 1: return launch_reg<1>(img, w, W, blocks, out, to_table, stream);
        case 2: return launch_reg<2>(img, w, W, blocks, out, to_table, stream);
        case 3: return launch_reg<3>(img, w, W, blocks, out, to_table, stream);
        case 4: return launch_reg<4>(img, w, W, blocks, out, to_table, stream);
        case 5: return launch_reg<5>(img, w, W, blocks, out, to_table, stream);
        case 6: return launch_reg<6>(img, w, W, blocks, out, to_table, stream);
        case 7: return launch_reg<7>(img, w, W, blocks, out, to_table, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename PixT>
hipError_t launch_fht_t(const PixT* img, const Geometry& g, int32_t* tables, void* scratch,
                        hipStream_t stream) {
    if (g.p <= kRegMaxP) return launch_reg_p<PixT>(g.p, img, g.w, g.W, g.k, tables, 1, stream);
    // Tall bands: 128-row sub-blocks first, then the coarse levels.
    const int sub_blocks = g.h >> kRegMaxP;
    int32_t* sub = static_cast<int32_t*>(scratch);
    hipError_t e = launch_reg_p<PixT>(kRegMaxP, img, g.w, g.W, sub_blocks, sub, 0, stream);
    if (e != hipSuccess) return e;
    const int tiles_x = (g.W + 255) / 256;
    const long long gx = (long long)tiles_x * g.n;
    if (gx > 0x7fffffffLL || g.k > 65535) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)gx, 2, (unsigned)g.k);
    hipLaunchKernelGGL(fht_combine_kernel, grid, dim3(256), 0, stream, sub, g.p, g.W, tiles_x,
                       tables);
    return hipGetLastError();
}

}  // namespace

size_t fht_scratch_bytes(const Geometry& g) {
    if (g.p <= kRegMaxP) return 0;
    // [h/128 sub-blocks][2 directions][128 shifts][W] int32
    return (size_t)(g.h >> kRegMaxP) * 2 * (1u << kRegMaxP) * (size_t)g.W * sizeof(int32_t);
}

hipError_t launch_fht(const void* img, int dtype, const Geometry& g, int32_t* tables,
                      void* scratch, hipStream_t stream) {
    if (dtype == 0)
        return launch_fht_t(static_cast<const uint8_t*>(img), g, tables, scratch, stream);
    return launch_fht_t(static_cast<const uint16_t*>(img), g, tables, scratch, stream);
}

}  // namespace fhtp
