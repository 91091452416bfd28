// pcg_stream.hip -- streaming-bandwidth probe (pcg_stream_probe): plain
// read and read/write streams over device memory, the ceilings the fused
// iteration passes are compared with on this device.
//
// Each launch streams `nin` input vectors and `nout` output vectors of n
// binary64 values in tiles of kProbeBlock * kProbeEPT elements over a
// persistent grid (the fused passes' tiling): every thread loads its
// elements of every input before it stores any output, as the fused passes
// do.  Output j receives in_j + c_j * (sum of the inputs), so every load is
// used and every store depends on every input.  With no outputs, each block
// writes its sum of the inputs to a sink (one double per block) so the loads
// cannot be dropped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "pcg.h"
#include "pcg_internal.h"

using namespace pcg;

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeEPT = 4;
constexpr int kProbeMaxStreams = 16;
constexpr int kProbeGrid = 4 * kNumCU;  // four blocks per CU, grid-stride over tiles
constexpr size_t kProbeSinkBytes = 65536;

struct Streams {
    const void *in[kProbeMaxStreams];
    void *out[kProbeMaxStreams];
    double *sink;
    int nin, nout;
    uint32_t tile_bytes;  // blocked layout: bytes of one 512-value tile of all streams (0: plain vectors)
    int wide;             // 16-byte accesses per lane (k_stream16)
};

// Element e of a stream that starts at p: plain vectors, or the blocked
// layout of the solver's workspace (512-value tiles of every stream one
// after another, the stream's slice of tile e / 512 at p's offset).
template <typename V>
__device__ __forceinline__ int64_t at(const Streams &s, int64_t e)
{
    if (!s.tile_bytes) return e;
    return (e >> 9) * (int64_t)(s.tile_bytes / sizeof(V)) + (e & 511);
}

template <bool NT, typename V>
__device__ __forceinline__ double ldp(const V *p)
{
    if constexpr (NT) return (double)__builtin_nontemporal_load(p);
    else return (double)*p;
}

template <bool NT, typename V>
__device__ __forceinline__ void stp(V *p, double v)
{
    if constexpr (NT) __builtin_nontemporal_store((V)v, p);
    else *p = (V)v;
}

// The same streams with 16-byte accesses: each lane moves 16 / sizeof(V)
// consecutive values of a stream per access (plain vectors only).
typedef float ProbeF4 __attribute__((ext_vector_type(4)));
typedef double ProbeD2 __attribute__((ext_vector_type(2)));
template <typename V, int NIN, int NOUT, bool NT>
__global__ void __launch_bounds__(kProbeBlock) k_stream16(Streams s, int64_t n)
{
    using W = typename std::conditional<sizeof(V) == 4, ProbeF4, ProbeD2>::type;
    constexpr int VB = 16 / sizeof(V);
    const int64_t groups = n / VB;  // n is a multiple of VB
    const int64_t tile_g = (int64_t)kProbeBlock * kProbeEPT;
    const int64_t ntiles = (groups + tile_g - 1) / tile_g;
    double keep = 0.0;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        W v[NIN][kProbeEPT];
        int64_t g[kProbeEPT];
#pragma unroll
        for (int j = 0; j < kProbeEPT; ++j) {
            const int64_t k = t * tile_g + (int64_t)j * kProbeBlock + threadIdx.x;
            g[j] = k < groups ? k : groups - 1;
        }
#pragma unroll
        for (int i = 0; i < NIN; ++i)
#pragma unroll
            for (int j = 0; j < kProbeEPT; ++j) {
                const W *p = static_cast<const W *>(s.in[i]) + g[j];
                v[i][j] = NT ? __builtin_nontemporal_load(p) : *p;
            }
#pragma unroll
        for (int j = 0; j < kProbeEPT; ++j) {
            const int64_t k = t * tile_g + (int64_t)j * kProbeBlock + threadIdx.x;
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < NIN; ++i) {
                if constexpr (VB == 4) sum += (double)v[i][j].x + v[i][j].y + v[i][j].z + v[i][j].w;
                else sum += v[i][j].x + v[i][j].y;
            }
            if constexpr (NOUT == 0) {
                keep += sum;
            } else if (k < groups) {
#pragma unroll
                for (int o = 0; o < NOUT; ++o) {
                    W w = v[o % NIN][j];
                    const V c = (V)((0.5 + o) * 1e-3 * sum);
                    w.x += c;
                    w.y += c;
                    if constexpr (VB == 4) {
                        w.z += c;
                        w.w += c;
                    }
                    W *p = static_cast<W *>(s.out[o]) + k;
                    if (NT) __builtin_nontemporal_store(w, p);
                    else *p = w;
                }
            }
        }
    }
    if constexpr (NOUT == 0) {
        __shared__ double red[kProbeBlock];
        red[threadIdx.x] = keep;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int k = 0; k < kProbeBlock; ++k) tot += red[k];
            s.sink[blockIdx.x] = tot;
        }
    }
}

// NIN inputs and NOUT outputs fixed at compile time: all of a tile's loads
// stay in registers.
template <typename V, int NIN, int NOUT, bool NT>
__global__ void __launch_bounds__(kProbeBlock) k_stream(Streams s, int64_t n)
{
    const int64_t tile_elems = (int64_t)kProbeBlock * kProbeEPT;
    const int64_t ntiles = (n + tile_elems - 1) / tile_elems;
    double keep = 0.0;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        double v[NIN][kProbeEPT];
        int64_t e[kProbeEPT];
#pragma unroll
        for (int j = 0; j < kProbeEPT; ++j) {
            const int64_t k = t * tile_elems + (int64_t)j * kProbeBlock + threadIdx.x;
            e[j] = k < n ? k : n - 1;
        }
#pragma unroll
        for (int j = 0; j < kProbeEPT; ++j) e[j] = at<V>(s, e[j]);
#pragma unroll
        for (int i = 0; i < NIN; ++i)
#pragma unroll
            for (int j = 0; j < kProbeEPT; ++j) v[i][j] = ldp<NT>(static_cast<const V *>(s.in[i]) + e[j]);
#pragma unroll
        for (int j = 0; j < kProbeEPT; ++j) {
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < NIN; ++i) sum += v[i][j];
            if constexpr (NOUT == 0) {
                keep += sum;
            } else {
                const int64_t k = t * tile_elems + (int64_t)j * kProbeBlock + threadIdx.x;
                if (k < n) {
#pragma unroll
                    for (int o = 0; o < NOUT; ++o)
                        stp<NT>(static_cast<V *>(s.out[o]) + e[j], v[o % NIN][j] + (0.5 + o) * 1e-3 * sum);
                }
            }
        }
    }
    if constexpr (NOUT == 0) {
        __shared__ double red[kProbeBlock];
        red[threadIdx.x] = keep;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int k = 0; k < kProbeBlock; ++k) tot += red[k];
            s.sink[blockIdx.x] = tot;
        }
    }
}

using ProbeFn = void (*)(const Streams &, int64_t, int, hipStream_t);

template <typename V, int NIN, int NOUT, bool NT>
void launch(const Streams &s, int64_t n, int grid, hipStream_t st)
{
    if (s.wide) hipLaunchKernelGGL((k_stream16<V, NIN, NOUT, NT>), dim3(grid), dim3(kProbeBlock), 0, st, s, n);
    else hipLaunchKernelGGL((k_stream<V, NIN, NOUT, NT>), dim3(grid), dim3(kProbeBlock), 0, st, s, n);
}

// The shapes the measurements use: read only, copy, and the fused passes'
// mixes of read and written streams.
template <typename V, bool NT>
ProbeFn pick(int nin, int nout)
{
    if (nout == 0) {
        switch (nin) {
        case 1: return launch<V, 1, 0, NT>;
        case 2: return launch<V, 2, 0, NT>;
        case 4: return launch<V, 4, 0, NT>;
        case 8: return launch<V, 8, 0, NT>;
        case 9: return launch<V, 9, 0, NT>;
        case 16: return launch<V, 16, 0, NT>;
        default: return nullptr;
        }
    }
    if (nin == 1 && nout == 1) return launch<V, 1, 1, NT>;
    if (nin == 2 && nout == 1) return launch<V, 2, 1, NT>;
    if (nin == 4 && nout == 4) return launch<V, 4, 4, NT>;
    if (nin == 5 && nout == 4) return launch<V, 5, 4, NT>;
    if (nin == 8 && nout == 8) return launch<V, 8, 8, NT>;
    if (nin == 9 && nout == 8) return launch<V, 9, 8, NT>;
    if (nin == 9 && nout == 9) return launch<V, 9, 9, NT>;
    return nullptr;
}

size_t round4k(size_t v) { return (v + 4095) & ~size_t(4095); }

}  // namespace

extern "C" pcg_status pcg_stream_probe(int32_t nin, int32_t nout, int32_t flags, int64_t n, void *buffer,
                                       size_t bytes, int32_t reps, void *hip_stream, double *us_per_launch)
{
    if (!us_per_launch) return invalid("us_per_launch is null");
    if (n < 1 || n > (int64_t(1) << 34)) return invalid("n must be in [1, 2^34]");
    if (reps < 1 || reps > 100000) return invalid("reps must be in [1, 100000]");
    if (flags & ~(PCG_PROBE_NT | PCG_PROBE_BLOCKED | PCG_PROBE_FP32 | PCG_PROBE_WIDE | (0xf << 8)))
        return invalid("unknown probe flags");
    if ((flags & PCG_PROBE_WIDE) && (flags & PCG_PROBE_BLOCKED))
        return invalid("PCG_PROBE_WIDE streams plain vectors only");
    if ((flags & PCG_PROBE_WIDE) && (n % ((flags & PCG_PROBE_FP32) ? 4 : 2)))
        return invalid("PCG_PROBE_WIDE needs n a multiple of the values per 16 bytes");
    const int per_cu = (flags >> 8) & 0xf;  // blocks per CU of the persistent grid (0: 4)
    const bool nt = (flags & PCG_PROBE_NT) != 0, blocked = (flags & PCG_PROBE_BLOCKED) != 0;
    const bool f32 = (flags & PCG_PROBE_FP32) != 0;
    const ProbeFn fn = f32 ? (nt ? pick<float, true>(nin, nout) : pick<float, false>(nin, nout))
                           : (nt ? pick<double, true>(nin, nout) : pick<double, false>(nin, nout));
    if (!fn) return invalid("unsupported (nin, nout) stream mix");
    const size_t vb = round4k((size_t)n * 8);  // a whole number of 512-value tiles
    const size_t need = (size_t)(nin + nout) * vb + kProbeSinkBytes;
    if (!buffer || ((uintptr_t)buffer % 256)) return invalid("buffer must be non-null and 256-byte aligned");
    if (bytes < need) return invalid("buffer too small: (nin + nout) * round_up(8 n, 4096) + 65536 bytes needed");
    Streams s{};
    char *base = (char *)buffer;
    // plain: stream k is the k-th vector; blocked: stream k is slice k of every tile
    const size_t es = f32 ? 4 : 8, slice = 512 * es;
    const size_t stride = blocked ? slice : vb;
    for (int i = 0; i < nin; ++i) s.in[i] = base + (size_t)i * stride;
    for (int o = 0; o < nout; ++o) s.out[o] = base + (size_t)(nin + o) * stride;
    s.sink = (double *)(base + (size_t)(nin + nout) * vb);
    s.nin = nin;
    s.nout = nout;
    s.tile_bytes = blocked ? (uint32_t)((nin + nout) * slice) : 0u;
    s.wide = (flags & PCG_PROBE_WIDE) != 0;
    const int64_t per_tile = (int64_t)kProbeBlock * kProbeEPT * (s.wide ? 16 / (int64_t)es : 1);
    const int64_t tiles = (n + per_tile - 1) / per_tile;
    const int grid = (int)std::min<int64_t>(per_cu ? per_cu * kNumCU : kProbeGrid, tiles);
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he;
    if ((he = hipEventCreate(&e0)) != hipSuccess) return hip_fail(he, "hipEventCreate");
    if ((he = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    auto done = [&](pcg_status r) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return r;
    };
    fn(s, n, grid, st);  // warm-up (first touch, code load)
    if ((he = hipEventRecord(e0, st)) != hipSuccess) return done(hip_fail(he, "hipEventRecord"));
    for (int r = 0; r < reps; ++r) fn(s, n, grid, st);
    if ((he = hipEventRecord(e1, st)) != hipSuccess) return done(hip_fail(he, "hipEventRecord"));
    if ((he = hipEventSynchronize(e1)) != hipSuccess) return done(hip_fail(he, "hipEventSynchronize"));
    if ((he = hipGetLastError()) != hipSuccess) return done(hip_fail(he, "k_stream"));
    float ms = 0.f;
    if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return done(hip_fail(he, "hipEventElapsedTime"));
    *us_per_launch = (double)ms * 1e3 / reps;
    return done(PCG_OK);
}
