// batched.hip -- many species and cells in one persistent launch.
//
// A plan lays the segments out back to back (segment s owns output positions
// start[s] .. start[s+1]-1) and keeps on the device: the segment boundaries,
// each segment's Table 1 setup (computed once on the host, as the paper
// prescribes) with its drift, and a tile -> first-segment map.  The
// persistent kernel walks the particle range with a grid stride; each group
// of U consecutive particles finds its segment by a binary search restricted
// to its tile's segment range.  Particle j of segment s uses the counter
// (j - start[s], seg_id[s]), so a segment's samples equal a single-species
// call with the same seed and seg_id, whatever the launch shape.  The device
// tables hold pieces of at most 2^32 particles (a longer segment is split),
// each with the Philox words its counters share through the first two rounds
// (SegWords), so a particle's block takes 18 products instead of 20.
//
// The launch can be captured once into a hipGraph and replayed; the shape
// (block, particles per thread, grid) is chosen by a timing sweep.
//
// Fused particle loading (positions with the velocities, for PIC start-up):
// when the plan holds a cell box per segment, the same launch also writes
// px, py, pz = lo + u * size with u from the block of draw 1 of the
// particle's counter (velocities use draw 0, so they are unchanged).
// u = (r + 1/2) 2^-32 in FP64; in FP32 u = (floor(r / 2^9) + 1/2) 2^-23,
// exact in float and below 1.  The box is half-open: a rounded lo + u size
// that reaches lo + size is capped at the largest value of the output type
// below it (precomputed per cell on the host).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kappa_device.hpp"
#include "kappa_internal.hpp"
#include "kappa_store.hpp"

namespace kappa {

namespace {

// Tiles of the segment map: 2^6 particles each, coarser (a power of two) for
// plans whose map would exceed 2^24 tiles.
constexpr uint32_t kTileShiftMin = 6;
constexpr uint64_t kMaxTiles = 1ull << 24;

struct alignas(16) SegF32 {
    float inv_kstar, a, neg_c_kstar, four_b_kstar, two_kstar, two_b, theta, dx, dy, dz;
    uint32_t seg_id;
};

struct alignas(16) SegF64 {
    double kstar, inv_kstar, a, b, c, two_b, neg_four_b, theta, dx, dy, dz;
};

struct CellF32 {
    float lo[3], size[3], hi[3];  // hi: largest float below the real lo + size (lo if size is 0)
};

struct CellF64 {
    double lo[3], size[3], hi[3];
};

struct BatchArgs {
    uint64_t total;
    uint32_t k0, k1;
    uint32_t nseg;
    uint32_t tile_shift;     // particles per tile: 2^tile_shift
    const uint64_t *start;   // nseg + 1
    const uint32_t *tile;    // ntiles + 1
    const SegF32 *seg32;     // nseg
    const SegF64 *seg64;     // nseg
    const SegWords *words;   // nseg
    const CellF32 *cell32;   // nseg, positions only
    const CellF64 *cell64;   // nseg, positions only
    void *vx, *vy, *vz;
    void *px, *py, *pz;      // positions only
};

// Largest s in [lo, hi] with start[s] <= j (start[lo] <= j holds).
template <typename I>
__device__ __forceinline__ uint32_t find_segment(const uint64_t *start, uint32_t lo, uint32_t hi, I j)
{
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (static_cast<I>(start[mid]) <= j)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// A group's U particles usually lie in one segment (PIC cells hold hundreds of
// particles per species): the segment's bounds, id and setup block are loaded
// once per group and reloaded only where the group crosses into the next
// segment.
template <int MODE>
struct SegParams;

template <>
struct SegParams<kModeF64> {
    SegF64 q;
    __device__ __forceinline__ void load(const BatchArgs &a, uint32_t s) { q = a.seg64[s]; }
};

template <int MODE>
struct SegParams {
    SegF32 q;
    __device__ __forceinline__ void load(const BatchArgs &a, uint32_t s) { q = a.seg32[s]; }
};

template <int MODE>
struct CellParams {
    CellF32 q;
    __device__ __forceinline__ void load(const BatchArgs &a, uint32_t s) { q = a.cell32[s]; }
    // u = (floor(r / 2^9) + 1/2) 2^-23: a 24-bit dyadic, exact in float, in (0, 1)
    __device__ __forceinline__ float coord(int k, uint32_t r) const
    {
        const float u = fmaf(static_cast<float>(r >> 9), 0x1p-23f, 0x1p-24f);
        return fminf(fmaf(u, q.size[k], q.lo[k]), q.hi[k]);
    }
};

template <>
struct CellParams<kModeF64> {
    CellF64 q;
    __device__ __forceinline__ void load(const BatchArgs &a, uint32_t s) { q = a.cell64[s]; }
    __device__ __forceinline__ double coord(int k, uint32_t r) const
    {
        const double u = fma(static_cast<double>(r), 0x1p-32, 0x1p-33);
        return fmin(fma(u, q.size[k], q.lo[k]), q.hi[k]);
    }
};

// I is the particle index type: uint32_t when the plan holds fewer than 2^31
// particles and the grid fewer than 2^31 threads (32-bit index arithmetic, 3%
// faster for 5.1e6 particles in 12,288 segments), else uint64_t.
template <int MODE, int U, bool POS, typename I>
__global__ void __launch_bounds__(256) batched_kernel(BatchArgs a)
{
    using T = typename std::conditional<MODE == kModeF64, double, float>::type;
    T *vx = static_cast<T *>(a.vx);
    T *vy = static_cast<T *>(a.vy);
    T *vz = static_cast<T *>(a.vz);
    const I total = static_cast<I>(a.total);
    const I ngroups = (total + U - 1) / U;
    const I stride = static_cast<I>(gridDim.x) * blockDim.x;
    for (I g = static_cast<I>(blockIdx.x) * blockDim.x + threadIdx.x; g < ngroups; g += stride) {
        const I j0 = g * U;
        const I t = j0 >> a.tile_shift;
        uint32_t s = find_segment<I>(a.start, a.tile[t], a.tile[t + 1], j0);
        I seg_begin = static_cast<I>(a.start[s]), seg_next = static_cast<I>(a.start[s + 1]);  // s + 1 <= nseg
        SegWords wd = a.words[s];
        SegParams<MODE> prm;
        prm.load(a, s);
        CellParams<MODE> cell;
        if constexpr (POS) cell.load(a, s);
        T x[U], y[U], z[U];
        T qx[U], qy[U], qz[U];  // positions (POS only)
        uint32_t seg_of[U];
        uint32_t tails = 0;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const I j = j0 + k;
            if (j >= total) {
                x[k] = y[k] = z[k] = T(0);
                if constexpr (POS) qx[k] = qy[k] = qz[k] = T(0);
                seg_of[k] = s;
                continue;
            }
            if (j >= seg_next) {
                // next non-empty segment; ends because j < total = start[nseg]
                do {
                    ++s;
                    seg_next = static_cast<I>(a.start[s + 1]);
                } while (j >= seg_next);
                seg_begin = static_cast<I>(a.start[s]);
                wd = a.words[s];
                prm.load(a, s);
                if constexpr (POS) cell.load(a, s);
            }
            seg_of[k] = s;
            // the piece holds at most 2^32 particles: j - seg_begin is the counter's low word
            const uint32_t c0 = static_cast<uint32_t>(j - seg_begin);
            if constexpr (POS) {
                const Block4 bp = philox4x32_10_seg(c0, 1, wd, a.k0, a.k1);
                qx[k] = cell.coord(0, bp.r0);
                qy[k] = cell.coord(1, bp.r1);
                qz[k] = cell.coord(2, bp.r2);
            }
            const Block4 b = philox4x32_10_seg(c0, 0, wd, a.k0, a.k1);
            const auto &q = prm.q;
            if constexpr (MODE == kModeF64) {
                SpeciesF64 sp{q.kstar, q.inv_kstar, q.a, q.b, q.c, q.two_b, q.neg_four_b, q.theta, 0, 0, 0};
                particle_f64(b, sp, x[k], y[k], z[k]);
            } else {
                SpeciesF32 sp{};
                sp.inv_kstar = q.inv_kstar;
                sp.a = q.a;
                sp.neg_c_kstar = q.neg_c_kstar;
                sp.four_b_kstar = q.four_b_kstar;
                sp.two_kstar = q.two_kstar;
                sp.two_b = q.two_b;
                sp.theta = q.theta;
                particle_f32(b, sp, x[k], y[k], z[k]);
                if constexpr (MODE == kModeF32) tails |= static_cast<uint32_t>(in_fp64_tail(b.r0)) << k;
            }
            x[k] += q.dx;
            y[k] += q.dy;
            z[k] += q.dz;
        }
        if constexpr (MODE == kModeF32) {
            if (__builtin_expect(tails != 0, 0)) {
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    if ((tails >> k) & 1u) {
                        const uint32_t sq = seg_of[k];
                        const SegF64 w = a.seg64[sq];
                        const SegF32 f = a.seg32[sq];
                        const SpeciesF64 s64{w.kstar, w.inv_kstar, w.a, w.b, w.c, w.two_b, w.neg_four_b, w.theta, 0, 0, 0};
                        const Block4 b =
                            philox4x32_10_seg(static_cast<uint32_t>(j0 + k - static_cast<I>(a.start[sq])), 0, a.words[sq], a.k0, a.k1);
                        tail_particle_f32(b, s64, x[k], y[k], z[k]);
                        x[k] += f.dx;
                        y[k] += f.dy;
                        z[k] += f.dz;
                    }
                }
            }
        }
        store_or_tail<T, U, I>(vx, j0, total, x);
        store_or_tail<T, U, I>(vy, j0, total, y);
        store_or_tail<T, U, I>(vz, j0, total, z);
        if constexpr (POS) {
            store_or_tail<T, U, I>(static_cast<T *>(a.px), j0, total, qx);
            store_or_tail<T, U, I>(static_cast<T *>(a.py), j0, total, qy);
            store_or_tail<T, U, I>(static_cast<T *>(a.pz), j0, total, qz);
        }
    }
}

template <int MODE, bool POS>
hipError_t launch_batched_mode(const Shape &sh, const BatchArgs &a, hipStream_t stream)
{
    log_launch(POS ? "batched_kernel+positions" : "batched_kernel", MODE, a.total, sh, stream);
    dim3 grid(sh.grid), block(sh.block);
    // 32-bit indices while the group index plus the grid stride stays below 2^32
    const bool narrow = a.total < (1ull << 31) && static_cast<uint64_t>(sh.grid) * sh.block < (1ull << 31);
    switch (sh.unroll * (narrow ? 1 : -1)) {
    case 1: hipLaunchKernelGGL((batched_kernel<MODE, 1, POS, uint32_t>), grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((batched_kernel<MODE, 2, POS, uint32_t>), grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((batched_kernel<MODE, 4, POS, uint32_t>), grid, block, 0, stream, a); break;
    case 8: hipLaunchKernelGGL((batched_kernel<MODE, 8, POS, uint32_t>), grid, block, 0, stream, a); break;
    case -1: hipLaunchKernelGGL((batched_kernel<MODE, 1, POS, uint64_t>), grid, block, 0, stream, a); break;
    case -2: hipLaunchKernelGGL((batched_kernel<MODE, 2, POS, uint64_t>), grid, block, 0, stream, a); break;
    case -4: hipLaunchKernelGGL((batched_kernel<MODE, 4, POS, uint64_t>), grid, block, 0, stream, a); break;
    case -8: hipLaunchKernelGGL((batched_kernel<MODE, 8, POS, uint64_t>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_batched_pos(const Shape &sh, const BatchArgs &a, hipStream_t stream)
{
    return a.px ? launch_batched_mode<MODE, true>(sh, a, stream) : launch_batched_mode<MODE, false>(sh, a, stream);
}

hipError_t launch_batched(int mode, const Shape &sh, const BatchArgs &a, hipStream_t stream)
{
    switch (mode) {
    case kModeF64: return launch_batched_pos<kModeF64>(sh, a, stream);
    case kModeF32: return launch_batched_pos<kModeF32>(sh, a, stream);
    case kModeF32NoTail: return launch_batched_pos<kModeF32NoTail>(sh, a, stream);
    default: return hipErrorInvalidValue;
    }
}

bool shape_valid(const Shape &s)
{
    const bool b = s.block == 64 || s.block == 128 || s.block == 256;
    const bool u = s.unroll == 1 || s.unroll == 2 || s.unroll == 4 || s.unroll == 8;
    return b && u && s.grid >= 1 && s.grid <= (1 << 23);
}

std::string cache_key(int mode, uint64_t total, uint32_t nseg)
{
    // bucket by powers of two of the total and the segment count
    int tb = 0, sb = 0;
    while ((1ull << tb) < total && tb < 63) ++tb;
    while ((1u << sb) < nseg && sb < 31) ++sb;
    char buf[96];
    std::snprintf(buf, sizeof buf, "batched|mode%d|total2^%d|nseg2^%d", mode, tb, sb);
    return buf;
}

}  // namespace

}  // namespace kappa

struct kappa_plan_s {
    int device = 0;
    int mode = 0;
    uint64_t total = 0;
    uint32_t nseg = 0;   // the caller's segments
    uint32_t npiece = 0; // device pieces: segments split at 2^32 particles
    std::vector<uint32_t> piece_seg;  // caller's segment of each piece
    uint32_t k0 = 0, k1 = 0;
    kappa::Shape shape{256, 4, 1};
    void *dev_block = nullptr;  // one allocation holding every table
    const uint64_t *start = nullptr;
    const uint32_t *tile = nullptr;
    uint32_t tile_shift = kappa::kTileShiftMin;
    const kappa::SegF32 *seg32 = nullptr;
    const kappa::SegF64 *seg64 = nullptr;
    const kappa::SegWords *words = nullptr;
    // cell boxes for fused particle loading (kappa_plan_set_cells)
    void *cell_block = nullptr;
    const kappa::CellF32 *cell32 = nullptr;
    const kappa::CellF64 *cell64 = nullptr;
    // captured graph and the outputs it was captured for
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;
    void *g_out[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    kappa::Shape g_shape{0, 0, 0};
};

namespace kappa {

namespace {

// Outputs of one launch: velocities, and positions when pos[0] is non-null.
struct Outputs {
    void *v[3];
    void *pos[3];
};

BatchArgs batch_args(const kappa_plan_s *p, const Outputs &o)
{
    BatchArgs a;
    a.total = p->total;
    a.k0 = p->k0;
    a.k1 = p->k1;
    a.nseg = p->npiece;
    a.start = p->start;
    a.tile = p->tile;
    a.tile_shift = p->tile_shift;
    a.seg32 = p->seg32;
    a.seg64 = p->seg64;
    a.words = p->words;
    a.cell32 = p->cell32;
    a.cell64 = p->cell64;
    a.vx = o.v[0];
    a.vy = o.v[1];
    a.vz = o.v[2];
    a.px = o.pos[0];
    a.py = o.pos[1];
    a.pz = o.pos[2];
    return a;
}

// One thread per group of particles: the whole plan in one pass of
// workgroups, with no partly filled second pass (a grid of a few workgroups
// per CU striding over 5e6 particles leaves one).
Shape default_batched_shape(int mode, uint64_t total)
{
    Shape s;
    s.block = 256;
    s.unroll = mode == kModeF64 ? 2 : 4;
    const uint64_t groups = (total + s.unroll - 1) / s.unroll;
    const uint64_t need = (groups + s.block - 1) / s.block;
    s.grid = static_cast<int>(std::max<uint64_t>(1, std::min<uint64_t>(need, 1ull << 23)));
    return s;
}

bool aligned_for(int mode, const Shape &s, const Outputs &o)
{
    const size_t esz = mode == kModeF64 ? 8 : 4;
    const size_t bytes = esz * s.unroll;
    const size_t need = bytes >= 16 ? 16 : bytes;
    for (int k = 0; k < 3; ++k) {
        if (reinterpret_cast<uintptr_t>(o.v[k]) % need) return false;
        if (o.pos[0] && reinterpret_cast<uintptr_t>(o.pos[k]) % need) return false;
    }
    return true;
}

// Shape actually launched: falls back to one particle per thread when the
// outputs are not aligned for the group's vector store.
Shape effective_shape(const kappa_plan_s *p, const Outputs &o)
{
    Shape s = p->shape;
    if (!aligned_for(p->mode, s, o)) s.unroll = 1;
    return s;
}

void drop_graph(kappa_plan_s *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

}  // namespace

}  // namespace kappa

using namespace kappa;

extern "C" kappa_status kappa_plan_create_impl(const kappa_segment *segs, uint32_t nseg, uint64_t seed, int precision,
                                               kappa_plan *out)
{
    auto *p = new (std::nothrow) kappa_plan_s();
    if (!p) return fail(KAPPA_ENOMEM, "host allocation of the plan failed");
    p->mode = precision;
    p->nseg = nseg;
    p->k0 = static_cast<uint32_t>(seed);
    p->k1 = static_cast<uint32_t>(seed >> 32);
    kappa_status st = check_hip(hipGetDevice(&p->device), "hipGetDevice");
    if (st != KAPPA_OK) {
        delete p;
        return st;
    }
    // host tables, one entry per piece of at most 2^32 particles
    constexpr uint64_t kPiece = 1ull << 32;
    std::vector<uint64_t> start;
    std::vector<SegF32> s32;
    std::vector<SegF64> s64;
    std::vector<SegWords> words;
    std::map<double, Setup> setups;  // species repeat across cells: set up each kappa once
    uint64_t acc = 0;
    for (uint32_t s = 0; s < nseg; ++s) {
        auto it = setups.find(segs[s].kappa);
        if (it == setups.end()) it = setups.emplace(segs[s].kappa, make_setup(segs[s].kappa)).first;
        const SpeciesF64 a = species_f64(it->second, segs[s].theta);
        const SpeciesF32 b = species_f32(it->second, segs[s].theta);
        const SegF64 q64{a.kstar, a.inv_kstar, a.a, a.b, a.c, a.two_b, a.neg_four_b, a.theta,
                         segs[s].drift[0], segs[s].drift[1], segs[s].drift[2]};
        const SegF32 q32{b.inv_kstar, b.a, b.neg_c_kstar, b.four_b_kstar, b.two_kstar, b.two_b, b.theta,
                         static_cast<float>(segs[s].drift[0]), static_cast<float>(segs[s].drift[1]),
                         static_cast<float>(segs[s].drift[2]), segs[s].seg_id};
        // piece h of the segment: counters (h 2^32 + i) for i < 2^32, whose high word h enters
        // round 1 next to M_B seg_id
        for (uint64_t h = 0, left = segs[s].count; h == 0 || left > 0; ++h) {
            const uint64_t n = std::min(left, kPiece);
            const uint64_t pb = static_cast<uint64_t>(kMulB) * segs[s].seg_id;
            SegWords w;
            w.c0 = static_cast<uint32_t>(pb >> 32) ^ static_cast<uint32_t>(h) ^ p->k0;
            w.c1 = static_cast<uint32_t>(pb);
            const uint64_t pa = static_cast<uint64_t>(kMulA) * w.c0;
            w.pa_hi = static_cast<uint32_t>(pa >> 32);
            w.pa_lo = static_cast<uint32_t>(pa);
            start.push_back(acc);
            s32.push_back(q32);
            s64.push_back(q64);
            words.push_back(w);
            p->piece_seg.push_back(s);
            acc += n;
            left -= n;
        }
    }
    const uint32_t npiece = static_cast<uint32_t>(start.size());
    p->npiece = npiece;
    start.push_back(acc);
    p->total = acc;
    uint32_t shift = kTileShiftMin;
    while ((acc >> shift) >= kMaxTiles) ++shift;
    p->tile_shift = shift;
    const uint64_t ntiles = (acc + (1ull << shift) - 1) >> shift;
    std::vector<uint32_t> tile(ntiles + 1);
    {
        uint32_t s = 0;
        for (uint64_t t = 0; t <= ntiles; ++t) {
            const uint64_t j = std::min<uint64_t>(t << shift, acc > 0 ? acc - 1 : 0);
            while (s + 1 < npiece && start[s + 1] <= j) ++s;
            tile[t] = s;
        }
    }
    // one device allocation: start | tile | seg32 | seg64 | words, each 256-byte aligned
    auto up = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
    const size_t o_start = 0;
    const size_t o_tile = o_start + up(start.size() * sizeof(uint64_t));
    const size_t o_s32 = o_tile + up(tile.size() * sizeof(uint32_t));
    const size_t o_s64 = o_s32 + up(s32.size() * sizeof(SegF32));
    const size_t o_words = o_s64 + up(s64.size() * sizeof(SegF64));
    const size_t bytes = o_words + up(words.size() * sizeof(SegWords));
    if (hipMalloc(&p->dev_block, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return fail(KAPPA_ENOMEM, "hipMalloc of %zu bytes for the plan tables failed", bytes);
    }
    std::vector<unsigned char> host(bytes, 0);
    std::memcpy(host.data() + o_start, start.data(), start.size() * sizeof(uint64_t));
    std::memcpy(host.data() + o_tile, tile.data(), tile.size() * sizeof(uint32_t));
    std::memcpy(host.data() + o_s32, s32.data(), s32.size() * sizeof(SegF32));
    std::memcpy(host.data() + o_s64, s64.data(), s64.size() * sizeof(SegF64));
    std::memcpy(host.data() + o_words, words.data(), words.size() * sizeof(SegWords));
    st = check_hip(hipMemcpy(p->dev_block, host.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy plan tables");
    if (st != KAPPA_OK) {
        (void)hipFree(p->dev_block);
        delete p;
        return st;
    }
    auto *base = static_cast<unsigned char *>(p->dev_block);
    p->start = reinterpret_cast<const uint64_t *>(base + o_start);
    p->tile = reinterpret_cast<const uint32_t *>(base + o_tile);
    p->seg32 = reinterpret_cast<const SegF32 *>(base + o_s32);
    p->seg64 = reinterpret_cast<const SegF64 *>(base + o_s64);
    p->words = reinterpret_cast<const SegWords *>(base + o_words);
    p->shape = default_batched_shape(p->mode, p->total);
    {
        Shape s{};
        if (cache_lookup(cache_key(p->mode, p->total, p->nseg), s) && shape_valid(s)) p->shape = s;
    }
    *out = p;
    return KAPPA_OK;
}

namespace kappa {
namespace {
kappa_status check_plan_outputs(const kappa_plan_s *p, const Outputs &o)
{
    if (p->total == 0) return KAPPA_OK;
    const bool pos = o.pos[0] || o.pos[1] || o.pos[2];
    for (int k = 0; k < 3; ++k) {
        if (!o.v[k]) return fail(KAPPA_EINVAL, "null velocity pointer for a plan of %llu particles",
                                 (unsigned long long)p->total);
        if (pos && !o.pos[k]) return fail(KAPPA_EINVAL, "null position pointer");
    }
    if (pos && !p->cell_block) return fail(KAPPA_EINVAL, "positions asked for but the plan has no cells "
                                                         "(kappa_plan_set_cells)");
    const size_t e = p->mode == kModeF64 ? 8 : 4;
    for (int k = 0; k < 3; ++k)
        if (reinterpret_cast<uintptr_t>(o.v[k]) % e || (pos && reinterpret_cast<uintptr_t>(o.pos[k]) % e))
            return fail(KAPPA_EALIGN, "output pointers must be aligned to %zu bytes", e);
    return KAPPA_OK;
}

kappa_status plan_launch(kappa_plan p, const Outputs &o, void *stream)
{
    const kappa_status cs = check_plan_outputs(p, o);
    if (cs != KAPPA_OK || p->total == 0) return cs;
    const Shape s = effective_shape(p, o);
    return check_hip(launch_batched(p->mode, s, batch_args(p, o), static_cast<hipStream_t>(stream)),
                     "batched kernel launch");
}

// Captures the launch for these outputs and shape once, then replays it.
kappa_status plan_graph_launch(kappa_plan p, const Outputs &o, void *stream)
{
    const kappa_status cs = check_plan_outputs(p, o);
    if (cs != KAPPA_OK || p->total == 0) return cs;
    const Shape s = effective_shape(p, o);
    const void *want[6] = {o.v[0], o.v[1], o.v[2], o.pos[0], o.pos[1], o.pos[2]};
    bool stale = !p->exec || p->g_shape.block != s.block || p->g_shape.unroll != s.unroll || p->g_shape.grid != s.grid;
    for (int k = 0; k < 6; ++k) stale = stale || p->g_out[k] != want[k];
    if (stale) {
        drop_graph(p);
        kappa_status st;
        if (!p->capture_stream) {
            st = check_hip(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
            if (st != KAPPA_OK) return st;
        }
        st = check_hip(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        if (st != KAPPA_OK) return st;
        const hipError_t le = launch_batched(p->mode, s, batch_args(p, o), p->capture_stream);
        const hipError_t ce = hipStreamEndCapture(p->capture_stream, &p->graph);
        if (le != hipSuccess) return check_hip(le, "batched kernel capture");
        st = check_hip(ce, "hipStreamEndCapture");
        if (st != KAPPA_OK) return st;
        st = check_hip(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        if (st != KAPPA_OK) {
            drop_graph(p);
            return st;
        }
        for (int k = 0; k < 6; ++k) p->g_out[k] = const_cast<void *>(want[k]);
        p->g_shape = s;
    }
    return check_hip(hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
}

Outputs velocities(void *vx, void *vy, void *vz) { return Outputs{{vx, vy, vz}, {nullptr, nullptr, nullptr}}; }
}  // namespace
}  // namespace kappa

extern "C" kappa_status kappa_plan_launch_impl(kappa_plan p, void *vx, void *vy, void *vz, void *stream)
{
    return plan_launch(p, velocities(vx, vy, vz), stream);
}

extern "C" kappa_status kappa_plan_graph_launch_impl(kappa_plan p, void *vx, void *vy, void *vz, void *stream)
{
    return plan_graph_launch(p, velocities(vx, vy, vz), stream);
}

extern "C" kappa_status kappa_plan_launch_pic_impl(kappa_plan p, void *px, void *py, void *pz, void *vx, void *vy,
                                                   void *vz, void *stream)
{
    return plan_launch(p, Outputs{{vx, vy, vz}, {px, py, pz}}, stream);
}

extern "C" kappa_status kappa_plan_graph_launch_pic_impl(kappa_plan p, void *px, void *py, void *pz, void *vx,
                                                         void *vy, void *vz, void *stream)
{
    return plan_graph_launch(p, Outputs{{vx, vy, vz}, {px, py, pz}}, stream);
}

namespace kappa {
namespace {
// Makes the plan's device current for the lifetime of the guard.
struct PlanDevice {
    int prev = -1;
    explicit PlanDevice(const kappa_plan_s *p)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != p->device) (void)hipSetDevice(p->device);
    }
    ~PlanDevice()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};
}  // namespace
}  // namespace kappa

namespace kappa {
namespace {
// Largest value of T strictly below the real number lo + size, and not below
// lo (lo itself when size is 0): the rounded sum s and its exact error
// (Knuth's two-sum, in T's own arithmetic) tell whether s lies below the
// real sum (then s is the answer) or not (then the value just below s is).
template <typename T>
T box_upper(T lo, T size)
{
    if (!(size > T(0))) return lo;
    const T s = lo + size;
    const T t = s - lo;
    const T err = (lo - (s - t)) + (size - t);
    const T hi = err > T(0) ? s : std::nextafter(s, -std::numeric_limits<T>::infinity());
    return hi > lo ? hi : lo;
}
}  // namespace
}  // namespace kappa

extern "C" kappa_status kappa_plan_set_cells_impl(kappa_plan p, const kappa_cell *cells)
{
    PlanDevice guard(p);
    if (p->cell_block) {
        // launches in flight, or the captured graph, may still read the old table
        kappa_status st = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (st != KAPPA_OK) return st;
        drop_graph(p);
        st = check_hip(hipFree(p->cell_block), "hipFree cell table");
        p->cell_block = nullptr;
        p->cell32 = nullptr;
        p->cell64 = nullptr;
        if (st != KAPPA_OK) return st;
    }
    if (!cells) return KAPPA_OK;
    for (uint32_t s = 0; s < p->nseg; ++s)
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(cells[s].lo[k]) || !std::isfinite(cells[s].size[k]) || cells[s].size[k] < 0.0)
                return fail(KAPPA_EINVAL, "cell %u: lo must be finite and size finite and >= 0", s);
    std::vector<CellF32> c32(p->nseg);
    std::vector<CellF64> c64(p->nseg);
    for (uint32_t s = 0; s < p->nseg; ++s)
        for (int k = 0; k < 3; ++k) {
            c64[s].lo[k] = cells[s].lo[k];
            c64[s].size[k] = cells[s].size[k];
            c64[s].hi[k] = box_upper(c64[s].lo[k], c64[s].size[k]);
            c32[s].lo[k] = static_cast<float>(cells[s].lo[k]);
            c32[s].size[k] = static_cast<float>(cells[s].size[k]);
            c32[s].hi[k] = box_upper(c32[s].lo[k], c32[s].size[k]);
            if (p->mode != kModeF64 &&
                !(std::isfinite(c32[s].lo[k]) && std::isfinite(c32[s].size[k]) &&
                  std::isfinite(c32[s].lo[k] + c32[s].size[k])))
                return fail(KAPPA_EINVAL, "cell %u: lo, size and lo + size must be finite as floats for an FP32 plan", s);
        }
    // one entry per device piece (pieces of one segment share its box)
    if (p->npiece != p->nseg) {
        std::vector<CellF32> p32(p->npiece);
        std::vector<CellF64> p64(p->npiece);
        for (uint32_t v = 0; v < p->npiece; ++v) {
            p32[v] = c32[p->piece_seg[v]];
            p64[v] = c64[p->piece_seg[v]];
        }
        c32.swap(p32);
        c64.swap(p64);
    }
    const size_t o64 = (c32.size() * sizeof(CellF32) + 255) & ~static_cast<size_t>(255);
    const size_t bytes = o64 + c64.size() * sizeof(CellF64);
    if (hipMalloc(&p->cell_block, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->cell_block = nullptr;
        return fail(KAPPA_ENOMEM, "hipMalloc of %zu bytes for the cell table failed", bytes);
    }
    std::vector<unsigned char> host(bytes, 0);
    std::memcpy(host.data(), c32.data(), c32.size() * sizeof(CellF32));
    std::memcpy(host.data() + o64, c64.data(), c64.size() * sizeof(CellF64));
    kappa_status st = check_hip(hipMemcpy(p->cell_block, host.data(), bytes, hipMemcpyHostToDevice),
                                "hipMemcpy cell table");
    if (st != KAPPA_OK) {
        (void)hipFree(p->cell_block);
        p->cell_block = nullptr;
        return st;
    }
    auto *base = static_cast<unsigned char *>(p->cell_block);
    p->cell32 = reinterpret_cast<const CellF32 *>(base);
    p->cell64 = reinterpret_cast<const CellF64 *>(base + o64);
    return KAPPA_OK;
}

extern "C" kappa_status kappa_plan_autotune_impl(kappa_plan p, void *vx, void *vy, void *vz, int reps, void *stream)
{
    const Outputs o = velocities(vx, vy, vz);
    const kappa_status cs = check_plan_outputs(p, o);
    if (cs != KAPPA_OK || p->total == 0) return cs;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    kappa_status s = check_hip(hipEventCreate(&e0), "hipEventCreate");
    if (s != KAPPA_OK) return s;
    s = check_hip(hipEventCreate(&e1), "hipEventCreate");
    if (s != KAPPA_OK) {
        (void)hipEventDestroy(e0);
        return s;
    }
    const int cus = device_cu_count();
    const int blocks[] = {64, 128, 256};
    const int unrolls[] = {1, 2, 4, 8};
    const int per_cu[] = {0, 1, 2, 4, 8, 16};  // 0: one thread per group
    float best_ms = 1e30f;
    Shape best = p->shape;
    for (int b : blocks)
        for (int u : unrolls)
            for (int w : per_cu) {
                const uint64_t groups = (p->total + u - 1) / u;
                const uint64_t need = (groups + b - 1) / b;
                Shape cand{b, u, w > 0 ? w * cus : static_cast<int>(std::min<uint64_t>(need, 1ull << 23))};
                if (w > 0 && static_cast<uint64_t>(cand.grid) >= need) continue;  // same as one pass
                if (!aligned_for(p->mode, cand, o)) continue;
                const BatchArgs a = batch_args(p, o);
                hipError_t err = launch_batched(p->mode, cand, a, st);  // warm-up
                if (err != hipSuccess) {
                    s = check_hip(err, "autotune launch");
                    goto done;
                }
                err = hipEventRecord(e0, st);
                for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch_batched(p->mode, cand, a, st);
                if (err == hipSuccess) err = hipEventRecord(e1, st);
                if (err == hipSuccess) err = hipEventSynchronize(e1);
                float ms = 0.f;
                if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                s = check_hip(err, "autotune timing");
                if (s != KAPPA_OK) goto done;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                }
            }
    p->shape = best;
    cache_store(cache_key(p->mode, p->total, p->nseg), best);
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

extern "C" kappa_status kappa_plan_shape_impl(kappa_plan p, int *block, int *unroll, int *grid)
{
    if (block) *block = p->shape.block;
    if (unroll) *unroll = p->shape.unroll;
    if (grid) *grid = p->shape.grid;
    return KAPPA_OK;
}

extern "C" kappa_status kappa_plan_set_shape_impl(kappa_plan p, int block, int unroll, int grid)
{
    const Shape s{block, unroll, grid};
    if (!shape_valid(s)) return fail(KAPPA_EINVAL, "invalid launch shape (%d, %d, %d)", block, unroll, grid);
    p->shape = s;
    return KAPPA_OK;
}

extern "C" kappa_status kappa_plan_total_impl(kappa_plan p, uint64_t *total)
{
    *total = p->total;
    return KAPPA_OK;
}

extern "C" kappa_status kappa_plan_destroy_impl(kappa_plan p)
{
    PlanDevice guard(p);
    // launches of this plan may still be in flight on any stream
    (void)hipDeviceSynchronize();
    drop_graph(p);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->dev_block) (void)hipFree(p->dev_block);
    if (p->cell_block) (void)hipFree(p->cell_block);
    delete p;
    return KAPPA_OK;
}
