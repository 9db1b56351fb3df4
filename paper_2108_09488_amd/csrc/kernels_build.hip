// kernels_build.hip -- cell-linked list on gfx950: fixed-point hashing of the
// particles into cells, a counting sort by cell key (histogram and per-cell
// buckets by atomics, exclusive scan = cell-start table) whose placement
// orders the particles of each cell by id, so that the sorted order is a pure
// function of the positions (deterministic pair sums).
// Also: read-back of C and x in id order and the FP64 mass reduction.
#include "ade_device.h"

namespace ade {

// ---------------------------------------------------------------------------
// init: positions (double, SoA) -> fixed point, first hash and counting pass
// ---------------------------------------------------------------------------
template <int DIM, typename real>
__global__ __launch_bounds__(kTile) void k_init(const PlumeDev* __restrict__ plumes,
                                               const TileDev* __restrict__ tiles,
                                               const double* __restrict__ x,
                                               const real* __restrict__ C, uint32_t N,
                                               StateArrays U, CellLists lists) {
    const TileDev t = tiles[blockIdx.x];
    const PlumeDev& P = plumes[t.plume];
    const uint32_t i = t.start + threadIdx.x;
    if (i >= t.end) return;
    uint32_t u[3] = {0u, 0u, 0u};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double f = rint((x[(size_t)c * N + i] / P.L) * 4294967296.0);
        u[c] = (uint32_t)(int64_t)f;  // modulo 2^32: periodic wrap
        U.pos[c][i] = u[c];
    }
    static_cast<real*>(U.C)[i] = C[i];
    U.id[i] = i;
    const uint32_t key = cell_key<DIM>(P, u[0], u[1], u[2]);
    U.key[i] = key;
    enlist(lists, key, i);  // id = index here
}

// ---------------------------------------------------------------------------
// exclusive scan of the per-cell counts -> cell_start; counts are cleared.
// The tables are padded to whole 1024-cell chunks with zero counts, so the
// entry after the last cell receives the particle total (the sentinel).
// Two launches: the chunk totals, then every workgroup sums the totals of
// the chunks before its own (read by all its threads at once) and scans its
// chunk.  Past kDirectChunks chunks that sum would grow with the square of
// the table, so one workgroup scans the totals in place between the two
// launches and each chunk reads its own prefix.
// ---------------------------------------------------------------------------
constexpr int kCellVec = kCellChunk / (256 * 4);  // uint4 of counts per thread, contiguous
// chunks whose prefixes the final launch sums itself: 4096 for the cell scan
// of every step (the 2D sweep's 2.1M cells and the 3D plume's 3.6M take the
// two-launch path; a third launch for the totals cost the sweep's step 1.3%),
// 2048 for the neighbour-offset scan
constexpr uint32_t kDirectChunks = 4096;
constexpr uint32_t kDirectChunks64 = 2048;
constexpr int kPrefixBlock = 1024;                 // the workgroup of k_scan_prefix

// Exclusive scan in place of n chunk totals by one workgroup, in passes of
// 4 consecutive totals per thread carried from pass to pass.
template <typename T>
__global__ __launch_bounds__(kPrefixBlock) void k_scan_prefix(T* __restrict__ p, uint32_t n) {
    __shared__ T lds[kPrefixBlock / kWave];
    T carry = 0;
    for (uint32_t base = 0; base < n; base += 4u * kPrefixBlock) {
        const uint32_t j = base + 4u * threadIdx.x;
        T v[4];
        T s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = (j + k < n) ? p[j + k] : T(0);
            s += v[k];
        }
        T tot;
        T ex = block_exclusive_scan(s, lds, tot) + carry;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (j + k < n) p[j + k] = ex;
            ex += v[k];
        }
        carry += tot;
    }
}

// The total of the chunks before this workgroup's: summed here, or (after
// k_scan_prefix) read.
template <typename T>
__device__ __forceinline__ T chunk_prefix(const T* __restrict__ partial, uint32_t direct, T* lds) {
    if (!direct) return partial[blockIdx.x];
    // 16-byte loads of the totals (the array is 256-byte aligned), then the
    // few past the last whole vector
    constexpr uint32_t kPer = 16 / sizeof(T);
    struct alignas(16) Vec {
        T v[kPer];
    };
    const Vec* __restrict__ pv = reinterpret_cast<const Vec*>(partial);
    const uint32_t nv = blockIdx.x / kPer;
    T pre = 0;
    for (uint32_t b = threadIdx.x; b < nv; b += blockDim.x) {
        const Vec q = pv[b];
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) pre += q.v[k];
    }
    for (uint32_t b = nv * kPer + threadIdx.x; b < blockIdx.x; b += blockDim.x) pre += partial[b];
    return block_sum(pre, lds);
}

__global__ __launch_bounds__(256) void k_cscan_reduce(const uint4* __restrict__ count,
                                                     uint32_t* __restrict__ partial,
                                                     uint32_t* __restrict__ ovf_count) {
    __shared__ uint32_t lds[256 / kWave];
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // the overflow pairs of this build; restart the count
        ovf_count[1] = ovf_count[0];
        ovf_count[0] = 0;
    }
    const uint32_t j0 = (blockIdx.x * 256 + threadIdx.x) * kCellVec;
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < kCellVec; ++k) {
        const uint4 c = count[j0 + k];
        mine += c.x + c.y + c.z + c.w;
    }
    const uint32_t s = block_sum(mine, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_cscan_final(uint4* __restrict__ count,
                                                    const uint32_t* __restrict__ partial,
                                                    uint4* __restrict__ cell_start, uint32_t direct) {
    __shared__ uint32_t lds[256 / kWave];
    const uint32_t pre = chunk_prefix(partial, direct, lds);
    const uint32_t j0 = (blockIdx.x * 256 + threadIdx.x) * kCellVec;
    uint4 c[kCellVec];
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < kCellVec; ++k) {
        c[k] = count[j0 + k];
        mine += c[k].x + c[k].y + c[k].z + c[k].w;
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(mine, lds, tot) + pre;
#pragma unroll
    for (int k = 0; k < kCellVec; ++k) {
        uint4 o;
        o.x = run;
        o.y = o.x + c[k].x;
        o.z = o.y + c[k].y;
        o.w = o.z + c[k].z;
        run = o.w + c[k].w;
        cell_start[j0 + k] = o;
        count[j0 + k] = make_uint4(0u, 0u, 0u, 0u);
    }
}

hipError_t launch_scan(CellLists lists, uint32_t* cell_start, uint32_t* partial, uint32_t ncell,
                       hipStream_t s) {
    const uint32_t nchunks = (uint32_t)(cell_pad(ncell) / kCellChunk);
    uint4* cnt = reinterpret_cast<uint4*>(lists.count);
    const uint32_t direct = nchunks <= kDirectChunks ? 1u : 0u;
    hipLaunchKernelGGL(k_cscan_reduce, dim3(nchunks), dim3(256), 0, s, cnt, partial, lists.ovf_count);
    if (!direct) hipLaunchKernelGGL((k_scan_prefix<uint32_t>), dim3(1), dim3(kPrefixBlock), 0, s, partial, nchunks);
    hipLaunchKernelGGL(k_cscan_final, dim3(nchunks), dim3(256), 0, s, cnt, partial,
                       reinterpret_cast<uint4*>(cell_start), direct);
    return hipGetLastError();
}

// int64 exclusive scan in place (neighbour offsets); data has n + 1 entries,
// data[n] receives the total.
__global__ __launch_bounds__(kScanBlock) void k_scan64_partial(const int64_t* __restrict__ d,
                                                              int64_t* __restrict__ partial,
                                                              uint32_t n) {
    __shared__ int64_t lds[kScanBlock / kWave];
    const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * kScanPerThread;
    int64_t s = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint32_t j = base + k;
        s += (j < n) ? d[j] : 0;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kScanBlock) void k_scan64_final(int64_t* __restrict__ d,
                                                            const int64_t* __restrict__ partial,
                                                            uint32_t n, uint32_t nb, uint32_t direct) {
    __shared__ int64_t lds[kScanBlock / kWave];
    const int64_t pre = chunk_prefix(partial, direct, lds);
    const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * kScanPerThread;
    int64_t v[kScanPerThread];
    int64_t s = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint32_t j = base + k;
        v[k] = (j < n) ? d[j] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, lds, tot) + pre;
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint32_t j = base + k;
        if (j < n) d[j] = ex;
        ex += v[k];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == blockDim.x - 1) d[n] = ex;
}

hipError_t launch_scan64(int64_t* data, uint32_t n, int64_t* partial, hipStream_t s) {
    const uint32_t nb = (n + kScanChunk - 1) / kScanChunk;
    const uint32_t direct = nb <= kDirectChunks64 ? 1u : 0u;
    hipLaunchKernelGGL(k_scan64_partial, dim3(nb), dim3(kScanBlock), 0, s, data, partial, n);
    if (!direct) hipLaunchKernelGGL((k_scan_prefix<int64_t>), dim3(1), dim3(kPrefixBlock), 0, s, partial, nb);
    hipLaunchKernelGGL(k_scan64_final, dim3(nb), dim3(kScanBlock), 0, s, data, partial, n, nb, direct);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// placement: every particle of U goes to cell_start[key] + (its rank by id
// among the particles of its cell), found from the ids in the cell's bucket
// (and, for a cell of more than kBucket particles, the overflow list), so the sorted
// order is a pure function of the positions.  Writes the sorted state S and
// its candidate records (and, for a velocity field, its velocity and
// tensor); advances the step counter if asked.
// ---------------------------------------------------------------------------
template <int DIM, typename real>
__global__ __launch_bounds__(256) void k_place(StateArrays U, StateArrays S, CellLists L,
                                              const uint32_t* __restrict__ cell_start, uint32_t N,
                                              int64_t* step, int inc_step) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (inc_step && i == 0) *step += 1;
    if (i >= N) return;
    const uint32_t key = U.key[i];
    const uint32_t my = U.id[i];
    const uint32_t s = cell_start[key];
    const uint32_t n = cell_start[key + 1] - s;
    uint32_t rank = 0;
    if (n > 1) {  // alone in its cell: rank 0
        const uint4* __restrict__ bq = reinterpret_cast<const uint4*>(L.bucket + (size_t)key * kBucket);
        const uint4 b0 = bq[0];
        const uint4 b1 = (n > 4) ? bq[1] : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t m[kBucket] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (uint32_t t = 0; t < kBucket; ++t) rank += (t < n && m[t] < my) ? 1u : 0u;
        if (n > kBucket) {  // crowded cell: the rest of it is in the overflow list
            const uint32_t no = L.ovf_count[1];
            for (uint32_t p = 0; p < no; ++p) {
                const uint2 e = L.ovf[p];
                if (e.x == key) rank += (e.y < my) ? 1u : 0u;
            }
        }
    }
    const uint32_t d = s + rank;
    uint32_t u[3] = {0u, 0u, 0u};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        u[c] = U.pos[c][i];
        S.pos[c][d] = u[c];
    }
    const real C = static_cast<const real*>(U.C)[i];
    static_cast<real*>(S.C)[d] = C;
    S.id[d] = my;
    if (Rec<DIM, real>::kStageable) S.rec[d] = Rec<DIM, real>::pack(u[0], u[1], u[2], C);
    if (U.vel[0]) {  // velocity field: the particle's velocity and tensor travel with it
        real w[DIM + (DIM == 2 ? 3 : 6)];
#pragma unroll
        for (int c = 0; c < DIM; ++c) w[c] = static_cast<const real*>(U.vel[c])[i];
#pragma unroll
        for (int q = 0; q < (DIM == 2 ? 3 : 6); ++q) w[DIM + q] = static_cast<const real*>(U.rD[q])[i];
#pragma unroll
        for (int c = 0; c < DIM; ++c) static_cast<real*>(S.vel[c])[d] = w[c];
#pragma unroll
        for (int q = 0; q < (DIM == 2 ? 3 : 6); ++q) static_cast<real*>(S.rD[q])[d] = w[DIM + q];
        if (U.Cb) static_cast<real*>(S.Cb)[d] = static_cast<const real*>(U.Cb)[i];
        if (DIM == 2 && sizeof(real) == 4 && S.grec) {
            auto bits = [](real f) { return __float_as_uint((float)f); };
            S.grec[2 * (size_t)d] = make_uint4(u[0], u[1], bits(C), bits(w[0]));
            S.grec[2 * (size_t)d + 1] = make_uint4(bits(w[1]), bits(w[2]), bits(w[3]), bits(w[4]));
        }
    }
}

// ---------------------------------------------------------------------------
// read-back and mass
// ---------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void k_read_C(StateArrays S, uint32_t N, real* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    out[S.id[i]] = static_cast<const real*>(S.C)[i];
}

template <int DIM>
__global__ __launch_bounds__(kTile) void k_read_x(const PlumeDev* __restrict__ plumes,
                                                 const TileDev* __restrict__ tiles, StateArrays S,
                                                 uint32_t N, double* __restrict__ out) {
    const TileDev t = tiles[blockIdx.x];
    const double scale = plumes[t.plume].L * (1.0 / 4294967296.0);
    const uint32_t i = t.start + threadIdx.x;
    if (i >= t.end) return;
    const uint32_t id = S.id[i];
#pragma unroll
    for (int c = 0; c < DIM; ++c) out[(size_t)c * N + id] = (double)S.pos[c][i] * scale;
}

template <typename real>
__global__ __launch_bounds__(kTile) void k_mass_tiles(const TileDev* __restrict__ tiles,
                                                     StateArrays S, double* __restrict__ partial) {
    __shared__ double lds[kTile / kWave];
    const TileDev t = tiles[blockIdx.x];
    const uint32_t i = t.start + threadIdx.x;
    double c = (i < t.end) ? (double)static_cast<const real*>(S.C)[i] : 0.0;
    c = block_sum(c, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = c;
}

__global__ __launch_bounds__(256) void k_mass_plumes(const PlumeDev* __restrict__ plumes,
                                                    const double* __restrict__ partial,
                                                    double* __restrict__ out) {
    __shared__ double lds[256 / kWave];
    const PlumeDev& P = plumes[blockIdx.x];
    double s = 0.0;
    for (uint32_t k = threadIdx.x; k < P.tcount; k += blockDim.x) s += partial[P.tfirst + k];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = P.mass * s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_init(int dim, int real_bytes, const PlumeDev* plumes, const TileDev* tiles,
                       uint32_t ntiles, const double* x, const void* C, uint32_t N,
                       StateArrays U, CellLists lists, hipStream_t s) {
    dim3 g(ntiles), b(kTile);
    if (dim == 2 && real_bytes == 4)
        hipLaunchKernelGGL((k_init<2, float>), g, b, 0, s, plumes, tiles, x, (const float*)C, N, U, lists);
    else if (dim == 2)
        hipLaunchKernelGGL((k_init<2, double>), g, b, 0, s, plumes, tiles, x, (const double*)C, N, U, lists);
    else if (real_bytes == 4)
        hipLaunchKernelGGL((k_init<3, float>), g, b, 0, s, plumes, tiles, x, (const float*)C, N, U, lists);
    else
        hipLaunchKernelGGL((k_init<3, double>), g, b, 0, s, plumes, tiles, x, (const double*)C, N, U, lists);
    return hipGetLastError();
}

hipError_t launch_place(int dim, int real_bytes, StateArrays U, StateArrays S, CellLists lists,
                        const uint32_t* cell_start, uint32_t N, int64_t* step, int inc_step,
                        hipStream_t s) {
    dim3 g((N + 255) / 256), b(256);
    if (dim == 2 && real_bytes == 4)
        hipLaunchKernelGGL((k_place<2, float>), g, b, 0, s, U, S, lists, cell_start, N, step, inc_step);
    else if (dim == 2)
        hipLaunchKernelGGL((k_place<2, double>), g, b, 0, s, U, S, lists, cell_start, N, step, inc_step);
    else if (real_bytes == 4)
        hipLaunchKernelGGL((k_place<3, float>), g, b, 0, s, U, S, lists, cell_start, N, step, inc_step);
    else
        hipLaunchKernelGGL((k_place<3, double>), g, b, 0, s, U, S, lists, cell_start, N, step, inc_step);
    return hipGetLastError();
}

hipError_t launch_read_C(int real_bytes, StateArrays S, uint32_t N, void* out, hipStream_t s) {
    dim3 g((N + 255) / 256), b(256);
    if (real_bytes == 4) hipLaunchKernelGGL((k_read_C<float>), g, b, 0, s, S, N, (float*)out);
    else hipLaunchKernelGGL((k_read_C<double>), g, b, 0, s, S, N, (double*)out);
    return hipGetLastError();
}

hipError_t launch_read_x(int dim, const PlumeDev* plumes, const TileDev* tiles, uint32_t ntiles,
                         StateArrays S, uint32_t N, double* out, hipStream_t s) {
    if (dim == 2) hipLaunchKernelGGL((k_read_x<2>), dim3(ntiles), dim3(kTile), 0, s, plumes, tiles, S, N, out);
    else hipLaunchKernelGGL((k_read_x<3>), dim3(ntiles), dim3(kTile), 0, s, plumes, tiles, S, N, out);
    return hipGetLastError();
}

// Coincident positions: any particle of the sorted state that shares its
// position with another particle of its cell (two particles at one point are
// in one cell) sets *flag.  Cells hold a few particles, so each particle
// compares itself with the rest of its cell.
template <int DIM>
__global__ __launch_bounds__(kTile) void k_coincident(const PlumeDev* __restrict__ plumes,
                                                     const TileDev* __restrict__ tiles, StateArrays S,
                                                     const uint32_t* __restrict__ cell_start,
                                                     uint32_t* __restrict__ flag) {
    const TileDev t = tiles[blockIdx.x];
    const uint32_t i = t.start + threadIdx.x;
    if (i >= t.end) return;
    const PlumeDev& P = plumes[t.plume];
    const uint32_t ux = S.pos[0][i], uy = S.pos[1][i], uz = (DIM == 3) ? S.pos[2][i] : 0u;
    const uint32_t key = cell_key<DIM>(P, ux, uy, uz);
    const uint32_t e = cell_start[key + 1];
    bool same = false;
    for (uint32_t j = cell_start[key]; j < e; ++j)
        same |= j != i && S.pos[0][j] == ux && S.pos[1][j] == uy && (DIM == 2 || S.pos[2][j] == uz);
    if (same) *flag = 1u;
}

hipError_t launch_coincident(int dim, const PlumeDev* plumes, const TileDev* tiles, uint32_t ntiles,
                             StateArrays S, const uint32_t* cell_start, uint32_t* flag, hipStream_t s) {
    if (dim == 2) hipLaunchKernelGGL((k_coincident<2>), dim3(ntiles), dim3(kTile), 0, s, plumes, tiles, S, cell_start, flag);
    else hipLaunchKernelGGL((k_coincident<3>), dim3(ntiles), dim3(kTile), 0, s, plumes, tiles, S, cell_start, flag);
    return hipGetLastError();
}

hipError_t launch_mass(int real_bytes, const PlumeDev* plumes, int nplumes, const TileDev* tiles,
                       uint32_t ntiles, StateArrays S, double* partial, double* out,
                       hipStream_t s) {
    if (real_bytes == 4) hipLaunchKernelGGL((k_mass_tiles<float>), dim3(ntiles), dim3(kTile), 0, s, tiles, S, partial);
    else hipLaunchKernelGGL((k_mass_tiles<double>), dim3(ntiles), dim3(kTile), 0, s, tiles, S, partial);
    hipLaunchKernelGGL(k_mass_plumes, dim3(nplumes), dim3(256), 0, s, plumes, partial, out);
    return hipGetLastError();
}

}  // namespace ade
