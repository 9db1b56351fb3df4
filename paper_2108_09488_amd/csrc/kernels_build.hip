// kernels_build.hip -- cell-linked list on gfx950: fixed-point hashing of the
// particles into cells, a one-pass counting sort by cell key (histogram by
// atomic tickets, exclusive scan = cell-start table, scatter), and a
// canonicalisation that orders the particles of each cell by id so that the
// sorted order is a pure function of the positions (deterministic pair sums).
// Also: read-back of C and x in id order and the FP64 mass reduction.
#include "ade_device.h"

namespace ade {

// ---------------------------------------------------------------------------
// init: positions (double, SoA) -> fixed point, first hash + ticket
// ---------------------------------------------------------------------------
template <int DIM, typename real>
__global__ __launch_bounds__(kTile) void k_init(const PlumeDev* __restrict__ plumes,
                                               const TileDev* __restrict__ tiles,
                                               const double* __restrict__ x,
                                               const real* __restrict__ C, uint32_t N,
                                               StateArrays U, uint32_t* __restrict__ count) {
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
    U.tick[i] = atomicAdd(&count[key], 1u);
}

// ---------------------------------------------------------------------------
// exclusive scan of the per-cell counts -> cell_start; counts are cleared.
// The tables are padded to whole 1024-cell chunks with zero counts, so the
// entry after the last cell receives the particle total (the sentinel).
// Three launches: chunk totals, a one-workgroup scan of the totals, and the
// chunk scans with their offsets.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cscan_reduce(const uint4* __restrict__ count,
                                                     uint32_t* __restrict__ partial) {
    __shared__ uint32_t lds[256 / kWave];
    const uint4 c = count[blockIdx.x * 256 + threadIdx.x];
    const uint32_t s = block_sum(c.x + c.y + c.z + c.w, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_cscan_mid(uint32_t* __restrict__ partial, uint32_t nb) {
    __shared__ uint32_t lds[1024 / kWave];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += 4096) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t j = base + threadIdx.x * 4 + k;
            v[k] = (j < nb) ? partial[j] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(s, lds, tot) + carry;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t j = base + threadIdx.x * 4 + k;
            if (j < nb) partial[j] = ex;
            ex += v[k];
        }
        carry += tot;
    }
}

__global__ __launch_bounds__(256) void k_cscan_final(uint4* __restrict__ count,
                                                    const uint32_t* __restrict__ prefix,
                                                    uint4* __restrict__ cell_start) {
    __shared__ uint32_t lds[256 / kWave];
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    const uint4 c = count[j];
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(c.x + c.y + c.z + c.w, lds, tot) + prefix[blockIdx.x];
    uint4 o;
    o.x = ex;
    o.y = ex + c.x;
    o.z = o.y + c.y;
    o.w = o.z + c.z;
    cell_start[j] = o;
    count[j] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_scan(const uint32_t* count_in, uint32_t* cell_start, uint32_t* partial,
                       uint32_t ncell, hipStream_t s) {
    const uint32_t nb = (uint32_t)(cell_pad(ncell) / kCellChunk);
    uint4* cnt = reinterpret_cast<uint4*>(const_cast<uint32_t*>(count_in));
    hipLaunchKernelGGL(k_cscan_reduce, dim3(nb), dim3(256), 0, s, cnt, partial);
    hipLaunchKernelGGL(k_cscan_mid, dim3(1), dim3(1024), 0, s, partial, nb);
    hipLaunchKernelGGL(k_cscan_final, dim3(nb), dim3(256), 0, s, cnt, partial,
                       reinterpret_cast<uint4*>(cell_start));
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
                                                            uint32_t n, uint32_t nb) {
    __shared__ int64_t lds[kScanBlock / kWave];
    int64_t pre = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += blockDim.x) pre += partial[b];
    pre = block_sum(pre, lds);
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
    hipLaunchKernelGGL(k_scan64_partial, dim3(nb), dim3(kScanBlock), 0, s, data, partial, n);
    hipLaunchKernelGGL(k_scan64_final, dim3(nb), dim3(kScanBlock), 0, s, data, partial, n, nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scatter by (cell start + ticket), then order each cell by particle id
// ---------------------------------------------------------------------------
template <int DIM, typename real>
__global__ __launch_bounds__(256) void k_scatter(StateArrays U, StateArrays T,
                                                const uint32_t* __restrict__ cell_start,
                                                uint32_t N) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t key = U.key[i];
    const uint32_t slot = cell_start[key] + U.tick[i];
#pragma unroll
    for (int c = 0; c < DIM; ++c) T.pos[c][slot] = U.pos[c][i];
    static_cast<real*>(T.C)[slot] = static_cast<const real*>(U.C)[i];
    T.id[slot] = U.id[i];
    T.key[slot] = key;
}

template <int DIM, typename real>
__global__ __launch_bounds__(256) void k_canon(StateArrays T, StateArrays S,
                                              const uint32_t* __restrict__ cell_start,
                                              uint32_t N, int64_t* step, int inc_step) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (inc_step && j == 0) *step += 1;
    if (j >= N) return;
    const uint32_t key = T.key[j];
    const uint32_t s = cell_start[key], e = cell_start[key + 1];
    const uint32_t my = T.id[j];
    uint32_t rank = 0;
    for (uint32_t k = s; k < e; ++k) rank += (T.id[k] < my) ? 1u : 0u;
    const uint32_t d = s + rank;
    uint32_t u[3] = {0u, 0u, 0u};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        u[c] = T.pos[c][j];
        S.pos[c][d] = u[c];
    }
    const real C = static_cast<const real*>(T.C)[j];
    static_cast<real*>(S.C)[d] = C;
    S.id[d] = my;
    if (Rec<DIM, real>::kStageable) S.rec[d] = Rec<DIM, real>::pack(u[0], u[1], u[2], C);
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
                       StateArrays U, uint32_t* count, hipStream_t s) {
    dim3 g(ntiles), b(kTile);
    if (dim == 2 && real_bytes == 4)
        hipLaunchKernelGGL((k_init<2, float>), g, b, 0, s, plumes, tiles, x, (const float*)C, N, U, count);
    else if (dim == 2)
        hipLaunchKernelGGL((k_init<2, double>), g, b, 0, s, plumes, tiles, x, (const double*)C, N, U, count);
    else if (real_bytes == 4)
        hipLaunchKernelGGL((k_init<3, float>), g, b, 0, s, plumes, tiles, x, (const float*)C, N, U, count);
    else
        hipLaunchKernelGGL((k_init<3, double>), g, b, 0, s, plumes, tiles, x, (const double*)C, N, U, count);
    return hipGetLastError();
}

hipError_t launch_scatter(int dim, int real_bytes, StateArrays U, StateArrays T,
                          const uint32_t* cell_start, uint32_t N, hipStream_t s) {
    dim3 g((N + 255) / 256), b(256);
    if (dim == 2 && real_bytes == 4) hipLaunchKernelGGL((k_scatter<2, float>), g, b, 0, s, U, T, cell_start, N);
    else if (dim == 2) hipLaunchKernelGGL((k_scatter<2, double>), g, b, 0, s, U, T, cell_start, N);
    else if (real_bytes == 4) hipLaunchKernelGGL((k_scatter<3, float>), g, b, 0, s, U, T, cell_start, N);
    else hipLaunchKernelGGL((k_scatter<3, double>), g, b, 0, s, U, T, cell_start, N);
    return hipGetLastError();
}

hipError_t launch_canon(int dim, int real_bytes, StateArrays T, StateArrays S,
                        const uint32_t* cell_start, uint32_t N, int64_t* step, int inc_step,
                        hipStream_t s) {
    dim3 g((N + 255) / 256), b(256);
    if (dim == 2 && real_bytes == 4) hipLaunchKernelGGL((k_canon<2, float>), g, b, 0, s, T, S, cell_start, N, step, inc_step);
    else if (dim == 2) hipLaunchKernelGGL((k_canon<2, double>), g, b, 0, s, T, S, cell_start, N, step, inc_step);
    else if (real_bytes == 4) hipLaunchKernelGGL((k_canon<3, float>), g, b, 0, s, T, S, cell_start, N, step, inc_step);
    else hipLaunchKernelGGL((k_canon<3, double>), g, b, 0, s, T, S, cell_start, N, step, inc_step);
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

hipError_t launch_mass(int real_bytes, const PlumeDev* plumes, int nplumes, const TileDev* tiles,
                       uint32_t ntiles, StateArrays S, double* partial, double* out,
                       hipStream_t s) {
    if (real_bytes == 4) hipLaunchKernelGGL((k_mass_tiles<float>), dim3(ntiles), dim3(kTile), 0, s, tiles, S, partial);
    else hipLaunchKernelGGL((k_mass_tiles<double>), dim3(ntiles), dim3(kTile), 0, s, tiles, S, partial);
    hipLaunchKernelGGL(k_mass_plumes, dim3(nplumes), dim3(256), 0, s, plumes, partial, out);
    return hipGetLastError();
}

}  // namespace ade
