// Stable LSD radix sort of (uint32 or uint64 key, int32 value) pairs on the device, 8-bit
// digits: per pass, digit counts of every tile, one exclusive scan over the
// counts laid out digit-major (so each tile's share of a digit follows the
// earlier tiles'), then a scatter that keeps the order of equal digits inside
// a tile.  Plain kernel launches only (no memset, no host synchronisation),
// so a caller may capture it in a graph.  Used to put the stepping work list
// in spatial order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qsq_internal.h"

namespace qsq {

constexpr int kSortThreads = 256, kSortItems = 8, kSortTile = kSortThreads * kSortItems;

static int64_t sort_tiles(int64_t n_max) { return (n_max + kSortTile - 1) / kSortTile; }

int64_t sort_count_words(int64_t n_max) { return 256 * (sort_tiles(n_max) > 0 ? sort_tiles(n_max) : 1); }

// cnt[d * tiles + t] = items of tile t whose digit is d
template <typename K>
__global__ void __launch_bounds__(256) k_sort_count(const K *keys, const int64_t *n_dev, int64_t tiles,
                                                    int shift, int32_t *cnt)
{
    __shared__ int32_t h[256];
    const int64_t n = *n_dev;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        h[threadIdx.x] = 0;
        __syncthreads();
        const int64_t base = t * kSortTile;
        for (int k = 0; k < kSortItems; ++k) {
            const int64_t i = base + (int64_t)k * kSortThreads + threadIdx.x;
            if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1);
        }
        __syncthreads();
        cnt[(int64_t)threadIdx.x * tiles + t] = h[threadIdx.x];
        __syncthreads();
    }
}

// Items of a tile in rounds of 256 (index order = round, then thread); an
// item's place among the tile's items of its digit = items of that digit in
// earlier rounds + in lower waves of this round + in lower lanes of its wave
// (lanes with the same digit found with 8 ballots).
template <typename K>
__global__ void __launch_bounds__(256) k_sort_scatter(const K *kin, const int32_t *vin, const int64_t *n_dev,
                                                      int64_t tiles, int shift, const int32_t *off, K *kout,
                                                      int32_t *vout)
{
    __shared__ int32_t run[256];
    __shared__ int32_t wcnt[4][256];
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lower = (1ull << lane) - 1ull;
    const int64_t n = *n_dev;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        run[tid] = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t base = t * kSortTile;
        for (int k = 0; k < kSortItems; ++k) {
            const int64_t i = base + (int64_t)k * kSortThreads + tid;
            const bool valid = i < n;
            const K key = valid ? kin[i] : (K)0;
            const int32_t val = valid ? vin[i] : 0;
            const int d = (int)((uint32_t)(key >> shift) & 255u);
            uint64_t same = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint64_t ones = __ballot((d >> b) & 1);
                same &= ((d >> b) & 1) ? ones : ~ones;
            }
            const int rank = __popcll(same & lower);
            if (valid && rank == 0) wcnt[wave][d] = __popcll(same);
            __syncthreads();
            if (valid) {
                int before = run[d] + rank;
                for (int w = 0; w < wave; ++w) before += wcnt[w][d];
                const int64_t pos = (int64_t)off[(int64_t)d * tiles + t] + before;
                kout[pos] = key;
                vout[pos] = val;
            }
            __syncthreads();
            run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
#pragma unroll
            for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
            __syncthreads();
        }
    }
}

template <typename K>
__global__ void k_sort_copy(const K *ks, const int32_t *vs, const int64_t *n_dev, K *kd, int32_t *vd)
{
    const int64_t n = *n_dev;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

__global__ void k_sort_set_count(int64_t *p, int64_t v) { *p = v; }

template <typename K>
static void sort_pairs(K *keys, int32_t *vals, K *keys_tmp, int32_t *vals_tmp, int32_t *cnt, int64_t *scan_tmp,
                       int64_t *n_cnt, const int64_t *n_dev, int64_t n_max, int key_bits, hipStream_t st)
{
    const int64_t tiles = sort_tiles(n_max);
    if (tiles <= 0 || key_bits <= 0) return;
    const int cus = device_cu_count();
    const int blocks = (int)(tiles < (int64_t)cus * 8 ? tiles : (int64_t)cus * 8);
    hipLaunchKernelGGL(k_sort_set_count, dim3(1), dim3(1), 0, st, n_cnt, 256 * tiles);
    K *ka = keys, *kb = keys_tmp;
    int32_t *va = vals, *vb = vals_tmp;
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(k_sort_count<K>, dim3(blocks), dim3(256), 0, st, ka, n_dev, tiles, shift, cnt);
        // the scan's total (the item count) lands in n_cnt + 1
        launch_scan_i32(cnt, n_cnt, 256 * tiles, scan_tmp, cnt, n_cnt + 1, st);
        hipLaunchKernelGGL(k_sort_scatter<K>, dim3(blocks), dim3(256), 0, st, ka, va, n_dev, tiles, shift, cnt, kb,
                           vb);
        K *kt = ka;
        ka = kb;
        kb = kt;
        int32_t *vt = va;
        va = vb;
        vb = vt;
    }
    if (ka != keys) {
        const int cb = (int)((n_max + 255) / 256 < (int64_t)cus * 16 ? (n_max + 255) / 256 : (int64_t)cus * 16);
        hipLaunchKernelGGL(k_sort_copy<K>, dim3(cb), dim3(256), 0, st, ka, va, n_dev, keys, vals);
    }
}

void launch_sort_pairs(uint32_t *keys, int32_t *vals, uint32_t *keys_tmp, int32_t *vals_tmp, int32_t *cnt,
                       int64_t *scan_tmp, int64_t *n_cnt, const int64_t *n_dev, int64_t n_max, int key_bits,
                       hipStream_t st)
{
    sort_pairs<uint32_t>(keys, vals, keys_tmp, vals_tmp, cnt, scan_tmp, n_cnt, n_dev, n_max, key_bits, st);
}

void launch_sort_pairs64(uint64_t *keys, int32_t *vals, uint64_t *keys_tmp, int32_t *vals_tmp, int32_t *cnt,
                         int64_t *scan_tmp, int64_t *n_cnt, const int64_t *n_dev, int64_t n_max, int key_bits,
                         hipStream_t st)
{
    sort_pairs<uint64_t>(keys, vals, keys_tmp, vals_tmp, cnt, scan_tmp, n_cnt, n_dev, n_max, key_bits, st);
}

}  // namespace qsq
