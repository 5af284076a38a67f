// Exclusive scan on one workgroup of 1024 threads (device code shared by the
// grid sort and the pair-list kernels).
#pragma once

#include <hip/hip_runtime.h>

namespace mxn {

// Exclusive scan on one workgroup of 1024 threads; mode 0: values as is,
// 1: rounded up to a multiple of p, 2: ceil(v/p).  raw_total (optional)
// receives the sum of the untransformed values; clear (optional, the input
// array itself) is zeroed once read.  The input goes through LDS in tiles of
// 8192 values: each thread issues its eight coalesced loads of a tile
// together, scans eight consecutive values from LDS, and the 1024 chunk sums
// are scanned across the workgroup (wavefront scans, then the 16 wavefront
// totals); a running carry joins the tiles.
constexpr int kScanPer = 8, kScanTile = 1024 * kScanPer;

// inclusive scans of (s, r) over the workgroup's 1024 threads
__device__ inline void block_scan2(int &s, int &r, int *ws, int *wr) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int a = __shfl_up(s, o, 64), b = __shfl_up(r, o, 64);
        if (lane >= o) {
            s += a;
            r += b;
        }
    }
    if (lane == 63) {
        ws[w] = s;
        wr[w] = r;
    }
    __syncthreads();
    if (w == 0) {
        int a = lane < 16 ? ws[lane] : 0, b = lane < 16 ? wr[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int x = __shfl_up(a, o, 64), y = __shfl_up(b, o, 64);
            if (lane >= o) {
                a += x;
                b += y;
            }
        }
        if (lane < 16) {
            ws[lane] = a;
            wr[lane] = b;
        }
    }
    __syncthreads();
    if (w > 0) {
        s += ws[w - 1];
        r += wr[w - 1];
    }
}

__device__ inline void scan_body(const int *in, int *out, int n, int mode, int p, int *total, int *raw_total,
                                 int *clear = nullptr) {
    __shared__ int tile[kScanTile];
    __shared__ int ws[16], wr[16];
    const int t = threadIdx.x;
    auto tr = [&](int v) { return mode == 0 ? v : (mode == 1 ? (v + p - 1) / p * p : (v + p - 1) / p); };
    int carry = 0, rcarry = 0;
    for (int base = 0; base < n; base += kScanTile) {
        int v[kScanPer];
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            const int i = base + u * 1024 + t;
            v[u] = i < n ? in[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            const int i = base + u * 1024 + t;
            tile[u * 1024 + t] = v[u];
            if (clear && i < n) clear[i] = 0;
        }
        __syncthreads();
        int s = 0, r = 0;
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            v[u] = tile[t * kScanPer + u];
            s += tr(v[u]);
            r += v[u];
        }
        const int s0 = s;
        block_scan2(s, r, ws, wr);
        int run = carry + s - s0;
        __syncthreads();   // every thread has read the wavefront totals
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            tile[t * kScanPer + u] = run;
            run += tr(v[u]);
        }
        if (t == 1023) {   // inclusive sums of the last thread: the tile's totals
            ws[0] = s;
            wr[0] = r;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            const int i = base + u * 1024 + t;
            if (i < n) out[i] = tile[u * 1024 + t];
        }
        carry += ws[0];
        rcarry += wr[0];
        __syncthreads();   // tile and ws reused by the next tile
    }
    if (t == 0) {
        out[n] = carry;
        if (total) *total = carry;
        if (raw_total) *raw_total = rcarry;
    }
}

}  // namespace mxn
