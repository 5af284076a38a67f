// Exclusive scan on one workgroup of 1024 threads (device code shared by the
// grid sort and the pair-list kernels).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace mxn {

// Exclusive scan on one workgroup of 1024 threads; mode 0: values as is,
// 1: rounded up to a multiple of p, 2: ceil(v/p).  raw_total (optional)
// receives the sum of the untransformed values; clear (optional, the input
// array itself) is zeroed once read.  Tiles of 8192 values: thread t reads
// and writes the eight consecutive values t*8 .. t*8+7 of the tile straight
// from and to memory (two 16-byte accesses when the arrays are 16-byte
// aligned, which makes each wavefront access one contiguous 2 KB run), the
// 1024 chunk sums are scanned across the workgroup (wavefront scans, then the
// 16 wavefront totals), and a running carry joins the tiles.
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
    __shared__ int ws[16], wr[16];
    const int t = threadIdx.x;
    auto tr = [&](int v) { return mode == 0 ? v : (mode == 1 ? (v + p - 1) / p * p : (v + p - 1) / p); };
    const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    int carry = 0, rcarry = 0;
    for (int base = 0; base < n; base += kScanTile) {
        const int i0 = base + t * kScanPer;
        const bool whole = vec && i0 + kScanPer <= n;
        int v[kScanPer];
        if (whole) {
            const int4 a = *reinterpret_cast<const int4 *>(in + i0);
            const int4 b = *reinterpret_cast<const int4 *>(in + i0 + 4);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
#pragma unroll
            for (int u = 0; u < kScanPer; ++u) v[u] = i0 + u < n ? in[i0 + u] : 0;
        }
        if (clear) {
            if (whole) {
                *reinterpret_cast<int4 *>(clear + i0) = make_int4(0, 0, 0, 0);
                *reinterpret_cast<int4 *>(clear + i0 + 4) = make_int4(0, 0, 0, 0);
            } else {
#pragma unroll
                for (int u = 0; u < kScanPer; ++u)
                    if (i0 + u < n) clear[i0 + u] = 0;
            }
        }
        int s = 0, r = 0;
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            s += tr(v[u]);
            r += v[u];
        }
        const int s0 = s;
        block_scan2(s, r, ws, wr);
        int run = carry + s - s0;
        int o[kScanPer];
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            o[u] = run;
            run += tr(v[u]);
        }
        if (whole) {
            *reinterpret_cast<int4 *>(out + i0) = make_int4(o[0], o[1], o[2], o[3]);
            *reinterpret_cast<int4 *>(out + i0 + 4) = make_int4(o[4], o[5], o[6], o[7]);
        } else {
#pragma unroll
            for (int u = 0; u < kScanPer; ++u)
                if (i0 + u < n) out[i0 + u] = o[u];
        }
        __syncthreads();   // every thread has read the wavefront totals
        if (t == 1023) {   // inclusive sums of the last thread: the tile's totals
            ws[0] = s;
            wr[0] = r;
        }
        __syncthreads();
        carry += ws[0];
        rcarry += wr[0];
        __syncthreads();   // ws reused by the next tile
    }
    if (t == 0) {
        out[n] = carry;
        if (total) *total = carry;
        if (raw_total) *raw_total = rcarry;
    }
}

}  // namespace mxn
