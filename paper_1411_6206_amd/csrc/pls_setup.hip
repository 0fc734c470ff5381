// Set-up kernels: sample lists from the mask, layout permutations between the caller's
// [..][z][y][x] arrays and the internal [..][x][z][y] planes, and the permutation of the
// prior weights from canonical (Mallat) Haar order into the block-local in-place order
// that the sparse kernel produces.
#include "pls_common.hpp"
#include "pls_kernels.hpp"

namespace pls {

// One block per frame: exclusive scan of the mask over the (kz, ky) plane.
__global__ void __launch_bounds__(256) pls_mask_scan_kernel(const uint8_t* mask, int P,
                                                            int16_t* sidx, int* plist, int* ns) {
    __shared__ int part[256];
    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    const int chunk = (P + 255) / 256;
    const int b = tid * chunk;
    const int e = min(P, b + chunk);
    const uint8_t* m = mask + (size_t)t * P;
    int cnt = 0;
    for (int i = b; i < e; ++i) cnt += (m[i] != 0);
    part[tid] = cnt;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int i = 0; i < 256; ++i) {
            const int c = part[i];
            part[i] = run;
            run += c;
        }
        ns[t] = run;
    }
    __syncthreads();
    int s = part[tid];
    for (int i = b; i < e; ++i) {
        if (m[i] != 0) {
            sidx[(size_t)t * P + i] = (int16_t)s;
            plist[(size_t)t * P + s] = i;
            ++s;
        } else {
            sidx[(size_t)t * P + i] = -1;
        }
    }
}

void launch_mask_scan(const uint8_t* mask, int ny, int nz, int nt, int16_t* sidx, int* plist,
                      int* ns, hipStream_t s) {
    hipLaunchKernelGGL(pls_mask_scan_kernel, dim3(nt), dim3(256), 0, s, mask, ny * nz, sidx,
                       plist, ns);
}

// Tiled transpose of each (y, x) slice: in [F][nz][ny][nx] -> out [F][nx][nz][ny].
__global__ void __launch_bounds__(256) pls_pack_kernel(const float2* in, const float2* in2,
                                                       float2* out, int nx, int ny, int nz) {
    __shared__ float2 tile[32][33];
    const int fz = blockIdx.z;           // f * nz + z
    const int f = fz / nz, z = fz % nz;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const size_t src = (size_t)fz * ny * nx;
    for (int k = ty; k < 32; k += 8) {
        const int y = y0 + k, x = x0 + tx;
        if (y < ny && x < nx) {
            float2 v = in[src + (size_t)y * nx + x];
            if (in2) v = cadd(v, in2[src + (size_t)y * nx + x]);
            tile[k][tx] = v;
        }
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int x = x0 + k, y = y0 + tx;
        if (y < ny && x < nx) out[(((size_t)f * nx + x) * nz + z) * ny + y] = tile[tx][k];
    }
}

void launch_pack(const float2* in, const float2* in2, float2* out, int F, int nx, int ny, int nz,
                 hipStream_t s) {
    dim3 grid((nx + 31) / 32, (ny + 31) / 32, F * nz);
    hipLaunchKernelGGL(pls_pack_kernel, grid, dim3(256), 0, s, in, in2, out, nx, ny, nz);
}

// in internal [F][nx][nz][ny] (a + b) -> out user [F][nz][ny][nx]
__global__ void __launch_bounds__(256) pls_unpack_kernel(const float2* a, const float2* b,
                                                         float2* out, int nx, int ny, int nz) {
    __shared__ float2 tile[32][33];
    const int fz = blockIdx.z;
    const int f = fz / nz, z = fz % nz;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int x = x0 + k, y = y0 + tx;
        if (y < ny && x < nx) {
            const size_t gi = (((size_t)f * nx + x) * nz + z) * ny + y;
            float2 v = a[gi];
            if (b) v = cadd(v, b[gi]);
            tile[tx][k] = v;
        }
    }
    __syncthreads();
    const size_t dst = (size_t)fz * ny * nx;
    for (int k = ty; k < 32; k += 8) {
        const int y = y0 + k, x = x0 + tx;
        if (y < ny && x < nx) out[dst + (size_t)y * nx + x] = tile[k][tx];
    }
}

void launch_unpack(const float2* a, const float2* b, float2* out, int F, int nx, int ny, int nz,
                   hipStream_t s) {
    dim3 grid((nx + 31) / 32, (ny + 31) / 32, F * nz);
    hipLaunchKernelGGL(pls_unpack_kernel, grid, dim3(256), 0, s, a, b, out, nx, ny, nz);
}

// Number of trailing zeros of p, capped at cap (p = 0 -> cap).
__device__ __forceinline__ int tz_cap(int p, int cap) {
    int k = 0;
    while (k < cap && ((p >> k) & 1) == 0) ++k;
    return k;
}

// Canonical position along one axis of the in-place coefficient at position p, given the
// coefficient's level l (l = J: final approximation).
__device__ __forceinline__ int canon_axis(int p, int n, int l, int J) {
    if (l >= J) return p >> J;
    return ((p >> l) & 1) ? (n >> (l + 1)) + (p >> (l + 1)) : (p >> (l + 1));
}

// out[t][x][z][y] (in-place position) = in[t][zc][yc][xc] (canonical position)
__global__ void __launch_bounds__(256) pls_pack_w_kernel(const uint8_t* in, uint8_t* out, int nt,
                                                         int nx, int ny, int nz, int J) {
    const size_t n = (size_t)nt * nx * ny * nz;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(g % ny);
        size_t r = g / ny;
        const int z = (int)(r % nz);
        r /= nz;
        const int x = (int)(r % nx);
        const int t = (int)(r / nx);
        int l = J;
        if (nx > 1) l = min(l, tz_cap(x, J));
        if (ny > 1) l = min(l, tz_cap(y, J));
        if (nz > 1) l = min(l, tz_cap(z, J));
        const int xc = nx > 1 ? canon_axis(x, nx, l, J) : 0;
        const int yc = ny > 1 ? canon_axis(y, ny, l, J) : 0;
        const int zc = nz > 1 ? canon_axis(z, nz, l, J) : 0;
        out[g] = in[(((size_t)t * nz + zc) * ny + yc) * nx + xc];
    }
}

void launch_pack_weights(const uint8_t* in, uint8_t* out, int nt, int nx, int ny, int nz,
                         int levels, hipStream_t s) {
    const size_t n = (size_t)nt * nx * ny * nz;
    const size_t g0 = (n + 255) / 256;
    const int grid = (int)(g0 < 65536 ? g0 : 65536);
    hipLaunchKernelGGL(pls_pack_w_kernel, dim3(grid), dim3(256), 0, s, in, out, nt, nx, ny, nz,
                       levels);
}

__global__ void __launch_bounds__(256) pls_add_kernel(const float2* a, const float2* b,
                                                      float2* out, size_t n) {
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x)
        out[g] = b ? cadd(a[g], b[g]) : a[g];
}

void launch_add(const float2* a, const float2* b, float2* out, size_t n, hipStream_t s) {
    const size_t g0 = (n + 255) / 256;
    const int grid = (int)(g0 < 16384 ? g0 : 16384);
    hipLaunchKernelGGL(pls_add_kernel, dim3(grid), dim3(256), 0, s, a, b, out, n);
}

}  // namespace pls
