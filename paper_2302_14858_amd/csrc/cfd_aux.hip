// Auxiliary device kernels: face-ghost exchange for conforming periodic block
// tilings (the communication step that fills ghost nodes before each block's
// closure solve, Sec. 2.4) and element-wise stage combinations for explicit
// Runge-Kutta time stepping (Sec. 3).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cfd_internal.h"

namespace cfd {

// Ghost element e of the 6 faces of every block-field, for a lattice of
// identical blocks (n interior, ng ghosts) at in_off[b] with nfields fields.
// Face order: x-, x+, y-, y+, z-, z+; a face holds ng layers of the interior
// extent of the other two directions.
template <typename T>
__global__ void k_halo(T *__restrict__ data, const int64_t *__restrict__ off, int nx, int ny, int nz, int ng,
                       int nfields, int bx, int by, int bz, int64_t total) {
    const int64_t PX = nx + 2 * ng, PY = ny + 2 * ng, PZ = nz + 2 * ng;
    const int64_t fstride = PX * PY * PZ;
    const int64_t fx = (int64_t)ng * ny * nz, fy = (int64_t)ng * nx * nz, fz = (int64_t)ng * nx * ny;
    const int64_t per_field = 2 * (fx + fy + fz);
    const int64_t per_block = per_field * nfields;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / per_block;
        int64_t r = e - b * per_block;
        const int64_t f = r / per_field;
        r -= f * per_field;
        const int kx = (int)(b % bx), ky = (int)((b / bx) % by), kz = (int)(b / ((int64_t)bx * by));
        int x, y, z, nb;
        if (r < 2 * fx) {
            const int side = r >= fx;
            int64_t q = side ? r - fx : r;
            const int layer = (int)(q % ng);
            q /= ng;
            y = (int)(q % ny);
            z = (int)(q / ny);
            // ghost x and the source x in the neighbour
            x = side ? nx + layer : -ng + layer;
            const int nkx = (kx + (side ? 1 : bx - 1)) % bx;
            nb = (kz * by + ky) * bx + nkx;
            const int sx = side ? layer : nx - ng + layer;
            const int64_t dst = off[b] + f * fstride + ((int64_t)(z + ng) * PY + (y + ng)) * PX + (x + ng);
            const int64_t src = off[nb] + f * fstride + ((int64_t)(z + ng) * PY + (y + ng)) * PX + (sx + ng);
            data[dst] = data[src];
            continue;
        }
        r -= 2 * fx;
        if (r < 2 * fy) {
            const int side = r >= fy;
            int64_t q = side ? r - fy : r;
            x = (int)(q % nx);
            q /= nx;
            const int layer = (int)(q % ng);
            z = (int)(q / ng);
            y = side ? ny + layer : -ng + layer;
            const int nky = (ky + (side ? 1 : by - 1)) % by;
            nb = (kz * by + nky) * bx + kx;
            const int sy = side ? layer : ny - ng + layer;
            const int64_t dst = off[b] + f * fstride + ((int64_t)(z + ng) * PY + (y + ng)) * PX + (x + ng);
            const int64_t src = off[nb] + f * fstride + ((int64_t)(z + ng) * PY + (sy + ng)) * PX + (x + ng);
            data[dst] = data[src];
            continue;
        }
        r -= 2 * fy;
        {
            const int side = r >= fz;
            int64_t q = side ? r - fz : r;
            x = (int)(q % nx);
            q /= nx;
            y = (int)(q % ny);
            const int layer = (int)(q / ny);
            z = side ? nz + layer : -ng + layer;
            const int nkz = (kz + (side ? 1 : bz - 1)) % bz;
            nb = (nkz * by + ky) * bx + kx;
            const int sz = side ? layer : nz - ng + layer;
            const int64_t dst = off[b] + f * fstride + ((int64_t)(z + ng) * PY + (y + ng)) * PX + (x + ng);
            const int64_t src = off[nb] + f * fstride + ((int64_t)(sz + ng) * PY + (y + ng)) * PX + (x + ng);
            data[dst] = data[src];
        }
    }
}

template <typename T>
__global__ void k_axpby(int64_t n, T a, const T *__restrict__ x, T b, T *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

template <typename T>
__global__ void k_xpcy(int64_t n, const T *__restrict__ x, T c, const T *__restrict__ y, T *__restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = x[i] + c * y[i];
}

static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_halo(int f32, void *data, const int64_t *off_dev, int nx, int ny, int nz, int ng, int nfields,
                       int bx, int by, int bz, hipStream_t st) {
    const int64_t per_field = 2 * ((int64_t)ng * ny * nz + (int64_t)ng * nx * nz + (int64_t)ng * nx * ny);
    const int64_t total = per_field * nfields * (int64_t)bx * by * bz;
    if (total == 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_halo<float>, dim3(grid_for(total)), dim3(256), 0, st, (float *)data, off_dev, nx, ny, nz,
                           ng, nfields, bx, by, bz, total);
    else
        hipLaunchKernelGGL(k_halo<double>, dim3(grid_for(total)), dim3(256), 0, st, (double *)data, off_dev, nx, ny,
                           nz, ng, nfields, bx, by, bz, total);
    return hipGetLastError();
}

hipError_t launch_axpby(int f32, int64_t n, double a, const void *x, double b, void *y, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_axpby<float>, dim3(grid_for(n)), dim3(256), 0, st, n, (float)a, (const float *)x,
                           (float)b, (float *)y);
    else
        hipLaunchKernelGGL(k_axpby<double>, dim3(grid_for(n)), dim3(256), 0, st, n, a, (const double *)x, b,
                           (double *)y);
    return hipGetLastError();
}

hipError_t launch_xpcy(int f32, int64_t n, const void *x, double c, const void *y, void *z, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_xpcy<float>, dim3(grid_for(n)), dim3(256), 0, st, n, (const float *)x, (float)c,
                           (const float *)y, (float *)z);
    else
        hipLaunchKernelGGL(k_xpcy<double>, dim3(grid_for(n)), dim3(256), 0, st, n, (const double *)x, c,
                           (const double *)y, (double *)z);
    return hipGetLastError();
}

}  // namespace cfd
