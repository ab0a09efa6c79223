// Auxiliary device kernels: face-ghost exchange for conforming block tilings
// (periodic lattices or a neighbour table; the communication step that fills
// ghost nodes before each block's closure solve, Sec. 2.4) and element-wise
// stage combinations for explicit Runge-Kutta time stepping (Sec. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "cfd_internal.h"

namespace cfd {

// Face ghosts of every block-field, for a lattice of identical blocks (n
// interior, ng ghosts) at off[b] with nfields fields.  blockIdx.y is the
// block-field (b nfields + f, wave-uniform); thread r of it takes ghost r of
// its 6 faces in the order x-, x+, y-, y+, z-, z+, each face holding ng
// layers of the interior extent of the other two directions.  Index
// arithmetic within a field is 32-bit.
template <typename T>
__global__ void k_halo(T *__restrict__ data, const int64_t *__restrict__ off, int nx, int ny, int nz, int ng,
                       int nfields, int bx, int by, int bz, int per_field) {
    const int r0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (r0 >= per_field) return;
    const int bf = blockIdx.y;
    const int b = bf / nfields, f = bf - b * nfields;
    const int kx = b % bx, ky = (b / bx) % by, kz = b / (bx * by);
    const int PX = nx + 2 * ng, PY = ny + 2 * ng, PZ = nz + 2 * ng;
    const int64_t fbase = (int64_t)f * PX * PY * PZ;
    const int fx = ng * ny * nz, fy = ng * nx * nz;
    int r = r0;
    int nb, dst, src;
    if (r < 2 * fx) {
        const int side = r >= fx;
        int q = side ? r - fx : r;
        const int layer = q % ng;
        q /= ng;
        const int y = q % ny, z = q / ny;
        const int x = side ? nx + layer : -ng + layer;          // ghost x
        const int sx = side ? layer : nx - ng + layer;          // source x in the neighbour
        nb = (kz * by + ky) * bx + (kx + (side ? 1 : bx - 1)) % bx;
        const int row = ((z + ng) * PY + (y + ng)) * PX;
        dst = row + x + ng;
        src = row + sx + ng;
    } else if ((r -= 2 * fx) < 2 * fy) {
        const int side = r >= fy;
        int q = side ? r - fy : r;
        const int x = q % nx;
        q /= nx;
        const int layer = q % ng, z = q / ng;
        const int y = side ? ny + layer : -ng + layer;
        const int sy = side ? layer : ny - ng + layer;
        nb = (kz * by + (ky + (side ? 1 : by - 1)) % by) * bx + kx;
        dst = ((z + ng) * PY + (y + ng)) * PX + x + ng;
        src = ((z + ng) * PY + (sy + ng)) * PX + x + ng;
    } else {
        r -= 2 * fy;
        const int fz = ng * nx * ny;
        const int side = r >= fz;
        int q = side ? r - fz : r;
        const int x = q % nx;
        q /= nx;
        const int y = q % ny, layer = q / ny;
        const int z = side ? nz + layer : -ng + layer;
        const int sz = side ? layer : nz - ng + layer;
        nb = (((kz + (side ? 1 : bz - 1)) % bz) * by + ky) * bx + kx;
        dst = ((z + ng) * PY + (y + ng)) * PX + x + ng;
        src = ((sz + ng) * PY + (y + ng)) * PX + x + ng;
    }
    data[off[b] + fbase + dst] = data[off[nb] + fbase + src];
}

// Face ghosts by a neighbour table: pair = (block b, face, neighbour nb) with
// face = 2 d + side (d: 0 x, 1 y, 2 z; side 1: the + face).  blockIdx.y is
// (pair, field), wave-uniform; thread r takes ghost r of the face's ng layers
// (x fastest where x runs along the face, so a wave's stores are contiguous).
// b's ghost layer l on the + face is nb's interior layer l + shift, on the -
// face nb's interior layer n_nb - ng + l - shift (shift 1: vertex-centred
// blocks, whose extremal nodes are shared, so the ghosts continue past the
// shared node); the coordinates along the face are the same in both blocks
// (conforming faces).  shapes: (nx, ny, nz, ng) per block.
template <typename T>
__global__ void k_halo_table(T *__restrict__ data, const int64_t *__restrict__ off, const int *__restrict__ shapes,
                             const int *__restrict__ pairs, int nfields, int shift) {
    const int pf = blockIdx.y;
    const int pr = pf / nfields, f = pf - pr * nfields;
    const int b = pairs[3 * pr], face = pairs[3 * pr + 1], nb = pairs[3 * pr + 2];
    const int d = face >> 1, side = face & 1;
    const int n[3] = {shapes[4 * b], shapes[4 * b + 1], shapes[4 * b + 2]};
    const int ng = shapes[4 * b + 3];
    const int m[3] = {shapes[4 * nb], shapes[4 * nb + 1], shapes[4 * nb + 2]};
    const int ta = d == 0 ? n[1] : n[0];   // extents along the face, first one fastest
    const int tb = d == 2 ? n[1] : n[2];
    const int count = ng * ta * tb;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    int c[3], layer;
    if (d == 0) {   // x faces: layer fastest (rows of ng contiguous nodes), then y, z
        layer = r % ng;
        const int q = r / ng;
        c[1] = q % ta;
        c[2] = q / ta;
    } else {        // y and z faces: x fastest, then the other face direction, then the layer
        c[0] = r % ta;
        const int q = r / ta;
        const int o = q % tb;
        layer = q / tb;
        if (d == 1) c[2] = o; else c[1] = o;
    }
    int g[3] = {c[0], c[1], c[2]}, s[3] = {c[0], c[1], c[2]};
    g[d] = side ? n[d] + layer : layer - ng;
    s[d] = side ? layer + shift : m[d] - ng + layer - shift;
    const int64_t PXb = n[0] + 2 * ng, PYb = n[1] + 2 * ng, PZb = n[2] + 2 * ng;
    const int64_t PXn = m[0] + 2 * ng, PYn = m[1] + 2 * ng, PZn = m[2] + 2 * ng;
    const int64_t dst = off[b] + (int64_t)f * PXb * PYb * PZb + ((g[2] + ng) * PYb + (g[1] + ng)) * PXb + g[0] + ng;
    const int64_t src = off[nb] + (int64_t)f * PXn * PYn * PZn + ((s[2] + ng) * PYn + (s[1] + ng)) * PXn + s[0] + ng;
    data[dst] = data[src];
}

// Shared nodes of vertex-centred blocks along direction d: pair = (b, nb),
// nb across b's + face; b's last node and nb's first node along d are one
// point and both get the mean of the two values.  blockIdx.y is (pair, slot):
// slot = field of the input layout (ghosted = 1: ng ghost layers) or
// operator-field of the output layout (ghosted = 0, slots of npts elements).
// Within one direction every shared node belongs to one pair, so the pairs
// do not race; the host runs x, y, z in turn.
template <typename T>
__global__ void k_shared_avg(T *__restrict__ data, const int64_t *__restrict__ off, const int *__restrict__ shapes,
                             const int *__restrict__ pairs, int nslots, int ghosted, int d) {
    const int pf = blockIdx.y;
    const int pr = pf / nslots, sl = pf - pr * nslots;
    const int b = pairs[2 * pr], nb = pairs[2 * pr + 1];
    const int n[3] = {shapes[4 * b], shapes[4 * b + 1], shapes[4 * b + 2]};
    const int m[3] = {shapes[4 * nb], shapes[4 * nb + 1], shapes[4 * nb + 2]};
    const int g = ghosted ? shapes[4 * b + 3] : 0;
    const int ta = d == 0 ? n[1] : n[0];
    const int tb = d == 2 ? n[1] : n[2];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ta * tb) return;
    int c[3];
    c[d == 0 ? 1 : 0] = r % ta;
    c[d == 2 ? 1 : 2] = r / ta;
    int ca[3] = {c[0], c[1], c[2]}, cb[3] = {c[0], c[1], c[2]};
    ca[d] = n[d] - 1;
    cb[d] = 0;
    const int64_t PXa = n[0] + 2 * g, PYa = n[1] + 2 * g, PZa = n[2] + 2 * g;
    const int64_t PXb = m[0] + 2 * g, PYb = m[1] + 2 * g, PZb = m[2] + 2 * g;
    const int64_t ia = off[b] + (int64_t)sl * PXa * PYa * PZa + ((ca[2] + g) * PYa + (ca[1] + g)) * PXa + ca[0] + g;
    const int64_t ib = off[nb] + (int64_t)sl * PXb * PYb * PZb + ((cb[2] + g) * PYb + (cb[1] + g)) * PXb + cb[0] + g;
    const T v = (data[ia] + data[ib]) * T(0.5);
    data[ia] = v;
    data[ib] = v;
}

template <typename T>
__global__ void k_axpby(int64_t n, T a, const T *__restrict__ x, T b, T *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = b == T(0) ? a * x[i] : a * x[i] + b * y[i];   // b = 0: y is not read
}

template <typename T>
__global__ void k_xpcy(int64_t n, const T *__restrict__ x, T c, const T *__restrict__ y, T *__restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = x[i] + c * y[i];
}

// Method-of-lines stage for the first-order wave system
//   d_t phi = Pi,  d_t Pi = sum_i d_i psi_i,  d_t psi_i = d_i Pi
// on one block: k is assembled from the stage state src (its Pi) and the
// derivative outputs d = [D_x Pi, D_y Pi, D_z Pi, D_x psi_x, D_y psi_y,
// D_z psi_z] computed from src (interior, [op][z][y][x]); on interior nodes
// stage = u0 + a k (if stage is given; stage may alias src, each node is read
// before it is written by the same thread) and acc = acc_in + b k.  State
// arrays hold the five fields with ghosts, [f][z][y][x].
// One wave per 64 consecutive interior nodes of a block in x-fastest order
// (all blocks' pieces numbered consecutively, unitpre[b] = first piece of
// block b; a piece may span rows, so rows shorter than 64 nodes still fill
// the wave): the piece's block is found once, wave-uniform, and each lane
// takes one node.
// With a lattice (bx > 0: the blocks tile a periodic box as in
// cfd_halo_exchange) the state the next derivative reads (stage if given,
// else acc) also has its face ghosts refreshed: a node within ng of a face
// writes its new value into the facing ghost layer of the neighbour across
// that face.  Interior nodes are only read and ghost nodes only written here,
// so stage may still alias src.
template <typename T>
__global__ void __launch_bounds__(256)
k_wave_stage(const T *u0, const T *src, T *stage, const T *acc_in, T *acc, const T *__restrict__ d,
             const int64_t *__restrict__ in_off, const int64_t *__restrict__ out_off,
             const int *__restrict__ shapes, const int *__restrict__ unitpre, int nblocks, int nunits, T a, T b,
             int bx, int by, int bz) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool acc_is_u0 = acc_in == u0;
    T *next = stage ? stage : acc;
    for (int u = blockIdx.x * 4 + wv; u < nunits; u += gridDim.x * 4) {
        int lo = 0, hi = nblocks - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (unitpre[mid] <= u) lo = mid; else hi = mid - 1;
        }
        const int bi = lo;
        const int nx = shapes[4 * bi], ny = shapes[4 * bi + 1], nz = shapes[4 * bi + 2], ng = shapes[4 * bi + 3];
        const int64_t n3 = (int64_t)nx * ny * nz;
        const int64_t e = ((int64_t)(u - unitpre[bi]) << 6) + lane;   // interior node, x fastest
        if (e >= n3) continue;
        const int64_t rr = e / nx;   // row z ny + y
        const int x = (int)(e - rr * nx);
        const int z = (int)(rr / ny), y = (int)(rr - (int64_t)z * ny);
        const int64_t PX = nx + 2 * ng, PY = ny + 2 * ng, PZ = nz + 2 * ng;
        const int64_t fs = PX * PY * PZ;
        const int64_t ip = in_off[bi] + ((int64_t)(z + ng) * PY + (y + ng)) * PX + ng + x;
        const T *db = d + out_off[bi] + e;
        const T k[5] = {src[ip + fs], db[3 * n3] + db[4 * n3] + db[5 * n3], db[0], db[n3], db[2 * n3]};
        T nv[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            T v = T(0);
            if (stage || acc_is_u0) v = u0[ip + f * fs];
            const T ai = acc_is_u0 ? v : acc_in[ip + f * fs];
            const T sv = v + a * k[f], av = ai + b * k[f];
            if (stage) stage[ip + f * fs] = sv;
            acc[ip + f * fs] = av;
            nv[f] = stage ? sv : av;
        }
        if (bx > 0) {
            // ghost copies of this node in the neighbours across the faces it is near
            const int kx = bi % bx, ky = (bi / bx) % by, kz = bi / (bx * by);
            const int64_t here = ((int64_t)(z + ng) * PY + (y + ng)) * PX + ng + x;   // offset within a field
            auto put = [&](int nb, int64_t shift) {
                T *dst = next + in_off[nb] + here + shift;
#pragma unroll
                for (int f = 0; f < 5; ++f) dst[f * fs] = nv[f];
            };
            if (x < ng) put((kz * by + ky) * bx + (kx + bx - 1) % bx, nx);
            if (x >= nx - ng) put((kz * by + ky) * bx + (kx + 1) % bx, -(int64_t)nx);
            if (y < ng) put((kz * by + (ky + by - 1) % by) * bx + kx, (int64_t)ny * PX);
            if (y >= ny - ng) put((kz * by + (ky + 1) % by) * bx + kx, -(int64_t)ny * PX);
            if (z < ng) put((((kz + bz - 1) % bz) * by + ky) * bx + kx, (int64_t)nz * PX * PY);
            if (z >= nz - ng) put((((kz + 1) % bz) * by + ky) * bx + kx, -(int64_t)nz * PX * PY);
        }
    }
}

static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_halo(int f32, void *data, const int64_t *off_dev, int nx, int ny, int nz, int ng, int nfields,
                       int bx, int by, int bz, hipStream_t st) {
    const int64_t per_field = 2 * ((int64_t)ng * ny * nz + (int64_t)ng * nx * nz + (int64_t)ng * nx * ny);
    const int64_t nbf = (int64_t)nfields * bx * by * bz;
    if (per_field == 0 || nbf == 0) return hipSuccess;
    const dim3 grid((unsigned)((per_field + 255) / 256), (unsigned)nbf);
    if (f32)
        hipLaunchKernelGGL(k_halo<float>, grid, dim3(256), 0, st, (float *)data, off_dev, nx, ny, nz, ng, nfields, bx,
                           by, bz, (int)per_field);
    else
        hipLaunchKernelGGL(k_halo<double>, grid, dim3(256), 0, st, (double *)data, off_dev, nx, ny, nz, ng, nfields, bx,
                           by, bz, (int)per_field);
    return hipGetLastError();
}

hipError_t launch_halo_table(int f32, void *data, const int64_t *off_dev, const int *shapes_dev, const int *pairs_dev,
                             int npairs, int nfields, int max_face, int shift, hipStream_t st) {
    if (npairs == 0 || max_face == 0) return hipSuccess;
    const dim3 grid((unsigned)((max_face + 255) / 256), (unsigned)(npairs * nfields));
    if (f32)
        hipLaunchKernelGGL(k_halo_table<float>, grid, dim3(256), 0, st, (float *)data, off_dev, shapes_dev, pairs_dev,
                           nfields, shift);
    else
        hipLaunchKernelGGL(k_halo_table<double>, grid, dim3(256), 0, st, (double *)data, off_dev, shapes_dev,
                           pairs_dev, nfields, shift);
    return hipGetLastError();
}

hipError_t launch_shared_avg(int f32, void *data, const int64_t *off_dev, const int *shapes_dev, const int *pairs_dev,
                             int npairs, int nslots, int ghosted, int d, int max_face, hipStream_t st) {
    if (npairs == 0 || max_face == 0 || nslots == 0) return hipSuccess;
    const dim3 grid((unsigned)((max_face + 255) / 256), (unsigned)(npairs * nslots));
    if (f32)
        hipLaunchKernelGGL(k_shared_avg<float>, grid, dim3(256), 0, st, (float *)data, off_dev, shapes_dev, pairs_dev,
                           nslots, ghosted, d);
    else
        hipLaunchKernelGGL(k_shared_avg<double>, grid, dim3(256), 0, st, (double *)data, off_dev, shapes_dev,
                           pairs_dev, nslots, ghosted, d);
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

namespace cfd {
hipError_t launch_wave_stage(int f32, const void *u0, const void *src, void *stage, const void *acc_in, void *acc,
                             const void *d, const int64_t *in_off, const int64_t *out_off, const int *shapes,
                             const int *unitpre, int nblocks, int nunits, double a, double b, int bx, int by, int bz,
                             hipStream_t st) {
    if (nunits == 0) return hipSuccess;
    int g = (nunits + 3) / 4;
    if (g > 65535) g = 65535;
    if (f32)
        hipLaunchKernelGGL(k_wave_stage<float>, dim3(g), dim3(256), 0, st, (const float *)u0, (const float *)src,
                           (float *)stage, (const float *)acc_in, (float *)acc, (const float *)d, in_off, out_off,
                           shapes, unitpre, nblocks, nunits, (float)a, (float)b, bx, by, bz);
    else
        hipLaunchKernelGGL(k_wave_stage<double>, dim3(g), dim3(256), 0, st, (const double *)u0, (const double *)src,
                           (double *)stage, (const double *)acc_in, (double *)acc, (const double *)d, in_off, out_off,
                           shapes, unitpre, nblocks, nunits, a, b, bx, by, bz);
    return hipGetLastError();
}

}  // namespace cfd
