// edt_clearance.hip -- trajectory clearance cost on the distance field and its
// hand-written gradient (paper section III, Eq. 2, clearance term, in the
// squared-hinge form c(p) = max(0, margin - d(p))^2).
//
// d(p) is the trilinear interpolation of the metric field h*sqrt(s) at the
// point p (metres, voxel center i at i*h).  Per axis with n voxels and
// u = p / h: i0 = clamp(floor(u), 0, n-2), t = clamp(u - i0, 0, 1); an axis
// whose t was clamped has zero derivative.  The field stays exact integer
// arithmetic upstream; only this query is floating point.  The map from a
// waypoint to its cell (u, i0, t) is taken in fp64: it decides an integer
// (the cell, hence which one-sided gradient applies on a face), and in fp32
// u = p/h would carry an absolute error of ~|u| * 6e-8 into t.  The
// interpolation, the cost and its gradient are fp32, and each trajectory's
// cost is reduced in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include "edt.h"

namespace {

struct Tri {
    float v, gx, gy, gz;   // value and d/du (per voxel unit)
};

__device__ inline void axis_cell(float p, double h, int n, int& i0, float& t, float& live) {
    const double u = (double)p / h;
    double fl = floor(u);
    fl = fmin(fmax(fl, 0.0), (double)(n - 2));
    i0 = (int)fl;
    const double tr = u - fl;
    live = (tr >= 0.0 && tr <= 1.0) ? 1.0f : 0.0f;
    t = (float)fmin(fmax(tr, 0.0), 1.0);
}

__device__ inline float metric(const int32_t* __restrict__ s, int64_t idx, float h) {
    return h * sqrtf((float)__ldg(s + idx));
}

__device__ inline Tri trilinear(const int32_t* __restrict__ s, int nx, int ny, int nz, double hd,
                                float px, float py, float pz) {
    int ix, iy, iz;
    float tx, ty, tz, lx, ly, lz;
    axis_cell(px, hd, nx, ix, tx, lx);
    axis_cell(py, hd, ny, iy, ty, ly);
    axis_cell(pz, hd, nz, iz, tz, lz);
    const float h = (float)hd;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t b = ix + sy * iy + sz * iz;
    const float c000 = metric(s, b, h), c001 = metric(s, b + 1, h);
    const float c010 = metric(s, b + sy, h), c011 = metric(s, b + sy + 1, h);
    const float c100 = metric(s, b + sz, h), c101 = metric(s, b + sz + 1, h);
    const float c110 = metric(s, b + sz + sy, h), c111 = metric(s, b + sz + sy + 1, h);
    const float wx = 1.0f - tx, wy = 1.0f - ty, wz = 1.0f - tz;
    Tri r;
    r.v = wz * (wy * (wx * c000 + tx * c001) + ty * (wx * c010 + tx * c011)) +
          tz * (wy * (wx * c100 + tx * c101) + ty * (wx * c110 + tx * c111));
    r.gx = lx * (wz * (wy * (c001 - c000) + ty * (c011 - c010)) +
                 tz * (wy * (c101 - c100) + ty * (c111 - c110)));
    r.gy = ly * (wz * (wx * (c010 - c000) + tx * (c011 - c001)) +
                 tz * (wx * (c110 - c100) + tx * (c111 - c101)));
    r.gz = lz * (wy * (wx * (c100 - c000) + tx * (c101 - c001)) +
                 ty * (wx * (c110 - c010) + tx * (c111 - c011)));
    return r;
}

// One wave per trajectory: lane w accumulates waypoints w, w+64, ... in order,
// then a fixed butterfly reduction over the 64 lanes.
__global__ void __launch_bounds__(256) k_clear_fwd(const int32_t* __restrict__ s, int nx, int ny,
                                                   int nz, double h, float margin,
                                                   const float* __restrict__ wp, int64_t T, int W,
                                                   float* __restrict__ cost) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < T;
         t += nwaves) {
        float acc = 0.0f;
        for (int w = lane; w < W; w += 64) {
            const float* p = wp + (t * W + w) * 3;
            const Tri r = trilinear(s, nx, ny, nz, h, p[0], p[1], p[2]);
            const float hinge = fmaxf(0.0f, margin - r.v);
            acc += hinge * hinge;
        }
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) cost[t] = acc;
    }
}

__global__ void __launch_bounds__(256) k_clear_bwd(const int32_t* __restrict__ s, int nx, int ny,
                                                   int nz, double h, float margin,
                                                   const float* __restrict__ wp, int64_t T, int W,
                                                   const float* __restrict__ gcost,
                                                   float* __restrict__ gwp) {
    const int64_t n = T * W;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float* p = wp + i * 3;
        const Tri r = trilinear(s, nx, ny, nz, h, p[0], p[1], p[2]);
        const float hinge = fmaxf(0.0f, margin - r.v);
        const float k = gcost[i / W] * (-2.0f * hinge) * (float)(1.0 / h);
        gwp[i * 3 + 0] = k * r.gx;
        gwp[i * 3 + 1] = k * r.gy;
        gwp[i * 3 + 2] = k * r.gz;
    }
}

bool bad_field(const int32_t* s, int nx, int ny, int nz, double h) {
    return !s || nx < 2 || ny < 2 || nz < 2 || !(h > 0.0);
}

int grid_for(int64_t work, int per, int cap) {
    int64_t g = (work + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

extern "C" {

edt_status edt_clearance_fwd(const int32_t* d_s, int32_t nx, int32_t ny, int32_t nz, double h,
                             float margin, const float* d_wp, int64_t T, int32_t W, float* d_cost,
                             void* stream) {
    if (bad_field(d_s, nx, ny, nz, h) || T < 0 || W < 0) return EDT_ERR_ARG;
    if (T == 0) return EDT_OK;
    if (!d_wp || !d_cost) return EDT_ERR_ARG;
    hipLaunchKernelGGL(k_clear_fwd, dim3(grid_for(T, 4, 65535)), dim3(256), 0,
                       (hipStream_t)stream, d_s, nx, ny, nz, h, margin, d_wp, T, W, d_cost);
    return hipGetLastError() == hipSuccess ? EDT_OK : EDT_ERR_HIP;
}

edt_status edt_clearance_bwd(const int32_t* d_s, int32_t nx, int32_t ny, int32_t nz, double h,
                             float margin, const float* d_wp, int64_t T, int32_t W,
                             const float* d_gcost, float* d_gwp, void* stream) {
    if (bad_field(d_s, nx, ny, nz, h) || T < 0 || W < 0) return EDT_ERR_ARG;
    if (T == 0 || W == 0) return EDT_OK;
    if (!d_wp || !d_gcost || !d_gwp) return EDT_ERR_ARG;
    hipLaunchKernelGGL(k_clear_bwd, dim3(grid_for(T * W, 256, 65535)), dim3(256), 0,
                       (hipStream_t)stream, d_s, nx, ny, nz, h, margin, d_wp, T, W, d_gcost, d_gwp);
    return hipGetLastError() == hipSuccess ? EDT_OK : EDT_ERR_HIP;
}

}  // extern "C"
