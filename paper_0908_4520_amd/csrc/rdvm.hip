// rdvm.hip -- the reduced discrete-velocity model, many instances in one persistent launch.
//
// Section 4 reduces the linearised BGK equation of the shear wave to Eqs. ga and gb in
// (t, y, xi_y).  Started from rest, G_a stays zero (Eq. ga has no source), so the state is G_b
// on M Gauss-Hermite velocities xi_k times N_w cells, advanced as the lattice Boltzmann
// step of this library advances an off-lattice set: Beam-Warming advection per velocity, then
// the second-order relaxation and source of Eq. 2order on the shifted variable
//   G~ = G + dt/(2 Kn)(G - u) - dt F / 2:
//   u  = sum_k w_k G~_k + dt F / 2            (u = sum_k w_k G_k, the Gauss-Hermite u_x)
//   G~*_k = G~_k - omega (G~_k - u) + (1 - omega/2) dt F,   F = A cos(phi t) cos(2 pi j / N_w).
// The recorded stress is sum_k w_k xi_k G_k = (1 - omega/2) sum_k w_k xi_k G~_k (pre-collision).
//
// One workgroup owns one instance for the whole launch: the state sits in LDS (M N_w doubles),
// each thread owns one cell and keeps its M advected values in registers between the two
// barriers of a step (read all neighbours, then write the relaxed values).  Nothing touches
// HBM inside the step loop.
#include "kernels_impl.h"
#include "rdvm.h"

namespace lbm {

// Sum over the block in a fixed order (wave butterflies, then the waves in index order); every
// thread gets the result.
__device__ __forceinline__ double rdvm_block_sum(double x, double *red) {
    const double s = wave_sum(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kRdvmBlock / 64; ++w) t += red[w];
    return t;
}

__global__ __launch_bounds__(kRdvmBlock) void k_rdvm(RdvmArgs a) {
    extern __shared__ double lds[];
    const RdvmInst in = a.inst[blockIdx.x];
    const int M = in.M, nw = in.nw, j = threadIdx.x;
    const bool own = j < nw;
    double *G = lds;                          // [M][nw]
    double *red = lds + (size_t)M * nw;       // [kRdvmBlock / 64]
    double *gst = a.state + in.state_off;
    for (int i = threadIdx.x; i < M * nw; i += kRdvmBlock) G[i] = gst[i];
    const double *xi = a.nodes + in.node_off, *w = xi + M, *al = w + M, *be = al + M;
    const double cj = own ? a.tabs[in.tab_off + j] : 0.0;
    const double sj = own ? a.tabs[in.tab_off + nw + j] : 0.0;
    const int jc = own ? j : 0;
    const int jm1 = (jc + nw - 1) % nw, jm2 = (jc + 2 * nw - 2) % nw;
    const int jp1 = (jc + 1) % nw, jp2 = (jc + 2) % nw;
    const double om = in.omega, kf = 1.0 - 0.5 * om;
    __syncthreads();
    for (int64_t st = 0; st < a.steps; ++st) {
        double g[kRdvmMaxNodes];
        double u = 0.0, sig = 0.0;
#pragma unroll
        for (int k = 0; k < kRdvmMaxNodes; ++k) {
            if (k < M) {
                const double *row = G + (size_t)k * nw;
                const bool up_left = xi[k] > 0.0;            // upwind cells j-1, j-2
                const double f0 = row[jc];
                const double f1 = row[up_left ? jm1 : jp1], f2 = row[up_left ? jm2 : jp2];
                const double v = f0 - al[k] * (f0 - f1) + be[k] * (f1 - f2);
                g[k] = v;
                u += w[k] * v;
                sig += w[k] * xi[k] * v;
            }
        }
        __syncthreads();                                     // every neighbour read
        const double t = (double)(a.step0 + st + 1) * in.dt;
        const double dF = in.dt * in.amp * cos(in.freq * t) * cj;
        u += 0.5 * dF;
        if (own) {
#pragma unroll
            for (int k = 0; k < kRdvmMaxNodes; ++k)
                if (k < M) G[(size_t)k * nw + j] = g[k] - om * (g[k] - u) + kf * dF;
        }
        __syncthreads();                                     // every cell relaxed
        if (a.record > 0 && (st + 1) % a.record == 0) {
            const double su = rdvm_block_sum(own ? u * cj : 0.0, red);
            const double ss = rdvm_block_sum(own ? kf * sig * sj : 0.0, red);
            if (threadIdx.x == 0) {
                const int64_t r = (st + 1) / a.record - 1;
                a.log[in.log_off + r] = 2.0 * su / (double)nw;
                a.log[in.log_off + a.nrec + r] = 2.0 * ss / (double)nw;
            }
        }
    }
    for (int i = threadIdx.x; i < M * nw; i += kRdvmBlock) gst[i] = G[i];
}

hipError_t rdvm_allow_lds(size_t lds_bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rdvm), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_bytes);
}

hipError_t launch_rdvm(const RdvmArgs &a, uint32_t count, size_t lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_rdvm, dim3(count), dim3(kRdvmBlock), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace lbm
