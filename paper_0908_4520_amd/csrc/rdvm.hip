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
// One workgroup of 512 threads owns one instance for the whole launch: the state sits in LDS
// (M N_w doubles, twice when two buffers fit: a step then reads one and writes the other, and
// needs a single barrier); P threads share a cell (P consecutive lanes of one wave), each
// advecting and relaxing the velocities k = p, p + P, ... and keeping them, and their
// Beam-Warming coefficients, in registers.  Every thread reads all of its K velocity slots
// unconditionally (kernels with K <= 8, coefficients in registers) -- slots beyond M read row 0
// with zero weight -- so the 3K LDS reads of a step are all in flight at once.  u and the stress are summed over the P lanes by xor butterflies
// (every lane of the group gets the same bits).  The force's time factor cos(phi t) is
// tabulated in LDS for 512 steps at a time, one entry per thread.  Nothing touches HBM inside
// the step loop.
#include "kernels_impl.h"
#include "rdvm.h"

namespace lbm {

static_assert(kRdvmTf == kRdvmBlock, "one tabulated time factor per thread");

// The value of lane i ^ m (m = 1 or 2) by a DPP quad permutation: no trip through the LDS.
template <int CTRL>
__device__ __forceinline__ double quad_xor(double v) {
    const int2v x = __builtin_bit_cast(int2v, v);
    return __builtin_bit_cast(double, int2v{__builtin_amdgcn_mov_dpp(x.x, CTRL, 0xf, 0xf, false),
                                            __builtin_amdgcn_mov_dpp(x.y, CTRL, 0xf, 0xf, false)});
}
constexpr int kQuadXor1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);   // lane i <- lane i ^ 1
constexpr int kQuadXor2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);   // lane i <- lane i ^ 2

// K velocities per thread at most; CREG: coefficients in registers (else read from LDS).
template <int K, bool CREG>
__global__ __launch_bounds__(kRdvmBlock) void k_rdvm(RdvmArgs a, const int32_t *index) {
    extern __shared__ double lds[];
    const RdvmInst in = a.inst[index[blockIdx.x]];
    const int M = in.M, nw = in.nw, P = in.P;
    const int t = threadIdx.x, j = t / P, p = t % P;
    const bool own = j < nw;
    const size_t MN = (size_t)M * nw;
    double *Gr = lds;                              // [M][nw], read by the coming step
    double *Gw = a.two ? lds + MN : lds;           // written by it
    double *cst = lds + (a.two ? 2 : 1) * MN;      // xi[M], w[M], alpha[M], beta[M]
    double *red = cst + 4 * (size_t)M;             // [2 * kRdvmBlock / 64] per-wave record sums
    double *tfa = red + 2 * (kRdvmBlock / 64);     // [kRdvmTf] force time factors
    double *gst = a.state + in.state_off;
    for (int i = t; i < M * nw; i += kRdvmBlock) Gr[i] = gst[i];
    for (int i = t; i < 4 * M; i += kRdvmBlock) cst[i] = a.nodes[in.node_off + i];
    const int jc = own ? j : 0;
    const double cj = own ? a.tabs[in.tab_off + j] : 0.0;
    const double sj = own ? a.tabs[in.tab_off + nw + j] : 0.0;
    const int jm1 = (jc + nw - 1) % nw, jm2 = (jc + 2 * nw - 2) % nw;
    const int jp1 = (jc + 1) % nw, jp2 = (jc + 2) % nw;
    const double om = in.omega, kf = 1.0 - 0.5 * om;
    __syncthreads();
    // with CREG the thread's coefficients, rows and upwind neighbours live in registers
    double cx[CREG ? K : 1], cw[CREG ? K : 1], ca[CREG ? K : 1], cb[CREG ? K : 1];
    int row[CREG ? K : 1], up1[CREG ? K : 1], up2[CREG ? K : 1];
    if constexpr (CREG) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int k = p + q * P;
            const bool v = k < M;
            const int kk = v ? k : 0;
            cx[q] = v ? cst[kk] : 0.0;
            cw[q] = v ? cst[M + kk] : 0.0;
            ca[q] = v ? cst[2 * M + kk] : 0.0;
            cb[q] = v ? cst[3 * M + kk] : 0.0;
            row[q] = kk * nw;
            up1[q] = cx[q] > 0.0 ? jm1 : jp1;       // upwind neighbours
            up2[q] = cx[q] > 0.0 ? jm2 : jp2;
        }
    }
    int32_t to_rec = a.record, nrec = 0;             // steps to the next record, records done
    for (int64_t st = 0; st < a.steps; ++st) {
        const int slot = (int)(st % kRdvmTf);
        if (slot == 0) {                             // time factors of steps st .. st + kRdvmTf - 1
            tfa[t] = cos(in.freq * (double)(a.step0 + st + 1 + t) * in.dt);
            __syncthreads();
        }
        const double tfs = tfa[slot];
        double g[K];
        double u = 0.0, sig = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            if constexpr (CREG) {                    // every slot, no branch: all reads in flight
                const int r = row[q];
                const double f0 = Gr[r + jc], f1 = Gr[r + up1[q]], f2 = Gr[r + up2[q]];
                const double v = f0 - ca[q] * (f0 - f1) + cb[q] * (f1 - f2);
                g[q] = v;
                u += cw[q] * v;
                sig += cw[q] * cx[q] * v;
            } else {                                 // many slots: only the real ones (registers)
                const int k = p + q * P;
                if (k < M) {
                    const double xk = cst[k], wk = cst[M + k], al = cst[2 * M + k], be = cst[3 * M + k];
                    const int r = k * nw, i1 = xk > 0.0 ? jm1 : jp1, i2 = xk > 0.0 ? jm2 : jp2;
                    const double f0 = Gr[r + jc], f1 = Gr[r + i1], f2 = Gr[r + i2];
                    const double v = f0 - al * (f0 - f1) + be * (f1 - f2);
                    g[q] = v;
                    u += wk * v;
                    sig += wk * xk * v;
                }
            }
        }
        if (P >= 2) {                                // sum over the cell's P lanes (xor butterfly)
            u += quad_xor<kQuadXor1>(u);
            sig += quad_xor<kQuadXor1>(sig);
        }
        if (P >= 4) {
            u += quad_xor<kQuadXor2>(u);
            sig += quad_xor<kQuadXor2>(sig);
        }
        for (int off = 4; off < P; off <<= 1) {
            u += __shfl_xor(u, off, 64);
            sig += __shfl_xor(sig, off, 64);
        }
        if (!a.two) __syncthreads();                 // one buffer: every neighbour read before writing
        const double dF = in.dt * in.amp * tfs * cj;
        u += 0.5 * dF;
        if (own) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int k = p + q * P;
                if (k < M) Gw[(size_t)k * nw + j] = g[q] - om * (g[q] - u) + kf * dF;
            }
        }
        const bool rec = a.record > 0 && --to_rec == 0;
        __syncthreads();                             // every cell relaxed; every read of Gr and tfa done
        if (a.two) {
            double *tmp = Gr;
            Gr = Gw;
            Gw = tmp;
        }
        if (rec) {
            const bool lead = own && p == 0;
            double su = wave_sum(lead ? u * cj : 0.0), ss = wave_sum(lead ? kf * sig * sj : 0.0);
            if ((t & 63) == 0) {
                red[2 * (t >> 6)] = su;
                red[2 * (t >> 6) + 1] = ss;
            }
            __syncthreads();
            if (t == 0) {
                su = 0.0;
                ss = 0.0;
                for (int w = 0; w < kRdvmBlock / 64; ++w) {
                    su += red[2 * w];
                    ss += red[2 * w + 1];
                }
                a.log[in.log_off + nrec] = 2.0 * su / (double)nw;
                a.log[in.log_off + a.nrec + nrec] = 2.0 * ss / (double)nw;
            }
            __syncthreads();                         // red free again
            to_rec = a.record;
            ++nrec;
        }
    }
    for (int i = t; i < M * nw; i += kRdvmBlock) gst[i] = Gr[i];
}

hipError_t rdvm_allow_lds(size_t lds_bytes) {
    for (const void *f : {reinterpret_cast<const void *>(&k_rdvm<4, true>), reinterpret_cast<const void *>(&k_rdvm<5, true>),
                          reinterpret_cast<const void *>(&k_rdvm<6, true>), reinterpret_cast<const void *>(&k_rdvm<8, true>),
                          reinterpret_cast<const void *>(&k_rdvm<16, false>),
                          reinterpret_cast<const void *>(&k_rdvm<32, false>)}) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_rdvm(int K, const RdvmArgs &a, const int32_t *index, uint32_t count, size_t lds_bytes,
                       hipStream_t s) {
    if (K == 4)
        hipLaunchKernelGGL((k_rdvm<4, true>), dim3(count), dim3(kRdvmBlock), lds_bytes, s, a, index);
    else if (K == 5)
        hipLaunchKernelGGL((k_rdvm<5, true>), dim3(count), dim3(kRdvmBlock), lds_bytes, s, a, index);
    else if (K == 6)
        hipLaunchKernelGGL((k_rdvm<6, true>), dim3(count), dim3(kRdvmBlock), lds_bytes, s, a, index);
    else if (K == 8)
        hipLaunchKernelGGL((k_rdvm<8, true>), dim3(count), dim3(kRdvmBlock), lds_bytes, s, a, index);
    else if (K == 16)
        hipLaunchKernelGGL((k_rdvm<16, false>), dim3(count), dim3(kRdvmBlock), lds_bytes, s, a, index);
    else if (K == 32)
        hipLaunchKernelGGL((k_rdvm<32, false>), dim3(count), dim3(kRdvmBlock), lds_bytes, s, a, index);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lbm
