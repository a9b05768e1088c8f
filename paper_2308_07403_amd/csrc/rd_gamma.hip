// rd_gamma.hip -- gain bounds and a per-entry certificate of D.
//
// Spectral radius (the critical gain gamma_c = 1 / rho(A), Eq. critical-gain):
// for B = A + I (rho(B) = rho(A) + 1, Perron-Frobenius for A >= 0) and any
// positive vector x, the Collatz-Wielandt ratios bracket rho(B):
//   min_i (Bx)_i / x_i <= rho(B) <= max_i (Bx)_i / x_i.
// The power iteration x <- Bx / max(Bx) (kept above 2^-900, which keeps x
// positive and the bounds valid) tightens them; the best bounds of all steps
// are kept.  B x >= x, so every ratio is at least 1.
//
// Certificate of one entry (Sec. 3.1: Eq. Y-series-trunc and the walk-count
// bound Eq. Nijk-limit): with k = D_ij from the readout, the true distance
// is at least k (Y >= gamma^dist), and a true distance of k + 1 or more
// would give Y <= gamma^(k+1) Delta^k / (1 - gamma Delta) (Eq. Y-bracket).
// So Y above that bound proves D_ij exact; Y = 0 proves "unreachable" when
// gamma^(n-1) (the smallest value of a reachable entry) is well above DBL_MIN.
// With integer weights the bound sums over walk lengths (weighted_bound_ln).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "rd_device.h"
#include "rd_launch.h"

namespace rd {

namespace {

constexpr double kXFloor = 0x1p-900;

// Slots of the power iteration's scratch (doubles as bit patterns where
// atomics need them): per step, in a rotation of three, {min ratio, max
// ratio, max of Bx}; then the best bounds over all steps.
struct PowerScratch {
    unsigned long long slot[3][4];     // [0] min ratio, [1] max ratio, [2] max Bx (bits of positive doubles)
    unsigned long long best_lo, best_hi;
};

__device__ __forceinline__ unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

__global__ void k_gamma_init(PowerScratch *sc) {
    for (int s = 0; s < 3; ++s) {
        sc->slot[s][0] = dbits(__builtin_huge_val());
        sc->slot[s][1] = 0;
        sc->slot[s][2] = 0;
    }
    sc->best_lo = dbits(1.0);
    sc->best_hi = dbits(__builtin_huge_val());
}

// One step: y = (A + I) x with x = xin * scale (scale = 1 / max of the last
// y, from the previous step's slot), x kept >= kXFloor; ratios y_i / x_i
// into this step's slot; y stored for the next step.  One wavefront per row
// (grid-stride over rows), 8 bytes of A per lane; the workgroup reduces its
// rows' extremes before one atomic per value.  Workgroup 0 folds the
// previous step's completed bounds into the best ones and clears the slot
// of the next step.
__global__ __launch_bounds__(256) void k_power_step(const uint8_t *__restrict__ A, int n, const double *__restrict__ xin,
                                                    double *__restrict__ yout, PowerScratch *sc, int step) {
    __shared__ double red[3][4];
    const int cur = step % 3, prev = (step + 2) % 3, next = (step + 1) % 3;
    const double scale = step == 0 ? 1.0 : 1.0 / bitsd(sc->slot[prev][2]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (step > 0) {
            atomicMax(&sc->best_lo, sc->slot[prev][0]);
            atomicMin(&sc->best_hi, sc->slot[prev][1]);
        }
        sc->slot[next][0] = dbits(__builtin_huge_val());
        sc->slot[next][1] = 0;
        sc->slot[next][2] = 0;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    auto xv = [&](int j) { return step == 0 ? 1.0 : fmax(xin[j] * scale, kXFloor); };
    double rmin = __builtin_huge_val(), rmax = 0.0, ymax = 0.0;
    const bool aligned = (n % 8) == 0;
    for (int i = blockIdx.x * 4 + wv; i < n; i += gridDim.x * 4) {
        const uint8_t *__restrict__ row = A + (size_t)i * n;
        double acc = 0.0;
        if (aligned) {
            for (int w = lane; w < n / 8; w += 64) {
                unsigned long long bits = *reinterpret_cast<const unsigned long long *>(row + (size_t)w * 8);
                while (bits) {
                    const int b = __builtin_ctzll(bits) >> 3;
                    acc += xv(w * 8 + b);
                    bits &= ~(0xFFull << (8 * b));
                }
            }
        } else {
            for (int j = lane; j < n; j += 64)
                if (row[j]) acc += xv(j);
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
        const double xi = xv(i);
        const double y = acc + xi;
        if (lane == 0) yout[i] = y;
        rmin = fmin(rmin, y / xi);
        rmax = fmax(rmax, y / xi);
        ymax = fmax(ymax, y);
    }
    if (lane == 0) {
        red[0][wv] = rmin;
        red[1][wv] = rmax;
        red[2][wv] = ymax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = red[0][0], a1 = red[1][0], a2 = red[2][0];
        for (int w = 1; w < 4; ++w) {
            a0 = fmin(a0, red[0][w]);
            a1 = fmax(a1, red[1][w]);
            a2 = fmax(a2, red[2][w]);
        }
        if (a1 > 0.0) {   // the workgroup had rows
            atomicMin(&sc->slot[cur][0], dbits(a0));
            atomicMax(&sc->slot[cur][1], dbits(a1));
            atomicMax(&sc->slot[cur][2], dbits(a2));
        }
    }
}

// Folds the last step's bounds into the best ones.
__global__ void k_power_fold(PowerScratch *sc, int last_step) {
    const int s = last_step % 3;
    atomicMax(&sc->best_lo, sc->slot[s][0]);
    atomicMin(&sc->best_hi, sc->slot[s][1]);
}

// ln of the weighted bound for readout k (positive integer weights, Sec. 3.2):
// a true distance of k + 1 or more makes every walk of l edges weigh at least
// max(l, k + 1), so Y <= gamma^(k+1) (Delta^(k+1) - 1) / (Delta - 1)
// + (gamma Delta)^(k+2) / (Delta (1 - gamma Delta)); Delta = 1:
// (k + 1) gamma^(k+1) + gamma^(k+2) / (1 - gamma).
__device__ __forceinline__ double weighted_bound_ln(double k, double lg, double ld, double delta, double gamma) {
    double first, second;
    if (delta == 1.0) {
        first = log(k + 1.0) + (k + 1.0) * lg;
        second = (k + 2.0) * lg - log1p(-gamma);
    } else {
        first = (k + 1.0) * (lg + ld) + log1p(-exp(-(k + 1.0) * ld)) - log(delta - 1.0);
        second = (k + 2.0) * (lg + ld) - ld - log1p(-gamma * delta);
    }
    const double m = fmax(first, second);
    return m + log1p(exp(fmin(first, second) - m));
}

constexpr int kCertChunk = 2048;   // columns per step of the certificate pass (8 per thread)

// Per-entry certificate over a kept graph's Y: mask (nullable, n x n bytes,
// 1 = certified) and the certified count into *count.  Entries below
// DBL_MIN, and zeros where gamma^(n-1) could underflow, are not certified
// (their rounding has no relative bound).  Y's relative error is taken as
// rel, the larger of 2^-30, the inversion's error bound 8 n u / (1 - gamma
// Delta) and err_floor (the cap on the error bounds of a Y changed by edge
// updates, else 0), on both sides of the argument: with k the readout of
// Y, the true distance is at least k only if the true Y is below
// gamma^(k - 1 + eta), so Y (1 + rel) must be; and a distance of k + 1 or
// more is excluded only if Y (1 - rel) is above the bound of Eq. Y-bracket.
// First pass over a row: ln Y from the exponent bits and the FP32 logarithm
// of the mantissa (within 1e-6 of ln Y, as in the readout's short path)
// gives k and the decision for almost every entry; entries whose readout or
// decision lies within that error of a boundary are queued in LDS and
// finished after each chunk of 2048 columns with the FP64 logarithm, so few
// wavefronts diverge into it.  At most 1024 workgroups stride over rows
// (one count atomic each); each thread loads its 8 columns of a chunk before
// working on them.
template <bool W>
__global__ __launch_bounds__(256) void k_certify(const double *__restrict__ Y, int ld, int n,
                                                 const rdist_info *__restrict__ ginfo, double err_floor,
                                                 uint8_t *__restrict__ mask, unsigned long long *__restrict__ count) {
    __shared__ int queue[kCertChunk];
    __shared__ int qn;
    const double gamma = ginfo->gamma;
    const double delta = (double)max(ginfo->delta, 1);
    const double lgd = log(gamma * delta);
    const double gd = gamma * (double)ginfo->delta;
    const double rel = fmin(0.5, fmax(fmax(0x1p-30, err_floor), 8.0 * (double)n * 0x1p-53 / fmax(1.0 - gd, 1e-300)));
    const double margin = log1p(rel) - log1p(-rel);
    const double up = log1p(rel);                  // ln of Y's largest true value over the computed one
    const double l0 = -log(delta * (1.0 - gamma * delta)) + margin;
    const double lg = log(gamma), lde = log(delta);
    // ln of the bound for readout k, the margins included
    auto bound_ln = [&](double k) {
        return W ? weighted_bound_ln(k, lg, lde, delta, gamma) + margin : (k + 1.0) * lgd + l0;
    };
    const double il = rd_inv_log(gamma);
    const double s2 = kLn2 * il;                   // log2 units to R units (< 0)
    const double band = 1e-4 - 4e-6 * s2;          // the readout's short-path band
    // Y = 0 proves "no walk" only when no reachable entry can underflow:
    // every reachable entry is at least gamma^(n-1)
    const bool zero_ok = (double)(n - 1) * log(gamma) > log(kDblMin) + 1.0;
    unsigned long long c = 0;
    Counts dummy;
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const double *__restrict__ yr = Y + (size_t)i * ld;
        for (int c0 = 0; c0 < n; c0 += kCertChunk) {
            double yv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = c0 + u * 256 + (int)threadIdx.x;
                yv[u] = j < n ? yr[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = c0 + u * 256 + (int)threadIdx.x;
                if (j >= n) break;
                const double y = yv[u];
                int ok;                                   // 1 yes, 0 no, -1 deferred
                if (y == 0.0) {
                    ok = zero_ok;
                } else if (!(y >= kDblMin)) {
                    ok = 0;
                } else {
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(y);
                    const int e = (int)((bits >> 52) & 0x7FFull) - 1023;
                    const double m =
                        __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
                    const double l2 = (double)e + (double)__builtin_amdgcn_logf((float)m);
                    const double te = l2 * s2 - kEta;
                    ok = -1;
                    if (fabs(te - rint(te)) > band) {
                        const double k = fmin(fmax(ceil(te), kDMin), kDMax);
                        const double lny = l2 * kLn2;
                        const double diff = lny - bound_ln(k);                    // > 0: no distance above k
                        const double low = (k - 1.0 + kEta) * lg - (lny + up);    // > 0: no distance below k
                        if (diff < -1e-5 || low < -1e-5) ok = 0;
                        else if (diff > 1e-5 && low > 1e-5) ok = 1;
                    }
                }
                if (ok < 0) {
                    queue[atomicAdd(&qn, 1)] = j;
                } else {
                    if (mask) mask[(size_t)i * n + j] = (uint8_t)ok;
                    c += ok;
                }
            }
            __syncthreads();
            const int q = qn;
            for (int t = threadIdx.x; t < q; t += 256) {
                const int j = queue[t];
                const double y = yr[j];
                const int k = rd_encode(y, il, dummy);
                const double lny = log(y);
                const bool ok = lny > bound_ln((double)k) && lny + up < ((double)k - 1.0 + kEta) * lg;
                if (mask) mask[(size_t)i * n + j] = ok ? 1 : 0;
                c += ok ? 1 : 0;
            }
            __syncthreads();
            if (threadIdx.x == 0) qn = 0;
            __syncthreads();
        }
    }
    // one atomic per workgroup: the count's address is shared by every workgroup
    __shared__ unsigned long long part[4];
    const unsigned long long s = wave_sum_u64(c);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(count, t);
    }
}

}  // namespace

size_t power_scratch_bytes() { return sizeof(PowerScratch); }

void launch_power_init(void *scratch, hipStream_t s) {
    hipLaunchKernelGGL(k_gamma_init, dim3(1), dim3(1), 0, s, (PowerScratch *)scratch);
}

void launch_power_step(const uint8_t *A, int n, const double *x, double *y, void *scratch, int step, hipStream_t s) {
    const int blocks = std::min((n + 3) / 4, 1024);
    hipLaunchKernelGGL(k_power_step, dim3(blocks), dim3(256), 0, s, A, n, x, y, (PowerScratch *)scratch, step);
}

void launch_power_fold(void *scratch, int last_step, hipStream_t s) {
    hipLaunchKernelGGL(k_power_fold, dim3(1), dim3(1), 0, s, (PowerScratch *)scratch, last_step);
}

void power_read(const void *host_copy, double *lo_ratio, double *hi_ratio) {
    const PowerScratch *sc = (const PowerScratch *)host_copy;
    double lo, hi;
    memcpy(&lo, &sc->best_lo, 8);
    memcpy(&hi, &sc->best_hi, 8);
    *lo_ratio = lo;
    *hi_ratio = hi;
}

void launch_certify(const double *Y, int ld, int n, const rdist_info *ginfo, bool weighted, double err_floor,
                    uint8_t *mask, unsigned long long *count, hipStream_t s) {
    const int blocks = std::min(n, 1024);
    if (weighted)
        hipLaunchKernelGGL(k_certify<true>, dim3(blocks), dim3(256), 0, s, Y, ld, n, ginfo, err_floor, mask, count);
    else
        hipLaunchKernelGGL(k_certify<false>, dim3(blocks), dim3(256), 0, s, Y, ld, n, ginfo, err_floor, mask, count);
}

}  // namespace rd
