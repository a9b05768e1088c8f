// rd_dynamic.hip -- edge changes on a kept graph without a new inversion.
//
// Adding, removing or re-weighting the edge src -> dst changes one entry of
// M = I - X: M' = M - delta e_dst e_src^T with delta = X'_{dst,src} -
// X_{dst,src} (gamma^w for an edge of weight w, 0 for none; Sec. 3.2).  The
// Sherman-Morrison identity gives the new inverse from the old one,
//   Y' = Y + f Y[:, dst] Y[src, :],   f = delta / (1 - delta Y[src, dst]),
// one pass over Y instead of an O(n^3) solve (the dynamic re-planning of the
// paper's Discussion, Applications).  The change is applied only if the new
// graph still passes the gate gamma Delta' < 1 (then M' is a nonsingular
// M-matrix, Y' >= 0 and the denominator is positive); otherwise the graph is
// left as it was.
//
// Rounding.  A removal (delta < 0) subtracts: an entry whose walks mostly
// used the removed edge keeps only the rounding error of the old value, and
// an entry the removal disconnects comes out as a tiny residue instead of 0.
// So every entry carries a bound beta on its relative error, propagated
// through each update to first order,
//   beta' Y' >= beta Y + (beta_f + beta_c + beta_r + u) |t| + u Y'
// (t = f c r the update term, u = 2^-53), with a 2^-16 relative margin for
// the second-order terms.  beta is kept as a 16-bit fixed-point -log2 with
// 8 fraction bits (q = floor(-256 log2 beta), decoded upwards), one pass
// of 2 bytes per entry beside Y's 8.  An entry is lost when its Y' is not
// positive while the term was not zero, when beta' exceeds 2^-20, or when
// D is asked for and the readout's integer boundary lies within beta' of it
// (in log_gamma units): then D of the computed Y' might differ from D of
// the exact one.  Lost entries are counted; the host re-inverts the changed
// graph from its kept adjacency when there are any.  The starting bound of
// an inversion is an assumption, max(2^-40, 8 n u / (1 - gamma Delta)).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_device.h"
#include "rd_launch.h"

namespace rd {

namespace {

constexpr double kU = 1.1102230246251565e-16;      // 2^-53
constexpr double kBetaFCap = 5.9604644775390625e-08;   // 2^-24: f itself too uncertain
constexpr int kRows = 4;                          // rows per step of the apply pass
constexpr int kApplyGroups = 8192;                // workgroups of the apply pass (grid-stride)

// beta <= 2^(-q/256), decoded upwards (the FP32 exp2 is within an ulp or two).
__device__ __forceinline__ float beta_decode(uint16_t q) {
    return __builtin_amdgcn_exp2f(-(float)q * (1.0f / 256.0f)) * 1.0000010f;
}

// The largest q with 2^(-q/256) >= beta (0 for beta >= 1).
__device__ __forceinline__ uint16_t beta_encode(double beta) {
    const float b = (float)(beta * 1.000001);
    if (!(b < 1.0f)) return 0;
    const float q = floorf(-__builtin_amdgcn_logf(b) * 256.0f - 0.01f);
    return (uint16_t)fminf(fmaxf(q, 0.0f), 65535.0f);
}

// D for an entry with computed Y' = y > 0 and relative error bound beta:
// the readout of rd_encode; `near` is raised when an integer boundary of
// t = log_gamma Y' - eta lies within beta |il| (1 + 1%) of t.
__device__ __forceinline__ int16_t encode_bounded(double y, double beta, double il, Counts &c, bool &near) {
    const double w = -beta * il * 1.01;   // il < 0
    if (y >= kDblMin) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(y);
        const int e = (int)((bits >> 52) & 0x7FFull) - 1023;
        const double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
        const double l2m = (double)__builtin_amdgcn_logf((float)m);
        const double s = kLn2 * il;
        const double te = ((double)e + l2m) * s - kEta;
        const double band = 1e-4 - 4e-6 * s;
        if (fabs(te - rint(te)) > band + w) return rd_clamp_d(ceil(te), c);
    } else {
        ++c.subnormal;
    }
    const double t = log(y) * il - kEta;
    const double dt = fabs(t - rint(t));
    near = dt <= w;
    if (dt < kBeta) ++c.ambiguous;
    return rd_clamp_d(ceil(t), c);
}

}  // namespace

// Out-degree of node j = set bits of its successor row.
__global__ __launch_bounds__(256) void k_outdeg_from_bits(const unsigned long long *__restrict__ bits, int n, int nw,
                                                          int32_t *__restrict__ outdeg) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    int c = 0;
    for (int w = 0; w < nw; ++w) c += __popcll(bits[(size_t)j * nw + w]);
    outdeg[j] = c;
}

// hist[d] = number of nodes of out-degree d (hist zeroed beforehand, n + 1 entries).
__global__ __launch_bounds__(256) void k_deg_hist(const int32_t *__restrict__ outdeg, int n, int32_t *__restrict__ hist) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) atomicAdd(&hist[outdeg[j]], 1);
}

// Every entry's bound set to the starting bound of an inversion of this
// graph (its gain and Delta from the graph's info).
__global__ __launch_bounds__(256) void k_beta_fill(uint16_t *__restrict__ Q, size_t count,
                                                   const rdist_info *__restrict__ ginfo, int n) {
    const double gd = ginfo->gamma * (double)ginfo->delta;
    const double b0 = fmax(9.094947017729282e-13, 8.0 * n * kU / fmax(1.0 - gd, 1e-300));   // 2^-40
    const uint16_t q = beta_encode(b0);
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < count; k += (size_t)gridDim.x * 256) Q[k] = q;
}

// Gate and snapshots, one thread per node i.  The gate needs Delta' only:
// with hist[d] = number of nodes of out-degree d, an added out-edge of src
// (degree k -> k + 1) gives max(Delta, k + 1); a removed one (k -> k - 1)
// lowers Delta to k - 1 only when src was the one node of degree Delta.
// Workgroup 0 writes the call's info and f.  The graph's own adjacency,
// out-degrees, histogram and successor bit are changed by the apply pass,
// after every read here.
// sm: [0] f, [1] beta_f, [2, 11) the call's rdist_info, [12] 1 / log gamma,
// [15] 1 when f is too uncertain to use, [16, 16 + n) Y's column dst,
// [16 + n, 16 + 2n) Y's row src, then 2n floats: the bounds of that column
// and that row.
__global__ __launch_bounds__(256) void k_sm_prep(const double *__restrict__ Y, int ld, int n,
                                                 const uint8_t *__restrict__ A, const int32_t *__restrict__ outdeg,
                                                 const int32_t *__restrict__ hist, const uint16_t *__restrict__ Q,
                                                 const rdist_info *__restrict__ ginfo, double *__restrict__ sm, int src,
                                                 int dst, int w_new) {
    rdist_info *ci = reinterpret_cast<rdist_info *>(sm + 2);
    const double gamma = ginfo->gamma;
    const int delta = ginfo->delta;
    const int w_old = A[(size_t)dst * n + src];
    const int k = outdeg[src];
    const int k_new = k + (w_new != 0) - (w_old != 0);
    const int delta_new = k_new > k ? max(delta, k_new) : (k_new < k && k == delta && hist[k] == 1 ? k_new : delta);
    // the entries of X the inversion itself would build for these weights
    const double xo = w_old ? pow(gamma, (double)w_old) : 0.0;
    const double xn = w_new ? pow(gamma, (double)w_new) : 0.0;
    const double d = xn - xo;
    const double ysd = Y[(size_t)src * ld + dst];
    const double den = fma(-d, ysd, 1.0);
    const bool ok = ginfo->status == RDIST_OK && gamma * (double)delta_new < 1.0 && den > 0.0;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (ok && i < n) {
        float *bc = reinterpret_cast<float *>(sm + 16 + 2 * (size_t)n);
        sm[16 + i] = Y[(size_t)i * ld + dst];
        sm[16 + n + i] = Y[(size_t)src * ld + i];
        bc[i] = beta_decode(Q[(size_t)i * n + dst]);
        bc[n + i] = beta_decode(Q[(size_t)src * n + i]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double bd = (xo != 0.0 && xn != 0.0) ? kU : 0.0;
        const double bsd = beta_decode(Q[(size_t)src * n + dst]);
        const double bden = fabs(d) * ysd * (bd + bsd) / den + kU;
        const double bf = (bd + bden + kU) * (1.0 + 1.0 / 65536.0);
        ci->status = ginfo->status != RDIST_OK ? ginfo->status : (ok ? RDIST_OK : RDIST_E_NOT_DD);
        ci->delta = ok ? delta_new : delta;
        ci->gamma = gamma;
        ci->n_unreachable = ci->n_subnormal = ci->n_saturated = 0;
        ci->n_ambiguous = ci->n_negative = 0;
        ci->n_uncertified = (ok && !(bf <= kBetaFCap)) ? (int64_t)n * n : 0;
        ci->fallback_fraction = 0.0;
        sm[0] = ok ? d / den : 0.0;
        sm[1] = bf;
        sm[12] = rd_inv_log(gamma);
        sm[15] = (ok && !(bf <= kBetaFCap)) ? 1.0 : 0.0;
    }
}

// Y[i][j] += f c[i] r[j] with the bound update, and D[i][j] read out from
// the new Y when D is given (counters and lost entries into the call's
// info).  A workgroup takes 256 V columns and steps over the rows kRows at
// a time, grid-stride (a fixed grid of about kApplyGroups workgroups: fewer
// per-workgroup starts and counter flushes), loading a step's rows before
// working on any of them; r and its bounds are read once.  V = 4 needs n and
// ld multiples of 4 and D (when given) 8-byte aligned.
template <int V>
__global__ __launch_bounds__(256) void k_sm_apply(double *__restrict__ Y, int ld, int n, uint16_t *__restrict__ Q,
                                                  double *__restrict__ sm, int16_t *__restrict__ D,
                                                  uint8_t *__restrict__ A, int32_t *__restrict__ outdeg,
                                                  int32_t *__restrict__ hist, unsigned long long *__restrict__ bits,
                                                  rdist_info *__restrict__ ginfo,
                                                  int src, int dst, int w_new) {
    rdist_info *ci = reinterpret_cast<rdist_info *>(sm + 2);
    if (ci->status != RDIST_OK) return;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        // the graph follows the change (the prep pass has read it already)
        const int w_old = A[(size_t)dst * n + src];
        A[(size_t)dst * n + src] = (uint8_t)w_new;
        const int k = outdeg[src], k_new = k + (w_new != 0) - (w_old != 0);
        outdeg[src] = k_new;
        hist[k] -= 1;
        hist[k_new] += 1;
        unsigned long long *word = bits + (size_t)src * ((n + 63) / 64) + (dst >> 6);
        const unsigned long long bit = 1ull << (dst & 63);
        *word = w_new ? (*word | bit) : (*word & ~bit);
        ginfo->delta = ci->delta;
    }
    if (sm[15] != 0.0) return;   // f too uncertain: the host re-inverts
    const double f = sm[0], bf = sm[1];
    const double *__restrict__ c = sm + 16;
    const double *__restrict__ r = sm + 16 + n;
    const float *__restrict__ bc = reinterpret_cast<const float *>(sm + 16 + 2 * (size_t)n);
    const float *__restrict__ br = bc + n;
    const double il = sm[12];
    const int j0 = (blockIdx.x * 256 + threadIdx.x) * V;
    const bool active = j0 < n;
    Counts cnt;
    unsigned lost = 0;
    double rv[V], brv[V];
    if (active) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool in = V == 1 || j0 + v < n;
            rv[v] = in ? r[j0 + v] : 0.0;
            brv[v] = in ? (double)br[j0 + v] : 0.0;
        }
    }
    for (int i0 = blockIdx.y * kRows; i0 < n && active; i0 += gridDim.y * kRows) {
    // all rows' loads first, so that they are in flight together
    double ya[kRows][V];
    uint16_t qa[kRows][V];
#pragma unroll
    for (int ii = 0; ii < kRows; ++ii) {
        const int i = min(i0 + ii, n - 1);
        const double *__restrict__ yr = Y + (size_t)i * ld + j0;
        const uint16_t *__restrict__ qr = Q + (size_t)i * n + j0;
        if constexpr (V == 4) {
            const d4 y4 = *reinterpret_cast<const d4 *>(yr);
            const ushort4 q4 = *reinterpret_cast<const ushort4 *>(qr);
            ya[ii][0] = y4.x; ya[ii][1] = y4.y; ya[ii][2] = y4.z; ya[ii][3] = y4.w;
            qa[ii][0] = q4.x; qa[ii][1] = q4.y; qa[ii][2] = q4.z; qa[ii][3] = q4.w;
        } else {
            ya[ii][0] = yr[0];
            qa[ii][0] = qr[0];
        }
    }
#pragma unroll
    for (int ii = 0; ii < kRows; ++ii) {
        const int i = i0 + ii;
        if (i >= n) break;
        const double fc = f * c[i];
        const double bci = (double)bc[i] + bf + kU;
        double *__restrict__ yr = Y + (size_t)i * ld + j0;
        uint16_t *__restrict__ qr = Q + (size_t)i * n + j0;
        double *y = ya[ii];
        uint16_t *q = qa[ii];
        int16_t dv[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double t = fc * rv[v];
            const double yo = y[v];
            const double yn = fma(fc, rv[v], yo);
            y[v] = yn;
            // entries the term leaves alone keep their value, bound and D
            bool bad = false;
            double beta = 0.0;
            if (t != 0.0) {
                if (yn >= kDblMin) {
                    double inv = __builtin_amdgcn_rcp(yn);
                    inv = fma(fma(-yn, inv, 1.0), inv, inv);
                    beta = ((double)beta_decode(q[v]) * yo + (bci + brv[v]) * fabs(t)) * inv *
                               (1.0 + 1.0 / 65536.0) + 2.0 * kU;
                    bad = !(beta <= kBetaCap);
                } else {
                    bad = true;   // cancelled to zero or below, or no relative bound (subnormal)
                    beta = 1.0;
                }
                q[v] = beta_encode(beta);
            }
            if (D) {
                if (yn > 0.0) {
                    bool near = false;
                    dv[v] = encode_bounded(yn, beta, il, cnt, near);
                    bad |= t != 0.0 && near;
                } else {
                    dv[v] = kUnreachable;
                    if (t == 0.0) {
                        if (yn == 0.0) ++cnt.unreachable;
                        else ++cnt.negative;
                    }
                }
            }
            lost += bad ? 1u : 0u;
        }
        if constexpr (V == 4) {
            d4 o;
            o.x = y[0]; o.y = y[1]; o.z = y[2]; o.w = y[3];
            *reinterpret_cast<d4 *>(yr) = o;
            *reinterpret_cast<ushort4 *>(qr) = make_ushort4(q[0], q[1], q[2], q[3]);
            if (D) {
                short4 s4 = make_short4(dv[0], dv[1], dv[2], dv[3]);
                *reinterpret_cast<short4 *>(D + (size_t)i * n + j0) = s4;
            }
        } else {
            yr[0] = y[0];
            qr[0] = q[0];
            if (D) D[(size_t)i * n + j0] = dv[0];
        }
    }
    }
    // one atomic per counter and workgroup: every workgroup adds into the same info
    __shared__ unsigned long long part[6][4];
    const unsigned long long v[6] = {wave_sum_u64(cnt.unreachable), wave_sum_u64(cnt.subnormal),
                                     wave_sum_u64(cnt.saturated),   wave_sum_u64(cnt.ambiguous),
                                     wave_sum_u64(cnt.negative),    wave_sum_u64(lost)};
    if ((threadIdx.x & 63) == 0)
        for (int t = 0; t < 6; ++t) part[t][threadIdx.x >> 6] = v[t];
    __syncthreads();
    if (threadIdx.x < 6) {
        const unsigned long long sum = part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] +
                                       part[threadIdx.x][3];
        unsigned long long *dst[6] = {(unsigned long long *)&ci->n_unreachable, (unsigned long long *)&ci->n_subnormal,
                                      (unsigned long long *)&ci->n_saturated, (unsigned long long *)&ci->n_ambiguous,
                                      (unsigned long long *)&ci->n_negative, (unsigned long long *)&ci->n_uncertified};
        if (sum) atomicAdd(dst[threadIdx.x], sum);
    }
}

// ---------------------------------------------------------------------------
// Several changes in one pass.  Applying changes 0 .. k-1 in order is the
// same as k rank-one steps, Y^(a+1) = Y^(a) + f_a c_a r_a^T with c_a the
// column dst_a and r_a the row src_a of Y^(a) (not of Y): a prep phase per
// change builds c_a and r_a from Y and the earlier terms (O(n a) each), with
// absolute error bounds, then one pass adds all k terms to every entry of Y
// and carries its bound through each term.  Batch scratch bs (doubles):
// [0, 8) f_a, [8, 16) beta_f_a, [16, 24) delta_a, [24, 32) beta of delta_a,
// [32, 40) new weights, [48, 48 + 6 k n): per change a the column, its bound,
// the row, its bound, f_a times the column and that product's bound (n each).
// ---------------------------------------------------------------------------

struct BatchOff {
    int n;
    __device__ __host__ size_t col(int a) const { return 48 + (size_t)a * 6 * n; }
    __device__ __host__ size_t ecol(int a) const { return col(a) + n; }
    __device__ __host__ size_t row(int a) const { return col(a) + 2 * (size_t)n; }
    __device__ __host__ size_t erow(int a) const { return col(a) + 3 * (size_t)n; }
    __device__ __host__ size_t fc(int a) const { return col(a) + 4 * (size_t)n; }    // f_a c_a[i]
    __device__ __host__ size_t efc(int a) const { return col(a) + 5 * (size_t)n; }   // its absolute bound
};

// f_b and its relative bound from Y^(b)[src_b, dst_b] = r_b[dst_b] (and its bound).
__device__ __forceinline__ void batch_f(const double *__restrict__ bs, const EdgeBatch &B, BatchOff o, int b,
                                        double &f, double &bf, double &den) {
    const double d = bs[16 + b], bd = bs[24 + b];
    const double ysd = bs[o.row(b) + B.dst[b]], eysd = bs[o.erow(b) + B.dst[b]];
    den = fma(-d, ysd, 1.0);
    f = d / den;
    bf = (bd + (fabs(d) * (eysd + fabs(ysd) * bd)) / den + 2.0 * kU) * (1.0 + 1.0 / 65536.0);
}

// Sequential checks of the batch (one thread): old weights (the graph's, or
// an earlier change's to the same edge), delta_a, and the gate on every
// intermediate graph through an upper bound of its Delta (the largest of
// Delta and every out-degree a change passes through).
__global__ void k_mb_gate(const uint8_t *__restrict__ A, const int32_t *__restrict__ outdeg, int n,
                          const rdist_info *__restrict__ ginfo, double *__restrict__ bs, double *__restrict__ sm,
                          EdgeBatch B) {
    rdist_info *ci = reinterpret_cast<rdist_info *>(sm + 2);
    const double gamma = ginfo->gamma;
    int dmax = ginfo->delta;
    bool ok = ginfo->status == RDIST_OK;
    for (int a = 0; a < B.k; ++a) {
        int w_old = A[(size_t)B.dst[a] * n + B.src[a]];
        int deg = outdeg[B.src[a]];
        for (int b = 0; b < a; ++b) {
            if (B.src[b] == B.src[a] && B.dst[b] == B.dst[a]) w_old = B.w[b];
        }
        // the running out-degree of src_a: the graph's plus the earlier changes at src_a
        int seen_w[8];
        int m = 0;
        for (int b = 0; b < a; ++b) {
            if (B.src[b] != B.src[a]) continue;
            bool first = true;
            for (int c = 0; c < m; ++c) first = first && seen_w[c] != B.dst[b];
            if (!first) continue;
            seen_w[m++] = B.dst[b];
            // the last change to edge src_a -> dst_b before a, against the graph's weight
            int last = B.w[b];
            for (int c = b + 1; c < a; ++c)
                if (B.src[c] == B.src[a] && B.dst[c] == B.dst[b]) last = B.w[c];
            deg += (last != 0) - (A[(size_t)B.dst[b] * n + B.src[a]] != 0);
        }
        const int deg_new = deg + (B.w[a] != 0) - (w_old != 0);
        dmax = max(dmax, deg_new);
        const double xo = w_old ? pow(gamma, (double)w_old) : 0.0;
        const double xn = B.w[a] ? pow(gamma, (double)B.w[a]) : 0.0;
        bs[16 + a] = xn - xo;
        bs[24 + a] = (xo != 0.0 && xn != 0.0) ? kU : 0.0;
        bs[32 + a] = (double)B.w[a];
    }
    ok = ok && gamma * (double)dmax < 1.0;
    ci->status = ginfo->status != RDIST_OK ? ginfo->status : (ok ? RDIST_OK : RDIST_E_NOT_DD);
    ci->delta = ginfo->delta;
    ci->gamma = gamma;
    ci->n_unreachable = ci->n_subnormal = ci->n_saturated = 0;
    ci->n_ambiguous = ci->n_negative = ci->n_uncertified = 0;
    ci->fallback_fraction = 0.0;
    sm[12] = rd_inv_log(gamma);
    sm[15] = 0.0;
}

// Phase a: column dst_a and row src_a of Y^(a), one thread per index,
// with absolute error bounds (first order; the product of two bounds kept).
__global__ __launch_bounds__(256) void k_mb_phase(const double *__restrict__ Y, int ld, int n,
                                                  const uint16_t *__restrict__ Q, double *__restrict__ bs,
                                                  const double *__restrict__ sm, EdgeBatch B, int a) {
    const rdist_info *ci = reinterpret_cast<const rdist_info *>(sm + 2);
    if (ci->status != RDIST_OK) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const BatchOff o{n};
    const int da = B.dst[a], sa = B.src[a];
    double c = Y[(size_t)i * ld + da], r = Y[(size_t)sa * ld + i];
    double ec = (double)beta_decode(Q[(size_t)i * n + da]) * fabs(c);
    double er = (double)beta_decode(Q[(size_t)sa * n + i]) * fabs(r);
    for (int b = 0; b < a; ++b) {
        double f, bf, den;
        batch_f(bs, B, o, b, f, bf, den);
        // column: + f_b c_b[i] r_b[dst_a]
        {
            const double cb = bs[o.col(b) + i], ecb = bs[o.ecol(b) + i];
            const double rb = bs[o.row(b) + da], erb = bs[o.erow(b) + da];
            const double t = f * cb * rb;
            c = fma(f * cb, rb, c);
            ec += fabs(f) * (ecb * fabs(rb) + fabs(cb) * erb + ecb * erb) + fabs(t) * (bf + 2.0 * kU) + kU * fabs(c);
        }
        // row: + f_b c_b[src_a] r_b[i]
        {
            const double cb = bs[o.col(b) + sa], ecb = bs[o.ecol(b) + sa];
            const double rb = bs[o.row(b) + i], erb = bs[o.erow(b) + i];
            const double t = f * cb * rb;
            r = fma(f * cb, rb, r);
            er += fabs(f) * (ecb * fabs(rb) + fabs(cb) * erb + ecb * erb) + fabs(t) * (bf + 2.0 * kU) + kU * fabs(r);
        }
    }
    bs[o.col(a) + i] = c;
    bs[o.ecol(a) + i] = ec * (1.0 + 1.0 / 65536.0);
    bs[o.row(a) + i] = r;
    bs[o.erow(a) + i] = er * (1.0 + 1.0 / 65536.0);
}

// f_a and its bound for every change; every denominator must be positive
// (it is, for graphs passing the gate, up to rounding); an f too uncertain to
// use leaves the whole batch to a re-inversion.
__global__ void k_mb_finish(double *__restrict__ bs, double *__restrict__ sm, EdgeBatch B, int n) {
    rdist_info *ci = reinterpret_cast<rdist_info *>(sm + 2);
    if (ci->status != RDIST_OK) return;
    const BatchOff o{n};
    bool lost = false;
    for (int a = 0; a < B.k; ++a) {
        double f, bf, den;
        batch_f(bs, B, o, a, f, bf, den);
        if (!(den > 0.0)) {
            ci->status = RDIST_E_NOT_DD;
            return;
        }
        bs[a] = f;
        bs[8 + a] = bf;
        lost = lost || !(bf <= kBetaFCap);
    }
    if (lost) {
        ci->n_uncertified = (int64_t)n * n;
        sm[15] = 1.0;
    }
}

// f_a c_a[i] and its absolute bound, one thread per row i (the pass reads
// them per row with scalar loads).
__global__ __launch_bounds__(256) void k_mb_fc(double *__restrict__ bs, const double *__restrict__ sm, EdgeBatch B,
                                               int n) {
    const rdist_info *ci = reinterpret_cast<const rdist_info *>(sm + 2);
    if (ci->status != RDIST_OK || sm[15] != 0.0) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const BatchOff o{n};
    // the pass's own rounding, u |y_a| after each of the k terms, is at most
    // k u (|y_0| + sum_a |t_a|): its share k u |f_a c_a[i]| |r_a[j]| rides
    // with the term's bound, the k u |y_0| share is added by the pass
    const double ku = (double)B.k * kU;
    for (int a = 0; a < B.k; ++a) {
        const double f = bs[a], bf = bs[8 + a];
        const double c = bs[o.col(a) + i], ec = bs[o.ecol(a) + i];
        const double fc = f * c;
        bs[o.fc(a) + i] = fc;
        bs[o.efc(a) + i] = fabs(f) * ec + fabs(fc) * (bf + kU + ku);
    }
}

// The batch's pass over Y: every entry gets all k terms in order, its
// absolute error bound grows by each term's, and the new bound, lost check
// and readout are those of the single change.  A workgroup takes 256 V
// columns (their rows r_a and bounds in registers) and steps over the rows
// two at a time, grid-stride.  Block (0, 0) applies the changes to the
// graph's adjacency, out-degrees, histogram (Delta' by the single change's
// rule, change by change) and successor bits.
template <int V>
__global__ __launch_bounds__(256) void k_mb_apply(double *__restrict__ Y, int ld, int n, uint16_t *__restrict__ Q,
                                                  const double *__restrict__ bs, double *__restrict__ sm,
                                                  int16_t *__restrict__ D, uint8_t *__restrict__ A,
                                                  int32_t *__restrict__ outdeg, int32_t *__restrict__ hist,
                                                  unsigned long long *__restrict__ bits, rdist_info *__restrict__ ginfo,
                                                  EdgeBatch B) {
    rdist_info *ci = reinterpret_cast<rdist_info *>(sm + 2);
    if (ci->status != RDIST_OK) return;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        int delta = ginfo->delta;
        const int nw = (n + 63) / 64;
        for (int a = 0; a < B.k; ++a) {
            const int s = B.src[a], d = B.dst[a], w = B.w[a];
            const int w_old = A[(size_t)d * n + s];
            const int k = outdeg[s], k_new = k + (w != 0) - (w_old != 0);
            delta = k_new > k ? max(delta, k_new) : (k_new < k && k == delta && hist[k] == 1 ? k_new : delta);
            A[(size_t)d * n + s] = (uint8_t)w;
            outdeg[s] = k_new;
            hist[k] -= 1;
            hist[k_new] += 1;
            unsigned long long *word = bits + (size_t)s * nw + (d >> 6);
            const unsigned long long bit = 1ull << (d & 63);
            *word = w ? (*word | bit) : (*word & ~bit);
        }
        ginfo->delta = delta;
        ci->delta = delta;
    }
    if (sm[15] != 0.0) return;   // an f too uncertain: the host re-inverts
    const BatchOff o{n};
    const int K = B.k;
    const double il = sm[12];
    const int j0 = (blockIdx.x * 256 + threadIdx.x) * V;
    const bool active = j0 < n;
    double rv[8][V];
    float erv[8][V];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool in = a < K && active && j0 + v < n;
            rv[a][v] = in ? bs[o.row(a) + j0 + v] : 0.0;
            erv[a][v] = in ? (float)(bs[o.erow(a) + j0 + v] * (1.0 + 1.0 / 65536.0)) : 0.0f;
        }
    }
    Counts cnt;
    unsigned lost = 0;
    for (int i0 = blockIdx.y * kRows; i0 < n && active; i0 += gridDim.y * kRows)
#pragma unroll 1
        for (int ii = 0; ii < kRows; ++ii) {
            const int i = i0 + ii;
            if (i >= n) break;
            double fc[8], efc[8];   // uniform over the workgroup: scalar loads
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                fc[a] = a < K ? bs[o.fc(a) + i] : 0.0;
                efc[a] = a < K ? bs[o.efc(a) + i] : 0.0;
            }
            double *__restrict__ yr = Y + (size_t)i * ld + j0;
            uint16_t *__restrict__ qr = Q + (size_t)i * n + j0;
            double y[V];
            uint16_t q[V];
            if constexpr (V == 2) {
                const double2 y2 = *reinterpret_cast<const double2 *>(yr);
                const ushort2 q2 = *reinterpret_cast<const ushort2 *>(qr);
                y[0] = y2.x; y[1] = y2.y;
                q[0] = q2.x; q[1] = q2.y;
            } else {
                y[0] = yr[0];
                q[0] = qr[0];
            }
            int16_t dv[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double y0 = y[v];
                double yn = y0, E = 0.0;
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    if (a >= K) break;
                    yn = fma(fc[a], rv[a][v], yn);
                    E = fma(efc[a], fabs(rv[a][v]), E);
                    E = fma(fabs(fc[a]), (double)erv[a][v], E);
                }
                // a term that is not exactly zero, or one whose operands are uncertain,
                // leaves a positive bound: those entries are the touched ones
                const bool touched = E > 0.0;
                y[v] = yn;
                bool bad = false;
                double beta = 0.0;
                if (touched) {
                    if (yn >= kDblMin) {
                        double inv = __builtin_amdgcn_rcp(yn);
                        inv = fma(fma(-yn, inv, 1.0), inv, inv);
                        beta = (((double)beta_decode(q[v]) + (double)K * kU) * fabs(y0) + E) * inv *
                                   (1.0 + 1.0 / 65536.0) + 2.0 * kU;
                        bad = !(beta <= kBetaCap);
                    } else {
                        bad = true;
                        beta = 1.0;
                    }
                    q[v] = beta_encode(beta);
                }
                if (D) {
                    if (yn > 0.0) {
                        bool near = false;
                        dv[v] = encode_bounded(yn, beta, il, cnt, near);
                        bad |= touched && near;
                    } else {
                        dv[v] = kUnreachable;
                        if (!touched) {
                            if (yn == 0.0) ++cnt.unreachable;
                            else ++cnt.negative;
                        }
                    }
                }
                lost += bad ? 1u : 0u;
            }
            if constexpr (V == 2) {
                *reinterpret_cast<double2 *>(yr) = make_double2(y[0], y[1]);
                *reinterpret_cast<ushort2 *>(qr) = make_ushort2(q[0], q[1]);
                if (D) *reinterpret_cast<short2 *>(D + (size_t)i * n + j0) = make_short2(dv[0], dv[1]);
            } else {
                yr[0] = y[0];
                qr[0] = q[0];
                if (D) D[(size_t)i * n + j0] = dv[0];
            }
        }
    __shared__ unsigned long long part[6][4];
    const unsigned long long vsum[6] = {wave_sum_u64(cnt.unreachable), wave_sum_u64(cnt.subnormal),
                                        wave_sum_u64(cnt.saturated),   wave_sum_u64(cnt.ambiguous),
                                        wave_sum_u64(cnt.negative),    wave_sum_u64(lost)};
    if ((threadIdx.x & 63) == 0)
        for (int t = 0; t < 6; ++t) part[t][threadIdx.x >> 6] = vsum[t];
    __syncthreads();
    if (threadIdx.x < 6) {
        const unsigned long long sum = part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] +
                                       part[threadIdx.x][3];
        unsigned long long *dst[6] = {(unsigned long long *)&ci->n_unreachable, (unsigned long long *)&ci->n_subnormal,
                                      (unsigned long long *)&ci->n_saturated, (unsigned long long *)&ci->n_ambiguous,
                                      (unsigned long long *)&ci->n_negative, (unsigned long long *)&ci->n_uncertified};
        if (sum) atomicAdd(dst[threadIdx.x], sum);
    }
}

size_t batch_scratch_doubles(int n) { return BatchOff{n}.col(kMaxBatch); }

void launch_edge_batch_prep(const double *Y, int ld, int n, const uint16_t *Q, double *sm, double *bs,
                            const uint8_t *A, const int32_t *outdeg, const rdist_info *ginfo, const EdgeBatch &B,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_mb_gate, dim3(1), dim3(1), 0, s, A, outdeg, n, ginfo, bs, sm, B);
    for (int a = 0; a < B.k; ++a)
        hipLaunchKernelGGL(k_mb_phase, dim3((n + 255) / 256), dim3(256), 0, s, Y, ld, n, Q, bs, sm, B, a);
    hipLaunchKernelGGL(k_mb_finish, dim3(1), dim3(1), 0, s, bs, sm, B, n);
    hipLaunchKernelGGL(k_mb_fc, dim3((n + 255) / 256), dim3(256), 0, s, bs, sm, B, n);
}

void launch_edge_batch_apply(double *Y, int ld, int n, uint16_t *Q, double *sm, const double *bs, int16_t *D,
                             uint8_t *A, int32_t *outdeg, int32_t *hist, unsigned long long *bits, rdist_info *ginfo,
                             const EdgeBatch &B, hipStream_t s) {
    const bool v2 = n % 2 == 0 && ld % 2 == 0 && ((uintptr_t)D & 3) == 0;
    const int gx = v2 ? (n / 2 + 255) / 256 : (n + 255) / 256;
    const int gy = std::max(1, std::min((n + kRows - 1) / kRows, kApplyGroups / gx));
    if (v2)
        hipLaunchKernelGGL(k_mb_apply<2>, dim3(gx, gy), dim3(256), 0, s, Y, ld, n, Q, bs, sm, D, A, outdeg, hist, bits,
                           ginfo, B);
    else
        hipLaunchKernelGGL(k_mb_apply<1>, dim3(gx, gy), dim3(256), 0, s, Y, ld, n, Q, bs, sm, D, A, outdeg, hist, bits,
                           ginfo, B);
}

void launch_outdeg_from_bits(const unsigned long long *bits, int n, int32_t *outdeg, hipStream_t s) {
    const int nw = (n + 63) / 64;
    hipLaunchKernelGGL(k_outdeg_from_bits, dim3((n + 255) / 256), dim3(256), 0, s, bits, n, nw, outdeg);
}

void launch_beta_fill(uint16_t *Q, int n, const rdist_info *ginfo, hipStream_t s) {
    const size_t count = (size_t)n * n;
    const int blocks = (int)std::min<size_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(k_beta_fill, dim3(blocks), dim3(256), 0, s, Q, count, ginfo, n);
}

void launch_deg_hist(const int32_t *outdeg, int n, int32_t *hist, hipStream_t s) {
    launch_fill_i32(hist, (size_t)n + 1, s);
    hipLaunchKernelGGL(k_deg_hist, dim3((n + 255) / 256), dim3(256), 0, s, outdeg, n, hist);
}

void launch_edge_prep(const double *Y, int ld, int n, const uint8_t *A, const int32_t *outdeg, const int32_t *hist,
                      const uint16_t *Q, const rdist_info *ginfo, double *sm, int src, int dst, int weight,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_sm_prep, dim3((n + 255) / 256), dim3(256), 0, s, Y, ld, n, A, outdeg, hist, Q, ginfo, sm,
                       src, dst, weight);
}

void launch_edge_apply(double *Y, int ld, int n, uint16_t *Q, double *sm, int16_t *D, uint8_t *A, int32_t *outdeg,
                       int32_t *hist, unsigned long long *bits, rdist_info *ginfo, int src, int dst, int weight,
                       hipStream_t s) {
    const bool v4 = n % 4 == 0 && ld % 4 == 0 && ((uintptr_t)D & 7) == 0;
    const int gx = v4 ? (n / 4 + 255) / 256 : (n + 255) / 256;
    const int gy = std::max(1, std::min((n + kRows - 1) / kRows, kApplyGroups / gx));
    if (v4) {
        hipLaunchKernelGGL(k_sm_apply<4>, dim3(gx, gy), dim3(256), 0, s, Y, ld, n, Q, sm, D, A, outdeg, hist, bits,
                           ginfo, src, dst, weight);
    } else {
        hipLaunchKernelGGL(k_sm_apply<1>, dim3(gx, gy), dim3(256), 0, s, Y, ld, n, Q, sm, D, A, outdeg, hist, bits,
                           ginfo, src, dst, weight);
    }
}

}  // namespace rd
