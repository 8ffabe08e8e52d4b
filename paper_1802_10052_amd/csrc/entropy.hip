// Bond (Schmidt) entropy of a pure state (Sec. IV, bond entropy; S(l) of the convergence
// section): rho_l = M M^dagger with M the state reshaped to d^l x d^(L-l), its eigenvalues
// Lambda_j, and S = -sum_j Lambda_j log Lambda_j. The paper computes rho_l by a matrix product
// and takes an eigendecomposition (noting the SVD of M gives the same spectrum).
//
// Here:
//   1. rho = R R^H on the FP64 matrix cores (v_mfma_f64_16x16x4f64), with R = M when
//      d^l <= d^(L-l) and R = M^T otherwise (same non-zero spectrum, smaller Gram matrix);
//      R is read in place from the state, never copied.
//   2. Householder reduction of the Hermitian rho to a real symmetric tridiagonal matrix on the
//      GPU: each step's rank-2 update of the trailing matrix is fused with the matrix-vector
//      product that the next step needs, on the lower triangle only (the product takes the upper
//      part as the conjugate of the lower), so half the trailing matrix streams once per step.
//   3. Eigenvalues of the tridiagonal matrix by bisection on Sturm counts on the GPU, one thread
//      per eigenvalue.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <utility>
#include <vector>

#include "ed_internal.h"

namespace ed {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------ Gram matrix
// rho[a][a'] = sum_b R[a][b] conj(R[a'][b]), R[r][c] = psi[r*rs + c*cs], n x K.
// Block tile 64 x 64 of rho per workgroup (4 waves, each 32 x 32 = 2 x 2 MFMA tiles), K consumed
// 16 at a time through LDS. Only blocks with I >= J are computed; the mirrored block is written
// as the conjugate transpose so rho is stored in full.
constexpr int kGB = 64;
constexpr int kGK = 16;

template <bool ROWC>  // ROWC: R's columns are contiguous in memory (cs == 1)
__global__ __launch_bounds__(256) void gram_mfma(const double2* __restrict__ psi, int64_t rs, int64_t cs,
                                                 int n, int64_t K, double2* __restrict__ rho, int nb) {
    __shared__ double Ar[kGB][kGK + 1], Ai[kGB][kGK + 1], Br[kGB][kGK + 1], Bi[kGB][kGK + 1];
    // triangular block index -> (I, J), I >= J
    int b = blockIdx.x, I = 0;
    while (b > I) {
        b -= I + 1;
        ++I;
    }
    const int J = b;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
    dbl4 accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            accr[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            acci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
    const int r0 = I * kGB, c0 = J * kGB;
    for (int64_t k0 = 0; k0 < K; k0 += kGK) {
        // load 64 x 16 of R rows r0.. and rows c0..; 1024 elements each, 4 per thread
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = t + 256 * e;
            int rr, kk;
            if (ROWC) {
                rr = idx / kGK;
                kk = idx % kGK;
            } else {
                rr = idx % kGB;
                kk = idx / kGB;
            }
            double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
            if (k0 + kk < K) {
                if (r0 + rr < n) va = psi[int64_t(r0 + rr) * rs + (k0 + kk) * cs];
                if (c0 + rr < n) vb = psi[int64_t(c0 + rr) * rs + (k0 + kk) * cs];
            }
            Ar[rr][kk] = va.x;
            Ai[rr][kk] = va.y;
            Br[rr][kk] = vb.x;
            Bi[rr][kk] = vb.y;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 4) {
            const int ka = kk + (lane >> 4), ra = lane & 15;
            double ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ar[i] = Ar[wr + 16 * i + ra][ka];
                ai[i] = Ai[wr + 16 * i + ra][ka];
                br[i] = Br[wc + 16 * i + ra][ka];
                bi[i] = Bi[wc + 16 * i + ra][ka];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accr[i][j], 0, 0, 0);
                    accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bi[j], accr[i][j], 0, 0, 0);
                    acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], acci[i][j], 0, 0, 0);
                    acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar[i], bi[j], acci[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // D[row][col] of a 16x16 f64 tile: register q of lane l holds row l/16 + 4q, column l%16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = r0 + wr + 16 * i + (lane >> 4) + 4 * q;
                const int col = c0 + wc + 16 * j + (lane & 15);
                if (row < n && col < n) {
                    const double re = accr[i][j][q], im = acci[i][j][q];
                    rho[int64_t(row) * n + col] = make_double2(re, im);
                    if (I != J) rho[int64_t(col) * n + row] = make_double2(re, -im);
                }
            }
}

// ------------------------------------------------------------------------------ Householder
// State of the reduction kept in device memory:
//   v[n]   current Householder vector (v[0] = 1) of the step, indexed from row k+1
//   y[n]   tau * A22 v, then w = y + alpha v
//   d[n], e[n]  tridiagonal diagonal / |sub-diagonal|
//   part[nblk][n] partial row sums of the fused update
//   sc[4]  tau (complex) at sc[0]
constexpr int kFR = 16;    // rows per workgroup tile of the fused update
constexpr int kFC = 512;   // columns per workgroup tile

__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * b
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// Fused rank-2 update and next product, lower triangle only: for the trailing block [s, n)
// (s = k + 2), A[i][j] -= v_i conj(w_j) + w_i conj(v_j) (the update of step k; v, w hold entries for
// rows >= k+1) and the partial sums of A_new vn (vn: the next Householder vector, rows >= k+2).
// rho is Hermitian, so only entries with j <= i of the trailing block are
// kept up to date (the upper triangle is never read again). The trailing block [s, n) is cut into
// 64 x 64 tiles (R, C), C <= R; each workgroup updates one tile and writes, for the next product
// y = A_new vn, the row sums of its rows (slot C) and the conjugate column sums of its strictly
// lower entries (slot R, y_j += conj(A_ij) vn_i). In a diagonal tile both go to slot R of the same
// index. Index i of block B thus gets slot b from tile (B, b) for b < B, (B, B) for b = B and
// (b, B) for b > B: every slot exactly once, summed in a fixed order by hh_reduce. Column s, the
// one the next step finishes, is also written to cn (rows >= s), so that step reads it
// contiguously.
constexpr int kSB = 64;

__global__ __launch_bounds__(256) void hh_fused_sym(double2* __restrict__ A, int n, int s,
                                                    const double2* __restrict__ v, const double2* __restrict__ w,
                                                    const double2* __restrict__ vn, double2* __restrict__ part,
                                                    double2* __restrict__ cn) {
    __shared__ double2 colred[4][kSB];
    __shared__ double2 rowred[kSB];
    int b = blockIdx.x, R = 0;
    while (b > R) {
        b -= R + 1;
        ++R;
    }
    const int C = b;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int j = s + C * kSB + lane;
    const bool jok = j < n;
    const double2 zero = make_double2(0.0, 0.0);
    const double2 vj = jok ? v[j] : zero, wj = jok ? w[j] : zero, vnj = jok ? vn[j] : zero;
    double2 colacc = zero;
    for (int rr = 0; rr < kSB / 4; ++rr) {
        const int li = wv * (kSB / 4) + rr;
        const int i = s + R * kSB + li;
        if (i >= n) break;  // uniform over the wave
        const double2 vi = v[i], wi = w[i], vni = vn[i];
        double2 rp = zero;
        if (jok && j <= i) {
            double2 a = A[int64_t(i) * n + j];
            const double2 t1 = cmulc(vi, conjd(wj)), t2 = cmulc(wi, conjd(vj));
            a.x -= t1.x + t2.x;
            a.y -= t1.y + t2.y;
            A[int64_t(i) * n + j] = a;
            if (C == 0 && lane == 0) cn[i] = a;  // j == s
            rp = cmulc(a, vnj);
            if (j < i) {
                const double2 q = cmulc(conjd(a), vni);
                colacc.x += q.x;
                colacc.y += q.y;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rp.x += __shfl_down(rp.x, off, 64);
            rp.y += __shfl_down(rp.y, off, 64);
        }
        if (lane == 0) {
            if (R == C) rowred[li] = rp;
            else part[int64_t(C) * n + i] = rp;
        }
    }
    colred[wv][lane] = colacc;
    __syncthreads();
    if (wv == 0 && jok) {
        double2 cs = colred[0][lane];
        for (int q = 1; q < 4; ++q) {
            cs.x += colred[q][lane].x;
            cs.y += colred[q][lane].y;
        }
        if (R == C) {
            cs.x += rowred[lane].x;
            cs.y += rowred[lane].y;
        }
        part[int64_t(R) * n + j] = cs;
    }
}

// ys[i] = sum over the nslots partial sums of row i (i in [c, n)). A workgroup takes 32 rows; its
// 8 groups of 32 threads sum the slots g, g + 8, g + 16, ... of each row, and the 8 group sums are
// added in group order (a fixed order, so results are reproducible).
constexpr int kRedRows = 32, kRedGroups = 8;

__global__ __launch_bounds__(kRedRows * kRedGroups) void hh_reduce(const double2* __restrict__ part, int nslots,
                                                                   int c, int n, double2* __restrict__ ys) {
    __shared__ double2 red[kRedGroups][kRedRows];
    const int r = int(threadIdx.x) % kRedRows, g = int(threadIdx.x) / kRedRows;
    const int i = c + int(blockIdx.x) * kRedRows + r;
    double2 acc = make_double2(0.0, 0.0);
    if (i < n)
        for (int b = g; b < nslots; b += kRedGroups) {
            const double2 p = part[int64_t(b) * n + i];
            acc.x += p.x;
            acc.y += p.y;
        }
    red[g][r] = acc;
    __syncthreads();
    if (g == 0 && i < n) {
        double2 sum = red[0][r];
#pragma unroll
        for (int q = 1; q < kRedGroups; ++q) {
            sum.x += red[q][r].x;
            sum.y += red[q][r].y;
        }
        ys[i] = sum;
    }
}

// Single-workgroup step kernel (1024 threads). Given ys = A22 v for the current step k (rows
// k+1..n-1, from hh_reduce) it: forms y = tau (A22 v); alpha = -1/2 tau (y^H v); w = y + alpha v;
// updates column k+1 of the trailing matrix (rows k+1..n-1) with the rank-2 term, into ys; records
// d[k+1]; builds the next Householder vector from rows k+2.. of that column, with tau, beta.
// For k = -1 it only builds the first Householder vector from column 0.
constexpr int kStepThreads = 1024;

__device__ double block_reduce(double v, double* lds) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kStepThreads / 64; ++i) s += lds[i];
    __syncthreads();
    return s;
}

// the same for a complex value: both parts reduced together, in a fixed order
__device__ double2 block_reduce2(double2 v, double2* lds) {
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_down(v.x, off, 64);
        v.y += __shfl_down(v.y, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    for (int i = 0; i < kStepThreads / 64; ++i) {
        s.x += lds[i].x;
        s.y += lds[i].y;
    }
    __syncthreads();
    return s;
}

// cin: column k+1 as the previous fused update left it, contiguous (rows >= k+1), or null to read
// it from the matrix. Every thread keeps the same rows i = k+1+t, k+1+t+1024, ... through the
// passes, so a value it wrote is read back by the same thread.
__global__ __launch_bounds__(kStepThreads) void hh_step(const double2* __restrict__ A, int n, int k,
                                                        double2* __restrict__ v, double2* __restrict__ y,
                                                        double2* __restrict__ vn, double2* __restrict__ ys,
                                                        double* __restrict__ d, double* __restrict__ e,
                                                        double2* __restrict__ sc, const double2* __restrict__ cin) {
    double2* const col = ys;  // column c of the trailing matrix after this step's update
    __shared__ double lds[kStepThreads / 64];
    __shared__ double2 lds2[kStepThreads / 64];
    __shared__ double2 syc;
    const int t = threadIdx.x;
    const int c = k + 1;  // column of the trailing matrix to finish now
    double nx = 0.0;      // |column c|^2 over rows c+2..n-1
    if (k >= 0) {
        const double2 tau = sc[0];
        // y_i = tau * (A22 v)_i, i = k+1..n-1 (the sums from hh_reduce); also y^H v
        double2 yhv = make_double2(0.0, 0.0);
        for (int i = c + t; i < n; i += kStepThreads) {
            const double2 yi = cmulc(tau, ys[i]);
            y[i] = yi;
            if (i == c) syc = yi;
            const double2 vi = v[i];
            // y^H v = sum conj(y_i) v_i
            yhv.x += yi.x * vi.x + yi.y * vi.y;
            yhv.y += yi.x * vi.y - yi.y * vi.x;
        }
        yhv = block_reduce2(yhv, lds2);
        // alpha = -1/2 tau (y^H v); w = y + alpha v
        const double2 tt = cmulc(tau, yhv);
        const double2 alpha = make_double2(-0.5 * tt.x, -0.5 * tt.y);
        const double2 vc = v[c], avc = cmulc(alpha, vc);
        const double2 wc = make_double2(syc.x + avc.x, syc.y + avc.y);
        // w, and the update of column c (rows c..n-1): A[i][c] -= v_i conj(w_c) + w_i conj(v_c).
        // Column c is finished by this step (later steps take rows and columns > c), so the
        // updated column goes to col = ys (free once y is formed) instead of back into A
        for (int i = c + t; i < n; i += kStepThreads) {
            const double2 vi = v[i], yi = y[i];
            const double2 av = cmulc(alpha, vi);
            const double2 wi = make_double2(yi.x + av.x, yi.y + av.y);
            y[i] = wi;
            double2 a = cin ? cin[i] : A[int64_t(i) * n + c];
            const double2 t1 = cmulc(vi, conjd(wc)), t2 = cmulc(wi, conjd(vc));
            a.x -= t1.x + t2.x;
            a.y -= t1.y + t2.y;
            col[i] = a;
            if (i >= c + 2) nx += a.x * a.x + a.y * a.y;
        }
    } else {
        for (int i = c + t; i < n; i += kStepThreads) {
            const double2 a = A[int64_t(i) * n + c];
            col[i] = a;
            if (i >= c + 2) nx += a.x * a.x + a.y * a.y;
        }
    }
    nx = block_reduce(nx, lds);  // its barriers also publish col
    // diagonal of row c and Householder vector of column c below the diagonal (rows c+1..)
    if (t == 0) d[c] = col[c].x;
    if (c + 1 >= n) return;
    const double2 al = col[c + 1];
    double2 tau = make_double2(0.0, 0.0);
    double beta;
    double2 inv = make_double2(0.0, 0.0);
    if (nx == 0.0 && al.y == 0.0) {
        beta = al.x;  // H = I
    } else {
        const double nrm = sqrt(al.x * al.x + al.y * al.y + nx);
        beta = al.x >= 0.0 ? -nrm : nrm;
        tau = make_double2((beta - al.x) / beta, -al.y / beta);
        // 1 / (alpha - beta)
        const double2 den = make_double2(al.x - beta, al.y);
        const double dd = den.x * den.x + den.y * den.y;
        inv = make_double2(den.x / dd, -den.y / dd);
    }
    if (t == 0) {
        e[c] = fabs(beta);
        sc[0] = tau;
        vn[c + 1] = make_double2(1.0, 0.0);
    }
    for (int i = c + 2 + t; i < n; i += kStepThreads) vn[i] = cmulc(col[i], inv);
}

// GEMV for the first step: part[cb][i] = sum_{j in tile} A[i][j] v_j over rows/cols >= s
__global__ __launch_bounds__(256) void hh_gemv(const double2* __restrict__ A, int n, int s,
                                               const double2* __restrict__ vn, double2* __restrict__ part) {
    const int r = n - s;
    const int ncb = (r + kFC - 1) / kFC;
    const int rb = blockIdx.x / ncb, cb = blockIdx.x % ncb;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cbeg = s + cb * kFC;
    for (int ii = 0; ii < kFR / 4; ++ii) {
        const int i = s + rb * kFR + wv * (kFR / 4) + ii;
        if (i >= n) break;
        double2 acc = make_double2(0.0, 0.0);
        for (int jj = lane; jj < kFC; jj += 64) {
            const int j = cbeg + jj;
            if (j >= n) break;
            const double2 p = cmulc(A[int64_t(i) * n + j], vn[j]);
            acc.x += p.x;
            acc.y += p.y;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            acc.x += __shfl_down(acc.x, off, 64);
            acc.y += __shfl_down(acc.y, off, 64);
        }
        if (lane == 0) part[int64_t(cb) * n + i] = acc;
    }
}

// ------------------------------------------------------------------------------ tridiagonal eigenvalues
// Every eigenvalue of the real symmetric tridiagonal T (diagonal d, off-diagonal e >= 0) by
// bisection on Sturm counts: the pivots of the LDL^T factorisation of T - x I have as many
// negative entries as T has eigenvalues below x (Sylvester's law of inertia), and the pivots
// obey q_0 = d_0 - x, q_i = d_i - x - e_{i-1}^2 / q_{i-1}. A pivot smaller in magnitude than
// pivmin is replaced by -pivmin (a perturbation of T of at most pivmin per entry), so no pivot
// is zero. Thread k finds the k-th smallest eigenvalue on its own, from the Gershgorin interval
// down to a width of eps |T|: its result depends on d, e and k only, not on the launch shape.
constexpr int kBisThreads = 256;
constexpr int kBndThreads = 1024;

// One workgroup: e2[i] = e[i]^2 (i < n-1); bnd = {lower, upper bound of the spectrum, pivmin,
// absolute tolerance}.
__global__ __launch_bounds__(kBndThreads) void tri_bounds(const double* __restrict__ d, const double* __restrict__ e,
                                                          int n, double* __restrict__ e2, double* __restrict__ bnd) {
    __shared__ double rlo[kBndThreads / 64], rhi[kBndThreads / 64], rem[kBndThreads / 64];
    const int t = threadIdx.x;
    double lo = HUGE_VAL, hi = -HUGE_VAL, em = 0.0;
    for (int i = t; i < n; i += kBndThreads) {
        const double el = i > 0 ? e[i - 1] : 0.0, er = i + 1 < n ? e[i] : 0.0;
        lo = fmin(lo, d[i] - el - er);
        hi = fmax(hi, d[i] + el + er);
        if (i + 1 < n) {
            e2[i] = er * er;
            em = fmax(em, er * er);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_down(lo, off, 64));
        hi = fmax(hi, __shfl_down(hi, off, 64));
        em = fmax(em, __shfl_down(em, off, 64));
    }
    if ((t & 63) == 0) {
        rlo[t >> 6] = lo;
        rhi[t >> 6] = hi;
        rem[t >> 6] = em;
    }
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < kBndThreads / 64; ++w) {
            lo = fmin(lo, rlo[w]);
            hi = fmax(hi, rhi[w]);
            em = fmax(em, rem[w]);
        }
        const double tnorm = fmax(fabs(lo), fabs(hi));
        const double pivmin = DBL_MIN * fmax(1.0, em);
        // widen by the rounding of the counts themselves, so that count(lower) = 0 and
        // count(upper) = n hold in floating point
        const double pad = 2.1 * DBL_EPSILON * tnorm * n + 4.2 * pivmin;
        bnd[0] = lo - pad;
        bnd[1] = hi + pad;
        bnd[2] = pivmin;
        bnd[3] = DBL_EPSILON * fmax(tnorm, DBL_MIN);
    }
}

__device__ __forceinline__ int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int n, double x,
                                           double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

// lam[k] = the k-th smallest eigenvalue, k < n. Invariant: count(lo) <= k < count(hi).
__global__ __launch_bounds__(kBisThreads) void tri_bisect(const double* __restrict__ d, const double* __restrict__ e2,
                                                          int n, const double* __restrict__ bnd, double* __restrict__ lam) {
    const int k = int(blockIdx.x) * kBisThreads + int(threadIdx.x);
    if (k >= n) return;
    double lo = bnd[0], hi = bnd[1];
    const double pivmin = bnd[2], tol = bnd[3];
    for (int it = 0; it < 2100 && hi - lo > tol; ++it) {
        const double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(d, e2, n, mid, pivmin) <= k) lo = mid;
        else hi = mid;
    }
    lam[k] = lo + 0.5 * (hi - lo);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct EntWS {
    double2* rho;
    double2* v;
    double2* y;
    double2* vn;
    double2* ys;
    double2* cn;  // the next step's column, written contiguously by the fused update
    double2* part;
    double* d;
    double* e;
    double2* sc;
};

// partial-sum slots: the first product's column blocks, or the symmetric tiles' block count
int part_slots(int n) { return std::max((n + kFC - 1) / kFC, (n + kSB - 1) / kSB) + 1; }

size_t entropy_bytes(int n) {
    return align256(size_t(n) * n * sizeof(double2)) + 5 * align256(size_t(n) * sizeof(double2)) +
           align256(size_t(part_slots(n)) * n * sizeof(double2)) + 2 * align256(size_t(n) * sizeof(double)) +
           align256(4 * sizeof(double2));
}

EntWS carve_ent(void* ws, int n) {
    char* p = static_cast<char*>(ws);
    EntWS w;
    w.rho = reinterpret_cast<double2*>(p);
    p += align256(size_t(n) * n * sizeof(double2));
    w.v = reinterpret_cast<double2*>(p);
    p += align256(size_t(n) * sizeof(double2));
    w.y = reinterpret_cast<double2*>(p);
    p += align256(size_t(n) * sizeof(double2));
    w.vn = reinterpret_cast<double2*>(p);
    p += align256(size_t(n) * sizeof(double2));
    w.ys = reinterpret_cast<double2*>(p);
    p += align256(size_t(n) * sizeof(double2));
    w.cn = reinterpret_cast<double2*>(p);
    p += align256(size_t(n) * sizeof(double2));
    w.part = reinterpret_cast<double2*>(p);
    p += align256(size_t(part_slots(n)) * n * sizeof(double2));
    w.d = reinterpret_cast<double*>(p);
    p += align256(size_t(n) * sizeof(double));
    w.e = reinterpret_cast<double*>(p);
    p += align256(size_t(n) * sizeof(double));
    w.sc = reinterpret_cast<double2*>(p);
    return w;
}

}  // namespace
}  // namespace ed

using namespace ed;

extern "C" ed_status ed_entropy_workspace(int L, int l_cut, size_t* bytes) {
    if (!bytes || L < 1 || L > 30 || l_cut < 0 || l_cut > L) return fail(ED_ERR_ARG, "bad argument");
    const int ls = l_cut <= L - l_cut ? l_cut : L - l_cut;
    if (ls > 14) return fail(ED_ERR_UNSUPPORTED, "the smaller side of the cut must have <= 14 sites");
    *bytes = entropy_bytes(1 << ls);
    return ED_OK;
}

extern "C" ed_status ed_entropy(const ed_c64* psi, int L, int d, int l_cut, double* S, double* spectrum,
                                void* ws, size_t ws_bytes, void* stream) {
    if (!psi || !S) return fail(ED_ERR_ARG, "null argument");
    if (d != 2) return fail(ED_ERR_UNSUPPORTED, "only d = 2 is supported");
    size_t need = 0;
    ED_TRY(ed_entropy_workspace(L, l_cut, &need));
    if (!ws) return fail(ED_ERR_ARG, "workspace is null");
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool left_small = l_cut <= L - l_cut;
    const int ls = left_small ? l_cut : L - l_cut;
    const int n = 1 << ls;
    const int64_t K = int64_t(1) << (L - ls);
    EntWS w = carve_ent(ws, n);
    const double2* p = reinterpret_cast<const double2*>(psi);
    // 1. Gram matrix on the matrix cores
    const int nb = (n + kGB - 1) / kGB;
    const int nblocks = nb * (nb + 1) / 2;
    if (left_small) {
        // R = M: row a of M is psi[a*K .. a*K+K)
        hipLaunchKernelGGL((gram_mfma<true>), dim3(nblocks), dim3(256), 0, s, p, K, int64_t(1), n, K, w.rho, nb);
    } else {
        // R = M^T: R[b][a] = psi[a*n + b] with n = 2^(L-l) columns of M
        hipLaunchKernelGGL((gram_mfma<false>), dim3(nblocks), dim3(256), 0, s, p, int64_t(1), int64_t(n), n, K, w.rho, nb);
    }
    ED_HIP_TRY(hipGetLastError());
    // 2. Householder tridiagonalisation
    ED_HIP_TRY(hipMemsetAsync(w.v, 0, size_t(n) * sizeof(double2), s));
    ED_HIP_TRY(hipMemsetAsync(w.y, 0, size_t(n) * sizeof(double2), s));
    ED_HIP_TRY(hipMemsetAsync(w.vn, 0, size_t(n) * sizeof(double2), s));
    ED_HIP_TRY(hipMemsetAsync(w.ys, 0, size_t(n) * sizeof(double2), s));
    if (n > 1) {
        // first Householder vector from column 0
        hipLaunchKernelGGL(hh_step, dim3(1), dim3(kStepThreads), 0, s, w.rho, n, -1, w.v, w.y, w.vn, w.ys, w.d,
                           w.e, w.sc, static_cast<const double2*>(nullptr));
        int nslots = 0;  // partial-sum slots of the current product
        for (int k = 0; k + 1 < n; ++k) {
            // the current vector (rows >= k+1) becomes v; A22 v over rows/cols >= k+1
            std::swap(w.v, w.vn);
            const int s0 = k + 1;
            const int r = n - s0;
            if (k == 0) {
                // nothing updated yet: full-row products of the Gram matrix, column blocks of kFC
                const int ncb = (r + kFC - 1) / kFC;
                const int nrb = (r + kFR - 1) / kFR;
                hipLaunchKernelGGL(hh_gemv, dim3(nrb * ncb), dim3(256), 0, s, w.rho, n, s0, w.v, w.part);
                nslots = ncb;
            }
            hipLaunchKernelGGL(hh_reduce, dim3((r + kRedRows - 1) / kRedRows), dim3(kRedRows * kRedGroups), 0, s, w.part,
                               nslots, s0, n, w.ys);
            // step kernel: y, w, column k+1 update, next Householder vector into vn
            // column k+1 from the previous step's fused update (k >= 1), else from the matrix
            const double2* cin = k >= 1 ? w.cn : nullptr;
            hipLaunchKernelGGL(hh_step, dim3(1), dim3(kStepThreads), 0, s, w.rho, n, k, w.v, w.y, w.vn, w.ys, w.d,
                               w.e, w.sc, cin);
            if (k + 2 < n) {
                // rank-2 update of the lower triangle of rows/cols >= k+2 fused with A_new * vn
                const int s1 = k + 2;
                const int nb = (n - s1 + kSB - 1) / kSB;
                hipLaunchKernelGGL(hh_fused_sym, dim3(nb * (nb + 1) / 2), dim3(256), 0, s, w.rho, n, s1, w.v, w.y,
                                   w.vn, w.part, w.cn);
                nslots = nb;
            }
            ED_HIP_TRY(hipGetLastError());
        }
    }
    // 3. eigenvalues of the tridiagonal matrix by bisection on the GPU (the partial-sum area is
    // free now: n eigenvalues, n squared off-diagonals, 4 bounds), sorted on the host
    std::vector<double> dd(n);
    if (n == 1) {
        // rho is the 1x1 matrix |psi|^2
        double2 r11;
        ED_HIP_TRY(hipMemcpyAsync(&r11, w.rho, sizeof(double2), hipMemcpyDeviceToHost, s));
        ED_HIP_TRY(hipStreamSynchronize(s));
        dd[0] = r11.x;
    } else {
        double* lam = reinterpret_cast<double*>(w.part);
        double* e2 = lam + n;
        double* bnd = e2 + n;
        hipLaunchKernelGGL(tri_bounds, dim3(1), dim3(kBndThreads), 0, s, w.d, w.e, n, e2, bnd);
        hipLaunchKernelGGL(tri_bisect, dim3((n + kBisThreads - 1) / kBisThreads), dim3(kBisThreads), 0, s, w.d, e2, n,
                           bnd, lam);
        ED_HIP_TRY(hipGetLastError());
        ED_HIP_TRY(hipMemcpyAsync(dd.data(), lam, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        ED_HIP_TRY(hipStreamSynchronize(s));
        std::sort(dd.begin(), dd.end());
    }
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += dd[i];
    if (!(tr > 0.0) || !std::isfinite(tr)) return fail(ED_ERR_NUMERIC, "state has zero or non-finite norm");
    double ent = 0.0;
    for (int i = 0; i < n; ++i) {
        const double lam = dd[i] / tr;
        if (lam > 1e-300) ent -= lam * std::log(lam);
    }
    *S = ent;
    if (spectrum)
        for (int i = 0; i < n; ++i) spectrum[i] = dd[n - 1 - i] / tr;  // descending
    return ED_OK;
}
