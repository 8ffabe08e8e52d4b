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
//   3. Eigenvalues of the tridiagonal matrix by multisection on Sturm counts on the GPU, 16 lanes
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
// Reduction of the Hermitian rho to a real symmetric tridiagonal matrix by n - 2 Householder
// steps. Step k takes the reflector I - tau v v^H (v_{k+1} = 1) that zeroes column k below row
// k + 1, forms y = tau A v, w = y - 1/2 tau (y^H v) v, and the rank-2 update
// A <- A - v w^H - w v^H of the trailing block (rows and columns > k).
//
// The updates are applied lazily, as in the blocked form of the reduction: the last np <= kPanel
// pairs (v_j, w_j) stay in a panel P (column j holds v_j, column kPanel + j holds w_j), and the
// trailing matrix is A_s - sum_j (v_j w_j^H + w_j v_j^H), with A_s the stored matrix (lower
// triangle kept). A step reads A_s once (hh_sweep: the product A_s v, read-only) and corrects
// that product and the column it finishes with the panel (hh_reduce_panel). Every kPanel steps
// the panel is folded into A_s by one rank-2 kPanel update on the matrix cores (hh_flush). The
// trailing matrix thus streams once per step instead of being read and written.
//
// Device state:
//   v[n]   the step's Householder vector (rows >= k+1); vn the next one
//   y[n]   tau A v, then w (rows >= k+1)
//   ys[n]  the product A v (rows >= k+1), then the finished column
//   cn[n]  column k+1 of the trailing matrix (rows >= k+1)
//   part[slots][n]  partial row sums of the sweep; dpart[chunks][2 kPanel] partial panel dots
//   P[2 kPanel][n]  the panel
//   d[n], e[n]  tridiagonal diagonal / |sub-diagonal|;  sc[0] = tau
constexpr int kSB = 64;          // tile edge of the sweep and of the flush
constexpr int kPanel = 32;       // pending rank-2 updates before a flush
constexpr int kPW = 2 * kPanel;  // panel columns
constexpr int kDotRows = 256;    // rows per panel-dot workgroup of the sweep

__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * b
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// Workgroups 0..ndot-1 (only when np > 0; two per chunk of kDotRows rows from s, one per half of
// the panel columns): dpart[chunk][m] = the sum over the chunk's rows i of conj(P_m[i]) v[i], for
// the panel columns m in use (m mod kPanel < np); wave w of half h takes columns
// kPanel h + 8 w .. kPanel h + 8 w + 7, its lanes consecutive rows.
// Workgroups ndot..: one 64 x 64 tile (R, C), C <= R, of the lower triangle of A_s over [s, n).
// The row sums of A_s v over its rows go to slot C, the conjugate column sums of its strictly
// lower entries (y_j += conj(A_ij) v_i) to slot R; a diagonal tile sends both to slot R. Row i of
// block B so gets slot b from tile (B, b) for b < B, (B, B) for b = B and (b, B) for b > B: every
// slot exactly once, summed in a fixed order by hh_reduce_panel. The tiles (R, 0) also copy
// column s of A_s to cn (rows >= s).
__global__ __launch_bounds__(256) void hh_sweep(const double2* __restrict__ A, int n, int s,
                                                const double2* __restrict__ v, double2* __restrict__ part,
                                                double2* __restrict__ cn, const double2* __restrict__ P, int np,
                                                int ndot, double2* __restrict__ dpart) {
    __shared__ double2 colred[4][kSB];
    __shared__ double2 rowred[kSB];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const double2 zero = make_double2(0.0, 0.0);
    if (int(blockIdx.x) < ndot) {
        constexpr int kM = kPanel / 4;  // panel columns per wave
        const int g = int(blockIdx.x) >> 1, m0 = kPanel * (int(blockIdx.x) & 1) + kM * wv;
        const int i0 = s + g * kDotRows;
        double2 acc[kM];
#pragma unroll
        for (int mm = 0; mm < kM; ++mm) acc[mm] = zero;
        for (int q = 0; q < kDotRows / 64; ++q) {
            const int i = i0 + 64 * q + lane;
            if (i >= n) break;
            const double2 vi = v[i];
#pragma unroll
            for (int mm = 0; mm < kM; ++mm) {
                const int m = m0 + mm;
                if ((m % kPanel) < np) {  // uniform over the wave
                    const double2 a = P[int64_t(m) * n + i];
                    acc[mm].x += a.x * vi.x + a.y * vi.y;
                    acc[mm].y += a.x * vi.y - a.y * vi.x;
                }
            }
        }
#pragma unroll
        for (int mm = 0; mm < kM; ++mm) {
            double2 a = acc[mm];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                a.x += __shfl_down(a.x, off, 64);
                a.y += __shfl_down(a.y, off, 64);
            }
            if (lane == 0) dpart[int64_t(g) * kPW + m0 + mm] = a;
        }
        return;
    }
    int b = int(blockIdx.x) - ndot, R = 0;
    while (b > R) {
        b -= R + 1;
        ++R;
    }
    const int C = b;
    const int j = s + C * kSB + lane;
    const bool jok = j < n;
    double2 vj = make_double2(0.0, 0.0);
    if (jok) vj = v[j];
    // the wave's 16 rows, all loads issued before any use
    constexpr int kRW = kSB / 4;
    const int i0 = __builtin_amdgcn_readfirstlane(s + R * kSB + wv * kRW);  // the same on every lane
    double2 a[kRW];
#pragma unroll
    for (int rr = 0; rr < kRW; ++rr) {
        const int i = i0 + rr;
        a[rr] = make_double2(0.0, 0.0);
        if (jok && i < n && j <= i) a[rr] = A[int64_t(i) * n + j];
    }
    if (C == 0 && lane == 0) {  // j == s
#pragma unroll
        for (int rr = 0; rr < kRW; ++rr)
            if (i0 + rr < n) cn[i0 + rr] = a[rr];
    }
    // column sums of the strictly lower entries; then a[rr] becomes the row product A_ij v_j
    double2 colacc = zero;
#pragma unroll
    for (int rr = 0; rr < kRW; ++rr) {
        const int i = i0 + rr;
        if (i < n) {
            const double2 q = cmulc(conjd(a[rr]), v[i]);
            if (j < i) {
                colacc.x += q.x;
                colacc.y += q.y;
            }
        }
        a[rr] = cmulc(a[rr], vj);
    }
    double2* const rp = a;
    // row sums over the 64 lanes, all 16 rows at once: at each of the exchanges 32, 16, 8, 4 a lane
    // keeps the half of its rows selected by that lane bit and adds the partner's values of them;
    // after 4 exchanges lane l holds row (l >> 2) & 15 summed over its group of 4 lanes, which the
    // exchanges 2 and 1 complete
#pragma unroll
    for (int h = kRW / 2, o = 32; h >= 1; h >>= 1, o >>= 1) {
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int q = 0; q < h; ++q) {
            const double2 keep = up ? rp[q + h] : rp[q];
            const double2 send = up ? rp[q] : rp[q + h];
            rp[q].x = keep.x + __shfl_xor(send.x, o, 64);
            rp[q].y = keep.y + __shfl_xor(send.y, o, 64);
        }
    }
#pragma unroll
    for (int o = 2; o >= 1; o >>= 1) {
        rp[0].x += __shfl_xor(rp[0].x, o, 64);
        rp[0].y += __shfl_xor(rp[0].y, o, 64);
    }
    if ((lane & 3) == 0) {
        const int li = wv * kRW + (lane >> 2);
        const int i = s + R * kSB + li;
        if (i < n) {
            if (R == C) rowred[li] = rp[0];
            else part[int64_t(C) * n + i] = rp[0];
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

// For rows i in [c, n), 32 per workgroup: ys[i] = the sum of the nslots partial sums of row i
// minus the panel's share of the product, sum_j v_j[i] (w_j^H v) + w_j[i] (v_j^H v); and column c
// of A_s in cn becomes column c of the trailing matrix: cn[i] -= sum_j v_j[i] conj(w_j[c]) +
// w_j[i] conj(v_j[c]). The panel dots are the sums over the sweep's nchunk row chunks. The 8 groups of 32
// threads take slots g, g + 8, ... and panel pairs g, g + 8, ...; their sums are added in group
// order (a fixed order, so results are reproducible).
constexpr int kRedRows = 32, kRedGroups = 8;

__global__ __launch_bounds__(kRedRows * kRedGroups) void hh_reduce_panel(
    const double2* __restrict__ part, int nslots, int c, int n, double2* __restrict__ ys, double2* __restrict__ cn,
    const double2* __restrict__ P, int np, const double2* __restrict__ dpart, int nchunk) {
    __shared__ double2 red[kRedGroups][kRedRows];
    __shared__ double2 redc[kRedGroups][kRedRows];
    __shared__ double2 dq[4][kPW];  // dot sums over chunks q = 4 u + quarter
    __shared__ double2 dsum[kPW];   // v_j^H v at j, w_j^H v at kPanel + j
    __shared__ double2 pc[kPW];     // v_j[c] at j, w_j[c] at kPanel + j
    const int tid = int(threadIdx.x), r = tid % kRedRows, g = tid / kRedRows;
    if (np > 0) {
        // thread (quarter u, column m) sums chunks u, u + 4, ...; the quarters are then added in order
        const int m = tid % kPW, u = tid / kPW;
        double2 a = make_double2(0.0, 0.0);
        if ((m % kPanel) < np) {
#pragma unroll 4
            for (int q = u; q < nchunk; q += 4) {
                const double2 p = dpart[int64_t(q) * kPW + m];
                a.x += p.x;
                a.y += p.y;
            }
            if (u == 0) pc[m] = P[int64_t(m) * n + c];
        }
        dq[u][m] = a;
        __syncthreads();
        if (tid < kPW) {
            double2 t4 = dq[0][tid];
            for (int q = 1; q < 4; ++q) {
                t4.x += dq[q][tid].x;
                t4.y += dq[q][tid].y;
            }
            dsum[tid] = t4;
        }
        __syncthreads();
    }
    const int i = c + int(blockIdx.x) * kRedRows + r;
    double2 acc = make_double2(0.0, 0.0), cc = make_double2(0.0, 0.0);
    if (i < n) {
#pragma unroll 4
        for (int b = g; b < nslots; b += kRedGroups) {
            const double2 p = part[int64_t(b) * n + i];
            acc.x += p.x;
            acc.y += p.y;
        }
#pragma unroll 2
        for (int jj = g; jj < np; jj += kRedGroups) {
            const double2 vj = P[int64_t(jj) * n + i], wj = P[int64_t(kPanel + jj) * n + i];
            const double2 a1 = cmulc(vj, dsum[kPanel + jj]), a2 = cmulc(wj, dsum[jj]);
            acc.x -= a1.x + a2.x;
            acc.y -= a1.y + a2.y;
            const double2 c1 = cmulc(vj, conjd(pc[kPanel + jj])), c2 = cmulc(wj, conjd(pc[jj]));
            cc.x += c1.x + c2.x;
            cc.y += c1.y + c2.y;
        }
    }
    red[g][r] = acc;
    redc[g][r] = cc;
    __syncthreads();
    if (g == 0 && i < n) {
        double2 sum = red[0][r], csum = redc[0][r];
#pragma unroll
        for (int q = 1; q < kRedGroups; ++q) {
            sum.x += red[q][r].x;
            sum.y += red[q][r].y;
            csum.x += redc[q][r].x;
            csum.y += redc[q][r].y;
        }
        ys[i] = sum;
        if (np > 0) {
            double2 a = cn[i];
            a.x -= csum.x;
            a.y -= csum.y;
            cn[i] = a;
        }
    }
}

// Single-workgroup step kernel (1024 threads). Given ys = A v for the current step k (rows
// k+1..n-1, from hh_reduce_panel) it: forms y = tau (A v); alpha = -1/2 tau (y^H v); w = y + alpha v;
// finishes column k+1 of the trailing matrix (rows k+1..n-1) with the step's own rank-2 term,
// into ys; records d[k+1]; builds the next Householder vector from rows k+2.. of that column,
// with tau, beta. v and w also go to the panel columns pv, pw (rows k+1..). For k = -1 it only
// builds the first Householder vector from column 0.
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

// cin: column k+1 of the trailing matrix before the step's own update, contiguous (rows >= k+1),
// or null to read it from the matrix (k = -1). Every thread keeps the same rows
// i = k+1+t, k+1+t+1024, ... through the passes, so a value it wrote is read back by the same thread.
__global__ __launch_bounds__(kStepThreads) void hh_step(const double2* __restrict__ A, int n, int k,
                                                        double2* __restrict__ v, double2* __restrict__ y,
                                                        double2* __restrict__ vn, double2* __restrict__ ys,
                                                        double* __restrict__ d, double* __restrict__ e,
                                                        double2* __restrict__ sc, const double2* __restrict__ cin,
                                                        double2* __restrict__ pv, double2* __restrict__ pw) {
    double2* const col = ys;  // column c of the trailing matrix after this step's update
    __shared__ double lds[kStepThreads / 64];
    __shared__ double2 lds2[kStepThreads / 64];
    __shared__ double2 syc;
    const int t = threadIdx.x;
    const int c = k + 1;  // column of the trailing matrix to finish now
    double nx = 0.0;      // |column c|^2 over rows c+2..n-1
    if (k >= 0) {
        const double2 tau = sc[0];
        // y_i = tau * (A v)_i, i = k+1..n-1; also y^H v
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
            pv[i] = vi;
            pw[i] = wi;
            double2 a = cin[i];
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

// The step kernel for k >= 0 with every row of the column held in registers (thread t owns rows
// c + t + 1024 q, q < RPT, as in hh_step): ys, v and the column are read once, and only the panel
// columns and the next Householder vector are written. Covers n - k - 1 <= 1024 RPT rows.
template <int RPT>
__global__ __launch_bounds__(kStepThreads) void hh_step_reg(int n, int k, const double2* __restrict__ v,
                                                            double2* __restrict__ vn, const double2* __restrict__ ys,
                                                            double* __restrict__ d, double* __restrict__ e,
                                                            double2* __restrict__ sc, const double2* __restrict__ cin,
                                                            double2* __restrict__ pv, double2* __restrict__ pw) {
    __shared__ double lds[kStepThreads / 64];
    __shared__ double2 lds2[kStepThreads / 64];
    __shared__ double2 sh_yc, sh_vc, sh_col[2];
    const int t = threadIdx.x;
    const int c = k + 1;
    const double2 tau = sc[0];
    const double2 zero = make_double2(0.0, 0.0);
    double2 yv[RPT], vv[RPT], cv[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = c + t + kStepThreads * q;
        yv[q] = zero;
        vv[q] = zero;
        cv[q] = zero;
        if (i < n) {
            yv[q] = ys[i];
            vv[q] = v[i];
            cv[q] = cin[i];
        }
    }
    // y = tau (A v) and y^H v
    double2 yhv = zero;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        yv[q] = cmulc(tau, yv[q]);
        yhv.x += yv[q].x * vv[q].x + yv[q].y * vv[q].y;
        yhv.y += yv[q].x * vv[q].y - yv[q].y * vv[q].x;
    }
    if (t == 0) {  // row c
        sh_yc = yv[0];
        sh_vc = vv[0];
    }
    yhv = block_reduce2(yhv, lds2);  // its barriers also publish sh_yc, sh_vc
    const double2 tt = cmulc(tau, yhv);
    const double2 alpha = make_double2(-0.5 * tt.x, -0.5 * tt.y);
    const double2 vc = sh_vc, avc = cmulc(alpha, vc);
    const double2 wc = make_double2(sh_yc.x + avc.x, sh_yc.y + avc.y);
    // w = y + alpha v to the panel with v; column c finished with the step's own rank-2 term
    double nx = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = c + t + kStepThreads * q;
        if (i < n) {
            const double2 av = cmulc(alpha, vv[q]);
            const double2 wi = make_double2(yv[q].x + av.x, yv[q].y + av.y);
            pv[i] = vv[q];
            pw[i] = wi;
            const double2 t1 = cmulc(vv[q], conjd(wc)), t2 = cmulc(wi, conjd(vc));
            cv[q].x -= t1.x + t2.x;
            cv[q].y -= t1.y + t2.y;
            if (i >= c + 2) nx += cv[q].x * cv[q].x + cv[q].y * cv[q].y;
        }
    }
    if (t < 2) sh_col[t] = cv[0];  // rows c and c + 1
    nx = block_reduce(nx, lds);    // its barriers also publish sh_col
    if (t == 0) d[c] = sh_col[0].x;
    if (c + 1 >= n) return;
    const double2 al = sh_col[1];
    double2 tau_n = zero;
    double beta;
    double2 inv = zero;
    if (nx == 0.0 && al.y == 0.0) {
        beta = al.x;  // H = I
    } else {
        const double nrm = sqrt(al.x * al.x + al.y * al.y + nx);
        beta = al.x >= 0.0 ? -nrm : nrm;
        tau_n = make_double2((beta - al.x) / beta, -al.y / beta);
        const double2 den = make_double2(al.x - beta, al.y);
        const double dd = den.x * den.x + den.y * den.y;
        inv = make_double2(den.x / dd, -den.y / dd);
    }
    if (t == 0) {
        e[c] = fabs(beta);
        sc[0] = tau_n;
        vn[c + 1] = make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = c + t + kStepThreads * q;
        if (i >= c + 2 && i < n) vn[i] = cmulc(cv[q], inv);
    }
}
constexpr int kStepRegRows = 8;  // rows per thread of hh_step_reg

// The panel folded into A_s: A_s[i][j] -= sum_m U[i][m] conj(Z[j][m]) for s <= j <= i < n, with
// U = [v_0 .. v_{kPanel-1} | w_0 .. w_{kPanel-1}] and Z = [w | v] (columns swapped by halves), that
// is sum_j (v_j w_j^H + w_j v_j^H) over the np pairs in use. 64 x 64 tiles (I >= J) of the
// trailing block, 4 waves of 2 x 2 FP64 MFMA tiles each (the Gram kernel's layout), the 2 kPanel
// panel columns through LDS 16 at a time.
__global__ __launch_bounds__(256) void hh_flush(double2* __restrict__ A, int n, int s, const double2* __restrict__ P,
                                                int np) {
    __shared__ double Ar[kGB][kGK + 1], Ai[kGB][kGK + 1], Br[kGB][kGK + 1], Bi[kGB][kGK + 1];
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
    const int r0 = s + I * kGB, c0 = s + J * kGB;
    for (int k0 = 0; k0 < kPW; k0 += kGK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = t + 256 * e;
            const int rr = idx % kGB, kk = idx / kGB;
            const int m = k0 + kk;
            const int mz = (m + kPanel) % kPW;
            double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
            if ((m % kPanel) < np) {
                if (r0 + rr < n) va = P[int64_t(m) * n + r0 + rr];
                if (c0 + rr < n) vb = P[int64_t(mz) * n + c0 + rr];
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
                if (row < n && col <= row) {
                    double2 a = A[int64_t(row) * n + col];
                    a.x -= accr[i][j][q];
                    a.y -= acci[i][j][q];
                    A[int64_t(row) * n + col] = a;
                }
            }
}

// ------------------------------------------------------------------------------ tridiagonal eigenvalues
// Every eigenvalue of the real symmetric tridiagonal T (diagonal d, off-diagonal e >= 0) by
// bisection on Sturm counts: the pivots of the LDL^T factorisation of T - x I have as many
// negative entries as T has eigenvalues below x (Sylvester's law of inertia), and the pivots
// obey q_0 = d_0 - x, q_i = d_i - x - e_{i-1}^2 / q_{i-1}. A pivot smaller in magnitude than
// pivmin is replaced by -pivmin (a perturbation of T of at most pivmin per entry), so no pivot
// is zero. A group of kMS lanes finds the k-th smallest eigenvalue on its own, from the
// Gershgorin interval down to a width of eps |T|, by multisection: each round the lanes count at
// kMS equally spaced interior points and the interval shrinks to the gap where the count first
// exceeds k (log2(kMS + 1) bits per round instead of one). The result depends on d, e and k only.
constexpr int kBisThreads = 256;
constexpr int kMS = 16;  // lanes per eigenvalue
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

// lam[k] = the k-th smallest eigenvalue, k < n; group k of kMS lanes. Invariant: count(lo) <= k <
// count(hi). Every lane of a group computes the same lo, hi and step, so the points are shared
// exactly: point l is lo + (l + 1) h, and the new bounds are points of the round.
__global__ __launch_bounds__(kBisThreads) void tri_bisect(const double* __restrict__ d, const double* __restrict__ e2,
                                                          int n, const double* __restrict__ bnd, double* __restrict__ lam) {
    const int gid = int(blockIdx.x) * kBisThreads + int(threadIdx.x);
    const int k0 = gid / kMS, l = gid % kMS;
    const int k = k0 < n ? k0 : n - 1;  // surplus lanes repeat the last eigenvalue and write nothing
    const int g0 = (int(threadIdx.x) & 63) & ~(kMS - 1);  // the group's first lane in the wave
    double lo = bnd[0], hi = bnd[1];
    const double pivmin = bnd[2], tol = bnd[3];
    for (int it = 0; it < 200 && hi - lo > tol; ++it) {
        const double h = (hi - lo) / (kMS + 1);
        const double x = lo + (l + 1) * h;
        const unsigned long long above = __ballot(sturm_count(d, e2, n, x, pivmin) > k);
        const unsigned gm = unsigned(above >> g0) & ((1u << kMS) - 1);
        const int f = gm ? __builtin_ctz(gm) : kMS;  // first point whose count exceeds k
        const double nlo = f == 0 ? lo : lo + f * h;
        const double nhi = f == kMS ? hi : lo + (f + 1) * h;
        if (!(nlo > lo || nhi < hi)) break;  // no point strictly inside: the interval cannot shrink
        lo = nlo;
        hi = nhi;
    }
    if (k0 < n && l == 0) lam[k0] = lo + 0.5 * (hi - lo);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct EntWS {
    double2* rho;
    double2* v;
    double2* y;
    double2* vn;
    double2* ys;
    double2* cn;  // the step's column of the trailing matrix, contiguous
    double2* part;
    double2* dpart;
    double2* panel;
    double* d;
    double* e;
    double2* sc;
};

// partial-sum slots of the sweep (its block count), at least 2 (the bisection reuses the area for
// 2n + 4 doubles)
int part_slots(int n) { return (n + kSB - 1) / kSB + 1; }
int dot_chunks(int n) { return (n + kDotRows - 1) / kDotRows; }

size_t entropy_bytes(int n) {
    return align256(size_t(n) * n * sizeof(double2)) + 5 * align256(size_t(n) * sizeof(double2)) +
           align256(size_t(part_slots(n)) * n * sizeof(double2)) +
           align256(size_t(dot_chunks(n)) * kPW * sizeof(double2)) + align256(size_t(kPW) * n * sizeof(double2)) +
           2 * align256(size_t(n) * sizeof(double)) + align256(4 * sizeof(double2));
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
    w.dpart = reinterpret_cast<double2*>(p);
    p += align256(size_t(dot_chunks(n)) * kPW * sizeof(double2));
    w.panel = reinterpret_cast<double2*>(p);
    p += align256(size_t(kPW) * n * sizeof(double2));
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
                           w.e, w.sc, static_cast<const double2*>(nullptr), static_cast<double2*>(nullptr),
                           static_cast<double2*>(nullptr));
        int np = 0;  // pending pairs in the panel
        for (int k = 0; k + 1 < n; ++k) {
            // the current vector (rows >= k+1) becomes v; the trailing block is rows/cols >= k+1
            std::swap(w.v, w.vn);
            const int s0 = k + 1;
            const int r = n - s0;
            const int nbs = (r + kSB - 1) / kSB;
            const int nchunk = np > 0 ? (r + kDotRows - 1) / kDotRows : 0;
            const int ndot = 2 * nchunk;
            // A_s v (read-only sweep of the lower triangle), column k+1 of A_s, panel dots
            hipLaunchKernelGGL(hh_sweep, dim3(ndot + nbs * (nbs + 1) / 2), dim3(256), 0, s, w.rho, n, s0, w.v, w.part,
                               w.cn, w.panel, np, ndot, w.dpart);
            // A v and column k+1 of the trailing matrix, with the panel's share
            hipLaunchKernelGGL(hh_reduce_panel, dim3((r + kRedRows - 1) / kRedRows), dim3(kRedRows * kRedGroups), 0, s,
                               w.part, nbs, s0, n, w.ys, w.cn, w.panel, np, w.dpart, nchunk);
            // step kernel: y, w, column k+1 finished, next Householder vector into vn; (v, w) to the panel
            if (r <= kStepThreads * kStepRegRows)
                hipLaunchKernelGGL(hh_step_reg<kStepRegRows>, dim3(1), dim3(kStepThreads), 0, s, n, k,
                                   static_cast<const double2*>(w.v), w.vn, static_cast<const double2*>(w.ys), w.d, w.e,
                                   w.sc, static_cast<const double2*>(w.cn), w.panel + size_t(np) * n,
                                   w.panel + size_t(kPanel + np) * n);
            else
                hipLaunchKernelGGL(hh_step, dim3(1), dim3(kStepThreads), 0, s, w.rho, n, k, w.v, w.y, w.vn, w.ys,
                                   w.d, w.e, w.sc, static_cast<const double2*>(w.cn), w.panel + size_t(np) * n,
                                   w.panel + size_t(kPanel + np) * n);
            ++np;
            if (np == kPanel && k + 2 < n) {
                // fold the panel into the lower triangle of rows/cols >= k+2
                const int nbf = (n - (k + 2) + kGB - 1) / kGB;
                hipLaunchKernelGGL(hh_flush, dim3(nbf * (nbf + 1) / 2), dim3(256), 0, s, w.rho, n, k + 2, w.panel, np);
                np = 0;
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
        hipLaunchKernelGGL(tri_bisect, dim3((n * kMS + kBisThreads - 1) / kBisThreads), dim3(kBisThreads), 0, s, w.d,
                           e2, n, bnd, lam);
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
