// Bond (Schmidt) entropy of a pure state (Sec. ed:sec:meas, bond entropy; S(l) of the convergence
// section): rho_l = M M^dagger with M the state reshaped to d^l x d^(L-l), its eigenvalues
// Lambda_j, and S = -sum_j Lambda_j log Lambda_j. The paper computes rho_l by a matrix product
// and takes an eigendecomposition (noting the SVD of M gives the same spectrum).
//
// Here:
//   1. rho = R R^H on the FP64 matrix cores (v_mfma_f64_16x16x4f64), with R = M when
//      d^l <= d^(L-l) and R = M^T otherwise (same non-zero spectrum, smaller Gram matrix);
//      R is read in place from the state, never copied. Only the lower triangle is stored.
//   2. Householder reduction of the Hermitian rho to a real symmetric tridiagonal matrix on the
//      GPU, in blocked form: a read-only matrix-vector sweep of the stored lower triangle per
//      step, the last kPanel rank-2 updates kept pending in a panel and folded into the matrix
//      every kPanel steps by one product on the matrix cores.
//   3. Eigenvalues of the tridiagonal matrix by multisection on Sturm counts on the GPU, 16 lanes
//      per eigenvalue.
// When every amplitude of the state has a zero imaginary part (a real state, such as the ground
// state of a real Hamiltonian started from a real vector), R and rho are real, and so are every
// Householder vector, tau and panel column: steps 1 and 2 then run in real arithmetic (kernels
// templated on T = double instead of T = double2), the same operations without their zero
// imaginary parts.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <utility>
#include <vector>

#include "ed_internal.h"

namespace ed {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------ scalars
// T = double2: a complex entry; T = double: a real one. The helpers give both the same spelling.
template <typename T>
constexpr bool kCx = sizeof(T) == sizeof(double2);

__device__ __forceinline__ double2 mul(double2 a, double2 b) {  // a * b
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double mul(double a, double b) { return a * b; }
__device__ __forceinline__ double2 cj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cj(double a) { return a; }
__device__ __forceinline__ double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double add(double a, double b) { return a + b; }
__device__ __forceinline__ double2 sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double sub(double a, double b) { return a - b; }
__device__ __forceinline__ double2 scale(double2 a, double f) { return make_double2(f * a.x, f * a.y); }
__device__ __forceinline__ double scale(double a, double f) { return f * a; }
__device__ __forceinline__ double re(double2 a) { return a.x; }
__device__ __forceinline__ double re(double a) { return a; }
__device__ __forceinline__ double im(double2 a) { return a.y; }
__device__ __forceinline__ double im(double) { return 0.0; }
__device__ __forceinline__ double abs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double abs2(double a) { return a * a; }
template <typename T>
__device__ __forceinline__ T mk(double r, double i);
template <>
__device__ __forceinline__ double2 mk<double2>(double r, double i) {
    return make_double2(r, i);
}
template <>
__device__ __forceinline__ double mk<double>(double r, double) {
    return r;
}
__device__ __forceinline__ double2 shfl_dn(double2 v, int o) {
    return make_double2(__shfl_down(v.x, o, 64), __shfl_down(v.y, o, 64));
}
__device__ __forceinline__ double shfl_dn(double v, int o) { return __shfl_down(v, o, 64); }
__device__ __forceinline__ double2 shfl_x(double2 v, int o) {
    return make_double2(__shfl_xor(v.x, o, 64), __shfl_xor(v.y, o, 64));
}
__device__ __forceinline__ double shfl_x(double v, int o) { return __shfl_xor(v, o, 64); }

// flag = 1 when some amplitude has a nonzero (or NaN) imaginary part
__global__ __launch_bounds__(256) void imag_any(const double2* __restrict__ psi, int64_t D, int* __restrict__ flag) {
    bool nz = false;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < D; i += int64_t(gridDim.x) * 256)
        nz |= !(psi[i].y == 0.0);
    if (__ballot(nz) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// ------------------------------------------------------------------------------ Gram matrix
// rho[a][a'] = sum_b R[a][b] conj(R[a'][b]), R[r][c] = psi[r*rs + c*cs], n x K.
// Block tile 64 x 64 of rho per workgroup (4 waves, each 32 x 32 = 2 x 2 MFMA tiles), K consumed
// 16 at a time through LDS. Only blocks with I >= J are computed and stored (the Householder
// kernels read the lower triangle only). A complex product takes four real MFMAs, a real one one.
constexpr int kGB = 64;
constexpr int kGK = 16;

template <bool ROWC, typename T>  // ROWC: R's columns are contiguous in memory (cs == 1)
__global__ __launch_bounds__(256) void gram_mfma(const double2* __restrict__ psi, int64_t rs, int64_t cs,
                                                 int n, int64_t K, T* __restrict__ rho) {
    constexpr bool CX = kCx<T>;
    constexpr int kIm = CX ? kGB : 1;  // rows of the imaginary-part tiles (unused when real)
    __shared__ double Ar[kGB][kGK + 1], Br[kGB][kGK + 1], Ai[kIm][kGK + 1], Bi[kIm][kGK + 1];
    // triangular block index -> (I, J), I >= J
    int b = blockIdx.x, I = 0;
    while (b > I) {
        b -= I + 1;
        ++I;
    }
    const int J = b;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
    const double* const psr = reinterpret_cast<const double*>(psi);
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
            const bool kok = k0 + kk < K;
            const bool aok = kok && r0 + rr < n, bok = kok && c0 + rr < n;
            const int64_t ia = int64_t(r0 + rr) * rs + (k0 + kk) * cs, ib = int64_t(c0 + rr) * rs + (k0 + kk) * cs;
            if constexpr (CX) {
                double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
                if (aok) va = psi[ia];
                if (bok) vb = psi[ib];
                Ar[rr][kk] = va.x;
                Ai[rr][kk] = va.y;
                Br[rr][kk] = vb.x;
                Bi[rr][kk] = vb.y;
            } else {
                double va = 0.0, vb = 0.0;
                if (aok) va = psr[2 * ia];  // the real part only
                if (bok) vb = psr[2 * ib];
                Ar[rr][kk] = va;
                Br[rr][kk] = vb;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 4) {
            const int ka = kk + (lane >> 4), ra = lane & 15;
            double ar[2], br[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ar[i] = Ar[wr + 16 * i + ra][ka];
                br[i] = Br[wc + 16 * i + ra][ka];
            }
            if constexpr (CX) {
                double ai[2], bi[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    ai[i] = Ai[wr + 16 * i + ra][ka];
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
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accr[i][j], 0, 0, 0);
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
                if (row < n && col < n) rho[int64_t(row) * n + col] = mk<T>(accr[i][j][q], acci[i][j][q]);
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
// Device state (T entries):
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
// One exchange round of the transposing butterfly per level, H = 8, 4, 2, 1 rows still held per
// lane at lane offsets 4H = 32, 16, 8, 4: a lane keeps the half of its rows selected by that lane
// bit and adds the partner's values of them. After the four rounds lane l holds row (l >> 2) & 15
// summed over its group of 4 lanes. Written as a recursion so that every row index is a constant.
template <int H, typename T>
__device__ __forceinline__ void row_butterfly(T* rp, int lane) {
    if constexpr (H >= 1) {
        constexpr int O = 4 * H;
        const bool up = (lane & O) != 0;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const T keep = up ? rp[q + H] : rp[q];
            const T send = up ? rp[q] : rp[q + H];
            rp[q] = add(keep, shfl_x(send, O));
        }
        row_butterfly<H / 2>(rp, lane);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void hh_sweep(const T* __restrict__ A, int n, int s, const T* __restrict__ v,
                                                T* __restrict__ part, T* __restrict__ cn, const T* __restrict__ P,
                                                int np, int ndot, T* __restrict__ dpart) {
    __shared__ T colred[4][kSB];
    __shared__ T rowred[kSB];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const T zero = mk<T>(0.0, 0.0);
    if (int(blockIdx.x) < ndot) {
        constexpr int kM = kPanel / 4;  // panel columns per wave
        const int g = int(blockIdx.x) >> 1, m0 = kPanel * (int(blockIdx.x) & 1) + kM * wv;
        const int i0 = s + g * kDotRows;
        T acc[kM];
#pragma unroll
        for (int mm = 0; mm < kM; ++mm) acc[mm] = zero;
        for (int q = 0; q < kDotRows / 64; ++q) {
            const int i = i0 + 64 * q + lane;
            if (i >= n) break;
            const T vi = v[i];
#pragma unroll
            for (int mm = 0; mm < kM; ++mm) {
                const int m = m0 + mm;
                if ((m % kPanel) < np)  // uniform over the wave
                    acc[mm] = add(acc[mm], mul(cj(P[int64_t(m) * n + i]), vi));
            }
        }
#pragma unroll
        for (int mm = 0; mm < kM; ++mm) {
            T a = acc[mm];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) a = add(a, shfl_dn(a, off));
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
    T vj = zero;
    if (jok) vj = v[j];
    // the wave's 16 rows, all loads issued before any use
    constexpr int kRW = kSB / 4;
    const int i0 = __builtin_amdgcn_readfirstlane(s + R * kSB + wv * kRW);  // the same on every lane
    T a[kRW];
#pragma unroll
    for (int rr = 0; rr < kRW; ++rr) {
        const int i = i0 + rr;
        a[rr] = zero;
        if (jok && i < n && j <= i) a[rr] = A[int64_t(i) * n + j];
    }
    if (C == 0 && lane == 0) {  // j == s
#pragma unroll
        for (int rr = 0; rr < kRW; ++rr)
            if (i0 + rr < n) cn[i0 + rr] = a[rr];
    }
    // column sums of the strictly lower entries; then a[rr] becomes the row product A_ij v_j
    T colacc = zero;
#pragma unroll
    for (int rr = 0; rr < kRW; ++rr) {
        const int i = i0 + rr;
        if (i < n) {
            const T q = mul(cj(a[rr]), v[i]);
            if (j < i) colacc = add(colacc, q);
        }
        a[rr] = mul(a[rr], vj);
    }
    T* const rp = a;
    // row sums over the 64 lanes, all 16 rows at once (row_butterfly); the exchanges 2 and 1 then
    // complete the sums over each group of 4 lanes
    row_butterfly<kRW / 2>(rp, lane);
#pragma unroll
    for (int o = 2; o >= 1; o >>= 1) rp[0] = add(rp[0], shfl_x(rp[0], o));
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
        T cs = colred[0][lane];
        for (int q = 1; q < 4; ++q) cs = add(cs, colred[q][lane]);
        if (R == C) cs = add(cs, rowred[lane]);
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

template <typename T>
__global__ __launch_bounds__(kRedRows * kRedGroups) void hh_reduce_panel(const T* __restrict__ part, int nslots,
                                                                        int c, int n, T* __restrict__ ys,
                                                                        T* __restrict__ cn, const T* __restrict__ P,
                                                                        int np, const T* __restrict__ dpart,
                                                                        int nchunk) {
    __shared__ T red[kRedGroups][kRedRows];
    __shared__ T redc[kRedGroups][kRedRows];
    __shared__ T dq[4][kPW];  // dot sums over chunks q = 4 u + quarter
    __shared__ T dsum[kPW];   // v_j^H v at j, w_j^H v at kPanel + j
    __shared__ T pc[kPW];     // v_j[c] at j, w_j[c] at kPanel + j
    const int tid = int(threadIdx.x), r = tid % kRedRows, g = tid / kRedRows;
    const T zero = mk<T>(0.0, 0.0);
    if (np > 0) {
        // thread (quarter u, column m) sums chunks u, u + 4, ...; the quarters are then added in order
        const int m = tid % kPW, u = tid / kPW;
        T a = zero;
        if ((m % kPanel) < np) {
#pragma unroll 4
            for (int q = u; q < nchunk; q += 4) a = add(a, dpart[int64_t(q) * kPW + m]);
            if (u == 0) pc[m] = P[int64_t(m) * n + c];
        }
        dq[u][m] = a;
        __syncthreads();
        if (tid < kPW) {
            T t4 = dq[0][tid];
            for (int q = 1; q < 4; ++q) t4 = add(t4, dq[q][tid]);
            dsum[tid] = t4;
        }
        __syncthreads();
    }
    const int i = c + int(blockIdx.x) * kRedRows + r;
    T acc = zero, cc = zero;
    if (i < n) {
#pragma unroll 4
        for (int b = g; b < nslots; b += kRedGroups) acc = add(acc, part[int64_t(b) * n + i]);
#pragma unroll 2
        for (int jj = g; jj < np; jj += kRedGroups) {
            const T vj = P[int64_t(jj) * n + i], wj = P[int64_t(kPanel + jj) * n + i];
            acc = sub(acc, add(mul(vj, dsum[kPanel + jj]), mul(wj, dsum[jj])));
            cc = add(cc, add(mul(vj, cj(pc[kPanel + jj])), mul(wj, cj(pc[jj]))));
        }
    }
    red[g][r] = acc;
    redc[g][r] = cc;
    __syncthreads();
    if (g == 0 && i < n) {
        T sum = red[0][r], csum = redc[0][r];
#pragma unroll
        for (int q = 1; q < kRedGroups; ++q) {
            sum = add(sum, red[q][r]);
            csum = add(csum, redc[q][r]);
        }
        ys[i] = sum;
        if (np > 0) cn[i] = sub(cn[i], csum);
    }
}

// Single-workgroup step kernel (1024 threads). Given ys = A v for the current step k (rows
// k+1..n-1, from hh_reduce_panel) it: forms y = tau (A v); alpha = -1/2 tau (y^H v); w = y + alpha v;
// finishes column k+1 of the trailing matrix (rows k+1..n-1) with the step's own rank-2 term,
// into ys; records d[k+1]; builds the next Householder vector from rows k+2.. of that column,
// with tau, beta. v and w also go to the panel columns pv, pw (rows k+1..). For k = -1 it only
// builds the first Householder vector from column 0.
constexpr int kStepThreads = 1024;

// sum over the workgroup, in a fixed order
template <typename T>
__device__ T block_sum(T v, T* lds) {
    for (int off = 32; off > 0; off >>= 1) v = add(v, shfl_dn(v, off));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    T s = lds[0];
    for (int i = 1; i < kStepThreads / 64; ++i) s = add(s, lds[i]);
    __syncthreads();
    return s;
}

// The reflector that zeroes a column below its first entry al, given nx = the squared norm of the
// rest: beta = -sign(Re al) |column|, tau = (beta - al) / beta, and inv = 1 / (al - beta), the
// scale of the rest of the vector (H = I when the rest is zero and al is real).
template <typename T>
__device__ __forceinline__ void reflector(T al, double nx, T* tau, double* beta, T* inv) {
    *tau = mk<T>(0.0, 0.0);
    *inv = mk<T>(0.0, 0.0);
    if (nx == 0.0 && im(al) == 0.0) {
        *beta = re(al);
        return;
    }
    const double nrm = sqrt(abs2(al) + nx);
    const double b = re(al) >= 0.0 ? -nrm : nrm;
    *beta = b;
    *tau = mk<T>((b - re(al)) / b, -im(al) / b);
    const T den = mk<T>(re(al) - b, im(al));
    const double dd = abs2(den);
    *inv = mk<T>(re(den) / dd, -im(den) / dd);
}

// cin: column k+1 of the trailing matrix before the step's own update, contiguous (rows >= k+1),
// or null to read it from the matrix (k = -1). Every thread keeps the same rows
// i = k+1+t, k+1+t+1024, ... through the passes, so a value it wrote is read back by the same thread.
template <typename T>
__global__ __launch_bounds__(kStepThreads) void hh_step(const T* __restrict__ A, int n, int k, T* __restrict__ v,
                                                        T* __restrict__ y, T* __restrict__ vn, T* __restrict__ ys,
                                                        double* __restrict__ d, double* __restrict__ e,
                                                        T* __restrict__ sc, const T* __restrict__ cin,
                                                        T* __restrict__ pv, T* __restrict__ pw) {
    T* const col = ys;  // column c of the trailing matrix after this step's update
    __shared__ double lds[kStepThreads / 64];
    __shared__ T lds2[kStepThreads / 64];
    __shared__ T syc;
    const int t = threadIdx.x;
    const int c = k + 1;  // column of the trailing matrix to finish now
    double nx = 0.0;      // |column c|^2 over rows c+2..n-1
    if (k >= 0) {
        const T tau = sc[0];
        // y_i = tau * (A v)_i, i = k+1..n-1; also y^H v
        T yhv = mk<T>(0.0, 0.0);
        for (int i = c + t; i < n; i += kStepThreads) {
            const T yi = mul(tau, ys[i]);
            y[i] = yi;
            if (i == c) syc = yi;
            yhv = add(yhv, mul(cj(yi), v[i]));
        }
        yhv = block_sum(yhv, lds2);
        // alpha = -1/2 tau (y^H v); w = y + alpha v
        const T alpha = scale(mul(tau, yhv), -0.5);
        const T vc = v[c];
        const T wc = add(syc, mul(alpha, vc));
        // w, and the update of column c (rows c..n-1): A[i][c] -= v_i conj(w_c) + w_i conj(v_c).
        // Column c is finished by this step (later steps take rows and columns > c), so the
        // updated column goes to col = ys (free once y is formed) instead of back into A
        for (int i = c + t; i < n; i += kStepThreads) {
            const T vi = v[i];
            const T wi = add(y[i], mul(alpha, vi));
            y[i] = wi;
            pv[i] = vi;
            pw[i] = wi;
            const T a = sub(cin[i], add(mul(vi, cj(wc)), mul(wi, cj(vc))));
            col[i] = a;
            if (i >= c + 2) nx += abs2(a);
        }
    } else {
        for (int i = c + t; i < n; i += kStepThreads) {
            const T a = A[int64_t(i) * n + c];
            col[i] = a;
            if (i >= c + 2) nx += abs2(a);
        }
    }
    nx = block_sum(nx, lds);  // its barriers also publish col
    // diagonal of row c and Householder vector of column c below the diagonal (rows c+1..)
    if (t == 0) d[c] = re(col[c]);
    if (c + 1 >= n) return;
    T tau, inv;
    double beta;
    reflector(col[c + 1], nx, &tau, &beta, &inv);
    if (t == 0) {
        e[c] = fabs(beta);
        sc[0] = tau;
        vn[c + 1] = mk<T>(1.0, 0.0);
    }
    for (int i = c + 2 + t; i < n; i += kStepThreads) vn[i] = mul(col[i], inv);
}

// The step kernel for k >= 0 with every row of the column held in registers (thread t owns rows
// c + t + 1024 q, q < RPT, as in hh_step): ys, v and the column are read once, and only the panel
// columns and the next Householder vector are written. Covers n - k - 1 <= 1024 RPT rows.
template <typename T, int RPT>
__global__ __launch_bounds__(kStepThreads) void hh_step_reg(int n, int k, const T* __restrict__ v, T* __restrict__ vn,
                                                            const T* __restrict__ ys, double* __restrict__ d,
                                                            double* __restrict__ e, T* __restrict__ sc,
                                                            const T* __restrict__ cin, T* __restrict__ pv,
                                                            T* __restrict__ pw) {
    __shared__ double lds[kStepThreads / 64];
    __shared__ T lds2[kStepThreads / 64];
    __shared__ T sh_yc, sh_vc, sh_col[2];
    const int t = threadIdx.x;
    const int c = k + 1;
    const T tau = sc[0];
    const T zero = mk<T>(0.0, 0.0);
    T yv[RPT], vv[RPT], cv[RPT];
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
    T yhv = zero;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        yv[q] = mul(tau, yv[q]);
        yhv = add(yhv, mul(cj(yv[q]), vv[q]));
    }
    if (t == 0) {  // row c
        sh_yc = yv[0];
        sh_vc = vv[0];
    }
    yhv = block_sum(yhv, lds2);  // its barriers also publish sh_yc, sh_vc
    const T alpha = scale(mul(tau, yhv), -0.5);
    const T vc = sh_vc;
    const T wc = add(sh_yc, mul(alpha, vc));
    // w = y + alpha v to the panel with v; column c finished with the step's own rank-2 term
    double nx = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = c + t + kStepThreads * q;
        if (i < n) {
            const T wi = add(yv[q], mul(alpha, vv[q]));
            pv[i] = vv[q];
            pw[i] = wi;
            cv[q] = sub(cv[q], add(mul(vv[q], cj(wc)), mul(wi, cj(vc))));
            if (i >= c + 2) nx += abs2(cv[q]);
        }
    }
    if (t < 2) sh_col[t] = cv[0];  // rows c and c + 1
    nx = block_sum(nx, lds);       // its barriers also publish sh_col
    if (t == 0) d[c] = re(sh_col[0]);
    if (c + 1 >= n) return;
    T tau_n, inv;
    double beta;
    reflector(sh_col[1], nx, &tau_n, &beta, &inv);
    if (t == 0) {
        e[c] = fabs(beta);
        sc[0] = tau_n;
        vn[c + 1] = mk<T>(1.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = c + t + kStepThreads * q;
        if (i >= c + 2 && i < n) vn[i] = mul(cv[q], inv);
    }
}
constexpr int kStepRegRows = 8;  // rows per thread of hh_step_reg

// The panel folded into A_s: A_s[i][j] -= sum_m U[i][m] conj(Z[j][m]) for s <= j <= i < n, with
// U = [v_0 .. v_{kPanel-1} | w_0 .. w_{kPanel-1}] and Z = [w | v] (columns swapped by halves), that
// is sum_j (v_j w_j^H + w_j v_j^H) over the np pairs in use. 64 x 64 tiles (I >= J) of the
// trailing block, 4 waves of 2 x 2 FP64 MFMA tiles each (the Gram kernel's layout), the 2 kPanel
// panel columns through LDS 16 at a time.
template <typename T>
__global__ __launch_bounds__(256) void hh_flush(T* __restrict__ A, int n, int s, const T* __restrict__ P, int np) {
    constexpr bool CX = kCx<T>;
    constexpr int kIm = CX ? kGB : 1;
    __shared__ double Ar[kGB][kGK + 1], Br[kGB][kGK + 1], Ai[kIm][kGK + 1], Bi[kIm][kGK + 1];
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
            T va = mk<T>(0.0, 0.0), vb = mk<T>(0.0, 0.0);
            if ((m % kPanel) < np) {
                if (r0 + rr < n) va = P[int64_t(m) * n + r0 + rr];
                if (c0 + rr < n) vb = P[int64_t(mz) * n + c0 + rr];
            }
            Ar[rr][kk] = re(va);
            Br[rr][kk] = re(vb);
            if constexpr (CX) {
                Ai[rr][kk] = im(va);
                Bi[rr][kk] = im(vb);
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 4) {
            const int ka = kk + (lane >> 4), ra = lane & 15;
            double ar[2], br[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ar[i] = Ar[wr + 16 * i + ra][ka];
                br[i] = Br[wc + 16 * i + ra][ka];
            }
            if constexpr (CX) {
                double ai[2], bi[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    ai[i] = Ai[wr + 16 * i + ra][ka];
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
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accr[i][j], 0, 0, 0);
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
                if (row < n && col <= row)
                    A[int64_t(row) * n + col] =
                        sub(A[int64_t(row) * n + col], mk<T>(accr[i][j][q], acci[i][j][q]));
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

// 1/q from the hardware reciprocal and two Newton steps r <- r + r (1 - q r), each of which squares
// the relative error: within an ulp or two of the quotient, at a third of the instructions of a
// correctly rounded division. |q| >= pivmin keeps 1/q finite. (Bisection only needs each count to
// be the exact count of a slightly perturbed T, which a faithful quotient gives; the bracketing
// below keeps count(lo) <= k < count(hi) whatever the counts are.)
__device__ __forceinline__ double recip(double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(r, fma(-q, r, 1.0), r);
    r = fma(r, fma(-q, r, 1.0), r);
    return r;
}

__device__ __forceinline__ int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int n, double x,
                                           double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
#pragma unroll 4
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] * recip(q);
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

// The workspace areas, sized for complex entries; the real path uses the first half of each.
template <typename T>
struct EntWS {
    T* rho;
    T* v;
    T* y;
    T* vn;
    T* ys;
    T* cn;  // the step's column of the trailing matrix, contiguous
    T* part;
    T* dpart;
    T* panel;
    double* d;
    double* e;
    T* sc;
    int* flag;  // imaginary parts seen
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

template <typename T>
EntWS<T> carve_ent(void* ws, int n) {
    char* p = static_cast<char*>(ws);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += align256(bytes);
        return q;
    };
    EntWS<T> w;
    w.rho = reinterpret_cast<T*>(take(size_t(n) * n * sizeof(double2)));
    w.v = reinterpret_cast<T*>(take(size_t(n) * sizeof(double2)));
    w.y = reinterpret_cast<T*>(take(size_t(n) * sizeof(double2)));
    w.vn = reinterpret_cast<T*>(take(size_t(n) * sizeof(double2)));
    w.ys = reinterpret_cast<T*>(take(size_t(n) * sizeof(double2)));
    w.cn = reinterpret_cast<T*>(take(size_t(n) * sizeof(double2)));
    w.part = reinterpret_cast<T*>(take(size_t(part_slots(n)) * n * sizeof(double2)));
    w.dpart = reinterpret_cast<T*>(take(size_t(dot_chunks(n)) * kPW * sizeof(double2)));
    w.panel = reinterpret_cast<T*>(take(size_t(kPW) * n * sizeof(double2)));
    w.d = reinterpret_cast<double*>(take(size_t(n) * sizeof(double)));
    w.e = reinterpret_cast<double*>(take(size_t(n) * sizeof(double)));
    char* sc = take(4 * sizeof(double2));
    w.sc = reinterpret_cast<T*>(sc);  // sc[0] = tau
    w.flag = reinterpret_cast<int*>(sc + 2 * sizeof(double2));
    return w;
}

// Steps 1 and 2 in arithmetic T: the Gram matrix of R (n x K, R = M when left_small, else M^T)
// and its reduction to the tridiagonal (w.d, w.e), all on stream s.
template <typename T>
ed_status gram_tridiagonal(const EntWS<T>& w0, const double2* p, bool left_small, int n, int64_t K, hipStream_t s) {
    EntWS<T> w = w0;
    // 1. Gram matrix on the matrix cores
    const int nb = (n + kGB - 1) / kGB;
    const int nblocks = nb * (nb + 1) / 2;
    if (left_small)  // R = M: row a of M is psi[a*K .. a*K+K)
        hipLaunchKernelGGL((gram_mfma<true, T>), dim3(nblocks), dim3(256), 0, s, p, K, int64_t(1), n, K, w.rho);
    else  // R = M^T: R[b][a] = psi[a*n + b] with n = 2^(L-l) columns of M
        hipLaunchKernelGGL((gram_mfma<false, T>), dim3(nblocks), dim3(256), 0, s, p, int64_t(1), int64_t(n), n, K,
                           w.rho);
    ED_HIP_TRY(hipGetLastError());
    if (n < 2) return ED_OK;
    // 2. Householder tridiagonalisation
    ED_HIP_TRY(hipMemsetAsync(w.v, 0, size_t(n) * sizeof(T), s));
    ED_HIP_TRY(hipMemsetAsync(w.y, 0, size_t(n) * sizeof(T), s));
    ED_HIP_TRY(hipMemsetAsync(w.vn, 0, size_t(n) * sizeof(T), s));
    ED_HIP_TRY(hipMemsetAsync(w.ys, 0, size_t(n) * sizeof(T), s));
    // first Householder vector from column 0
    hipLaunchKernelGGL(hh_step<T>, dim3(1), dim3(kStepThreads), 0, s, static_cast<const T*>(w.rho), n, -1, w.v, w.y,
                       w.vn, w.ys, w.d, w.e, w.sc, static_cast<const T*>(nullptr), static_cast<T*>(nullptr),
                       static_cast<T*>(nullptr));
    int np = 0;  // pending pairs in the panel
    for (int k = 0; k + 1 < n; ++k) {
        // the current vector (rows >= k+1) becomes v; the trailing block is rows/cols >= k+1
        std::swap(w.v, w.vn);
        const int s0 = k + 1;
        const int r = n - s0;
        const int nbs = (r + kSB - 1) / kSB;
        const int nchunk = np > 0 ? (r + kDotRows - 1) / kDotRows : 0;
        const int ndot = 2 * nchunk;
        T* const pv = w.panel + size_t(np) * n;
        T* const pw = w.panel + size_t(kPanel + np) * n;
        // A_s v (read-only sweep of the lower triangle), column k+1 of A_s, panel dots
        hipLaunchKernelGGL(hh_sweep<T>, dim3(ndot + nbs * (nbs + 1) / 2), dim3(256), 0, s,
                           static_cast<const T*>(w.rho), n, s0, static_cast<const T*>(w.v), w.part, w.cn,
                           static_cast<const T*>(w.panel), np, ndot, w.dpart);
        // A v and column k+1 of the trailing matrix, with the panel's share
        hipLaunchKernelGGL(hh_reduce_panel<T>, dim3((r + kRedRows - 1) / kRedRows), dim3(kRedRows * kRedGroups), 0, s,
                           static_cast<const T*>(w.part), nbs, s0, n, w.ys, w.cn, static_cast<const T*>(w.panel), np,
                           static_cast<const T*>(w.dpart), nchunk);
        // step kernel: y, w, column k+1 finished, next Householder vector into vn; (v, w) to the panel
        if (r <= kStepThreads * kStepRegRows)
            hipLaunchKernelGGL((hh_step_reg<T, kStepRegRows>), dim3(1), dim3(kStepThreads), 0, s, n, k,
                               static_cast<const T*>(w.v), w.vn, static_cast<const T*>(w.ys), w.d, w.e, w.sc,
                               static_cast<const T*>(w.cn), pv, pw);
        else
            hipLaunchKernelGGL(hh_step<T>, dim3(1), dim3(kStepThreads), 0, s, static_cast<const T*>(w.rho), n, k, w.v,
                               w.y, w.vn, w.ys, w.d, w.e, w.sc, static_cast<const T*>(w.cn), pv, pw);
        ++np;
        if (np == kPanel && k + 2 < n) {
            // fold the panel into the lower triangle of rows/cols >= k+2
            const int nbf = (n - (k + 2) + kGB - 1) / kGB;
            hipLaunchKernelGGL(hh_flush<T>, dim3(nbf * (nbf + 1) / 2), dim3(256), 0, s, w.rho, n, k + 2,
                               static_cast<const T*>(w.panel), np);
            np = 0;
        }
        ED_HIP_TRY(hipGetLastError());
    }
    return ED_OK;
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

namespace {
ed_status entropy_impl(const ed_c64* psi, int L, int d, int l_cut, double* S, double* spectrum, int* real_arith,
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
    const int64_t D = int64_t(1) << L;
    const double2* p = reinterpret_cast<const double2*>(psi);
    // real or complex arithmetic: does any amplitude have a nonzero imaginary part?
    const EntWS<double2> wc = carve_ent<double2>(ws, n);
    ED_HIP_TRY(hipMemsetAsync(wc.flag, 0, sizeof(int), s));
    hipLaunchKernelGGL(imag_any, dim3(unsigned(std::min<int64_t>((D + 255) / 256, 2048))), dim3(256), 0, s, p, D,
                       wc.flag);
    ED_HIP_TRY(hipGetLastError());
    int cx = 1;
    ED_HIP_TRY(hipMemcpyAsync(&cx, wc.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ED_HIP_TRY(hipStreamSynchronize(s));
    const bool real = cx == 0;
    if (real_arith) *real_arith = real ? 1 : 0;
    const EntWS<double> wr = carve_ent<double>(ws, n);
    if (real) ED_TRY(gram_tridiagonal<double>(wr, p, left_small, n, K, s));
    else ED_TRY(gram_tridiagonal<double2>(wc, p, left_small, n, K, s));
    // 3. eigenvalues of the tridiagonal matrix by bisection on the GPU (the partial-sum area is
    // free now: n eigenvalues, n squared off-diagonals, 4 bounds), sorted on the host
    std::vector<double> dd(n);
    if (n == 1) {
        // rho is the 1x1 matrix |psi|^2, its real part first in either arithmetic
        ED_HIP_TRY(hipMemcpyAsync(dd.data(), wr.rho, sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP_TRY(hipStreamSynchronize(s));
    } else {
        double* lam = wr.part;
        double* e2 = lam + n;
        double* bnd = e2 + n;
        hipLaunchKernelGGL(tri_bounds, dim3(1), dim3(kBndThreads), 0, s, wr.d, wr.e, n, e2, bnd);
        hipLaunchKernelGGL(tri_bisect, dim3((n * kMS + kBisThreads - 1) / kBisThreads), dim3(kBisThreads), 0, s, wr.d,
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
}  // namespace

extern "C" ed_status ed_entropy(const ed_c64* psi, int L, int d, int l_cut, double* S, double* spectrum, void* ws,
                                size_t ws_bytes, void* stream) {
    return entropy_impl(psi, L, d, l_cut, S, spectrum, nullptr, ws, ws_bytes, stream);
}

extern "C" ed_status ed_entropy_ex(const ed_c64* psi, int L, int d, int l_cut, double* S, double* spectrum,
                                   int* real_arith, void* ws, size_t ws_bytes, void* stream) {
    return entropy_impl(psi, L, d, l_cut, S, spectrum, real_arith, ws, ws_bytes, stream);
}
