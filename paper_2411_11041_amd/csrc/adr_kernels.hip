// gfx950 kernels of the directional diffusion splitting sweep (eq. (10)).
//
//  k_line     one workgroup (256 threads) per curve: gathers the grid field at
//             the curve's nodes (bilinear, eq. (21)-(23)), assembles the P1
//             rows of eq. (16)-(19) in LDS and solves the tridiagonal system
//             by a partitioned elimination: every thread eliminates a
//             contiguous chunk of rows, the chunk separators form a reduced
//             tridiagonal system that is solved by parallel cyclic reduction
//             in LDS, then every thread back-substitutes its chunk.
//  k_scatter  one thread per interior grid node: the crossing-record
//             interpolation of Sec. 6, a fixed 4-record stencil per node.
//  k_norm     per-instance FP64 reduction of the update norm (fixed order).
//
// All kernels early-exit for instances whose done flag is set, so a batch
// of instances shares every launch.
#include <hip/hip_runtime.h>

#include "adr_kernels.h"

namespace adr {

constexpr int kThreads = 256;

// LDS of a line-solve workgroup of nt threads: arrays of `stride` elements (the
// longest curve of the launch, at least the 6 nt entries of the reduced system)
__host__ __device__ inline int line_lds_stride(int nmax, int nt = kThreads) {
    return ((nmax > 6 * nt ? nmax : 6 * nt) + 3) & ~3;
}
__host__ __device__ inline int line_lds_arrays(int fam) { return fam == 0 ? 3 : 2; }

// 1/x: IEEE division in FP64 (parity with the FP64 oracle), the hardware
// reciprocal (v_rcp_f32, ~1 ulp) in the FP32 increment sweeps
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Workgroups are dispatched to the 8 XCDs in turn (workgroup w to XCD w mod 8,
// as its (w div 8)-th).  The bucketed launches deal the list to them in chunks
// of kXcdChunk positions: chunk c goes to XCD c mod 8, so the curves one XCD
// solves at a time are neighbours (their gathers share its L2) and every XCD
// gets a share of the whole list.  List position of workgroup w, or -1 past
// the end of a list of G (the grid is line_grid(G), a whole number of rounds).
__device__ inline int xcd_position(int w, int G) {
    const int x = w & 7, i = w >> 3;
    const int p = ((i / kXcdChunk) * 8 + x) * kXcdChunk + i % kXcdChunk;
    return p < G ? p : -1;
}
inline int line_grid(int G) {
    const int chunks = (G + kXcdChunk - 1) / kXcdChunk;
    return 8 * ((chunks + 7) / 8) * kXcdChunk;
}

// NT threads per curve (the workgroup); a curve of n nodes needs n <= NT * MAXJ.
// pos: the workgroup's position in the launch's part of the line list.
template <typename T, int FAM, int MAXJ, int NT, bool DIR>
__device__ __forceinline__ void line_body(const LineArgs<T> &a, const T *__restrict__ fin, T *__restrict__ vout,
                                          const double *__restrict__ par, const int *__restrict__ done, int nmax,
                                          int pos) {
    // LDS: line_lds_arrays(FAM) arrays of line_lds_stride(nmax) elements
    //   P0  gathered values U, then the solution X
    //   P1  chords h; after every thread has read its chunk, the reduced system
    //   P2  |beta| (beta family)
    // The matrix rows are rebuilt in registers from h and |beta| in chunk
    // order, so no row array is staged (a small footprint: more resident
    // workgroups per CU to hide the latency of the serial elimination).
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int S = line_lds_stride(nmax, NT);
    T *P0 = reinterpret_cast<T *>(smem_raw);
    T *P1 = P0 + S;
    T *P2 = P1 + S;
    T *U = P0, *X = P0;
    T *Hs = P1, *Ws = P2;
    // reduced system: two buffers of normalised rows (a, c, d); the chunks'
    // first rows FY, FA, FG occupy the second buffer until the first PCR step
    T *A0 = P1, *C0 = A0 + NT, *D0 = C0 + NT;
    T *A1 = D0 + NT, *C1 = A1 + NT, *D1 = C1 + NT;
    T *FY = A1, *FA = C1, *FG = D1;

    const int l = a.lidx ? a.lidx[a.lbase + pos] : a.lbase + pos;
    const int tid = threadIdx.x;
    const int inst = a.linst[l];
    if (done[inst]) return;
    const int o = a.loff[l];
    const int n = a.lcnt[l];
    const int N = n - 2;
    const int nx = a.inst_nx[inst];
    const double *pp = par + 8 * inst;
    const T cM = T(pp[0]), cK = T(pp[1]), cC = T(pp[2]);
    const T eM = T(pp[3]), eK = T(pp[4]), eC = T(pp[5]), eL = T(pp[6]);
    // Dirichlet values at the curve's ends (the state sweeps; zero for increments)
    T x0 = T(0), xn = T(0);
    if (a.gend && pp[7] != 0.0) {
        x0 = a.gend[2 * l];
        xn = a.gend[2 * l + 1];
    }
    const T ptol = T(a.ptol);
    bool bad = false;  // a pivot not finite or below ptol of its row's scale
    // exponentially fitted beta-lines: element e's stiffness scaled by
    // phi = Pe coth(Pe), Pe = |beta|_e h_e / (2 mu) (precomputed per element)
    const bool fit = FAM == 0 && a.phi != nullptr;

    // chunking of the rows: thread q owns rows rs .. rs+k-1, rs = q*m (m <= MAXJ)
    const int m = (N + NT - 1) / NT;
    const int Q = (N + m - 1) / m;  // non-empty chunks
    const int q = tid;
    const int rs = q * m;
    const int k = q < Q ? min(m, N - rs) : 0;

    // 1. all loads of this thread's nodes j = tid + 256 q (coalesced) issued
    //    before any use, then the bilinear gather (eq. (22)); node values to LDS
    T hj[MAXJ], wj[MAXJ], lk[MAXJ];
    int cj[MAXJ];
    T lxj[MAXJ], lyj[MAXJ];
    // direct transfer in the FP32 sweeps: the packed brackets (10 bytes, 3
    // registers per slot) are loaded with the other node data
    constexpr bool DIR16 = DIR && sizeof(T) == 4;
    int dk0j[DIR16 ? MAXJ : 1];
    int dkdj[DIR16 ? MAXJ : 1];
    unsigned dwj[DIR16 ? MAXJ : 1];
#pragma unroll
    for (int sl = 0; sl < MAXJ; ++sl) {
        const int j = tid + NT * sl;
        cj[sl] = -1;
        lxj[sl] = T(0);
        lyj[sl] = T(0);
        if (!DIR && j > 0 && j < n - 1) {
            const int kn = o + j;
            cj[sl] = a.cell[kn];
            lxj[sl] = a.lx[kn];
            lyj[sl] = a.ly[kn];
        }
        if constexpr (DIR16) {
            const bool in = j > 0 && j < n - 1;
            dk0j[sl] = in ? a.dk0[o + j] : -1;
            dkdj[sl] = in ? static_cast<int>(a.dkd[o + j]) : static_cast<int>(kDirNoRight);
            dwj[sl] = in ? a.dwp[o + j] : 0u;
        }
        if (j > 0 && j < n) hj[sl] = a.h[o + j];
        if (FAM == 0 && j < n) wj[sl] = a.w[o + j];
    }
    // gathers in groups of (up to) 4 slots: the 16 corner loads of a group are
    // issued together (cell 0 stands in for the end nodes, whose value is
    // dropped), then the group's values go to LDS; G divides MAXJ, so every
    // group's slots exist
    constexpr int G = MAXJ % 4 == 0 ? 4 : MAXJ % 3 == 0 ? 3 : MAXJ % 2 == 0 ? 2 : 1;
    static_assert(MAXJ % G == 0, "gather groups must tile the slots");
#pragma unroll
    for (int q0 = 0; q0 < MAXJ; q0 += G) {
        T p11[G], p12[G], p21[G], p22[G];
        if constexpr (DIR) {
            // the brackets of the direct transfer: two source segments (or the
            // curve's own ends) per node, their four values issued together
            int2 dk[G];
            T dw[G][4];
#pragma unroll
            for (int t = 0; t < G; ++t) {
                if constexpr (DIR16) {
                    const int k0 = dk0j[q0 + t], d = dkdj[q0 + t];
                    if (d == kDirNoLeft) {
                        dk[t] = make_int2(-1, k0);
                    } else {
                        int kr = k0 + d;
                        if (d == kDirNoRight) kr = -1;
                        else if (d == kDirEscape) kr = a.dk[o + tid + NT * (q0 + t)].y;  // rare
                        dk[t] = make_int2(k0, kr);
                    }
                    const unsigned e = dwj[q0 + t];
                    const T wl = static_cast<T>(e & 0x3ffu) * T(1.0f / 1023.0f);
                    const T tl = static_cast<T>((e >> 10) & 0x7ffu) * T(1.0f / 2047.0f);
                    const T tr = static_cast<T>(e >> 21) * T(1.0f / 2047.0f);
                    const T wr = T(1) - wl;
                    dw[t][1] = wl * tl;
                    dw[t][0] = wl - dw[t][1];
                    dw[t][3] = wr * tr;
                    dw[t][2] = wr - dw[t][3];
                } else {
                    const int j = tid + NT * (q0 + t);
                    const bool in = j > 0 && j < n - 1;
                    dk[t] = in ? a.dk[o + j] : make_int2(-1, -1);
#pragma unroll
                    for (int e = 0; e < 4; ++e) dw[t][e] = in ? a.dw[4 * static_cast<int64_t>(o + j) + e] : T(0);
                }
            }
#pragma unroll
            for (int t = 0; t < G; ++t) {
                const int kl = dk[t].x >= 0 ? dk[t].x : 0, kr = dk[t].y >= 0 ? dk[t].y : 0;
                p11[t] = fin[kl];
                p12[t] = fin[kl + 1];
                p21[t] = fin[kr];
                p22[t] = fin[kr + 1];
            }
#pragma unroll
            for (int t = 0; t < G; ++t) {
                const int sl = q0 + t;
                const int j = tid + NT * sl;
                const T vl = dk[t].x >= 0 ? dw[t][0] * p11[t] + dw[t][1] * p12[t] : dw[t][0] * x0;
                const T vr = dk[t].y >= 0 ? dw[t][2] * p21[t] + dw[t][3] * p22[t] : dw[t][2] * xn;
                const T uj = (j > 0 && j < n - 1) ? vl + vr : (j == 0 ? x0 : xn);
                if (j < n) {
                    U[j] = uj;
                    if (j > 0) Hs[j] = hj[sl];
                    if (FAM == 0) Ws[j] = wj[sl];
                }
            }
            continue;
        }
#pragma unroll
        for (int t = 0; t < G; ++t) {
            // blocked field (8 x 4 nodes per block): the corner's position in its
            // block is in the low bits of c; nx is the block-row stride
            const int c = cj[q0 + t] >= 0 ? cj[q0 + t] : 0;
            const int sx = (c & 7) == 7 ? 25 : 1;
            const int cu = c + (((c >> 3) & 3) == 3 ? nx - 24 : 8);
            p11[t] = fin[c];
            p12[t] = fin[c + sx];
            p21[t] = fin[cu];
            p22[t] = fin[cu + sx];
        }
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int sl = q0 + t;
            const int j = tid + NT * sl;
            const T lx = lxj[sl], ly = lyj[sl];
            const T ub = (T(1) - ly) * ((T(1) - lx) * p11[t] + lx * p12[t]) + ly * ((T(1) - lx) * p21[t] + lx * p22[t]);
            const T uj = cj[sl] >= 0 ? ub : (j == 0 ? x0 : xn);
            if (j < n) {
                U[j] = uj;
                if (j > 0) Hs[j] = hj[sl];
                if (FAM == 0) Ws[j] = wj[sl];
            }
        }
    }
    // loads of this thread's own rows (node rs + j + 1), in chunk order, in
    // flight across the barrier
    if (FAM == 0) {
#pragma unroll
        for (int j = 0; j < MAXJ; ++j) lk[j] = (j < k && eL != T(0)) ? a.L[o + rs + j + 1] : T(0);
    }
    __syncthreads();

    // 2. chunked elimination in registers.  Chunk q: rows rs..rs+k-1; its last
    //    row is a separator unless q is the last chunk; the others are interior
    //    rows, eliminated top-down with their dependence on the separators
    //    S_{q-1} (left) and S_q (right) carried along.
    const bool has_sep = q < Q - 1;
    const int kin = has_sep ? k - 1 : k;
    // rows and right-hand sides of the chunk, P1 rows of eq. (16)-(19):
    // M, K and C entries from the chords and |beta| (a sliding window over the
    // chunk's nodes), A = cM M + cK K + cC C, rhs = (eM M + eK K + eC C) u + eL L
    const T sixth = T(1) / T(6), third = T(1) / T(3);
    T ra_[MAXJ], rb_[MAXJ], rc_[MAXJ], rd_[MAXJ];
    {
        T um = T(0), u0 = T(0), hl = T(1), il = T(1), wm = T(0), w0 = T(0);
        if (k > 0) {
            um = U[rs];
            u0 = U[rs + 1];
            hl = Hs[rs + 1];
            il = recip(hl);
            if (FAM == 0) {
                wm = Ws[rs];
                w0 = Ws[rs + 1];
                if (fit) il *= a.phi[o + rs + 1];
            }
        }
#pragma unroll
        for (int j = 0; j < MAXJ; ++j) {
            if (j < k) {
                const int r = rs + j;
                const T up = U[r + 2], hr = Hs[r + 2];
                T ir = recip(hr);
                if (fit) ir *= a.phi[o + r + 2];
                const T mlo = hl * sixth, mdi = (hl + hr) * third, mup = hr * sixth;
                const T klo = -il, kdi = il + ir, kup = -ir;
                T lo = cM * mlo + cK * klo;
                T di = cM * mdi + cK * kdi;
                T hi = cM * mup + cK * kup;
                T rhs = eM * (mlo * um + mdi * u0 + mup * up) + eK * (klo * um + kdi * u0 + kup * up);
                if (FAM == 0) {
                    const T wp = Ws[r + 2];
                    const T clo = -(wm + T(2) * w0) * sixth;
                    const T cdi = (wm - wp) * sixth;
                    const T cup = (T(2) * w0 + wp) * sixth;
                    lo += cC * clo;
                    di += cC * cdi;
                    hi += cC * cup;
                    rhs += eC * (clo * um + cdi * u0 + cup * up) + eL * lk[j];
                    wm = w0;
                    w0 = wp;
                }
                ra_[j] = lo;
                rb_[j] = di;
                rc_[j] = hi;
                rd_[j] = rhs;
                um = u0;
                u0 = up;
                hl = hr;
                il = ir;
            }
        }
    }
    __syncthreads();  // U, h and |beta| read: P1 takes the reduced system, P0 the solution
    T sa = T(0), sb = T(1), sc = T(0), sd = T(0);  // separator row
    {
        T pc = T(0), py = T(0), pa = T(0);
#pragma unroll
        for (int j = 0; j < MAXJ; ++j) {
            if (j < kin) {
                const T ar = ra_[j];
                const T den = rb_[j] - ar * pc;
                bad |= !(fabs(den) > ptol * (fabs(rb_[j]) + fabs(ar * pc)));
                const T inv = recip(den);
                const T cp = rc_[j] * inv;
                const T yp = (rd_[j] - ar * py) * inv;
                const T al = (j == 0 ? -ar : -ar * pa) * inv;
                rc_[j] = cp;
                rd_[j] = yp;
                ra_[j] = al;
                pc = cp;
                py = yp;
                pa = al;
            } else if (has_sep && j == k - 1) {
                sa = ra_[j]; sb = rb_[j]; sc = rc_[j]; sd = rd_[j];
            }
        }
    }
    T yL = T(0), aL = T(1), gL = T(0);  // last interior row = yL + aL*S_{q-1} + gL*S_q
    T fy = T(0), fa = T(0), fg = T(1);  // first row (an empty chunk's first row is S_q)
    {
        T Y = T(0), Al = T(0), Ga = T(0);
#pragma unroll
        for (int j = MAXJ - 1; j >= 0; --j) {
            if (j == kin - 1) {
                Y = rd_[j]; Al = ra_[j]; Ga = -rc_[j];
                yL = Y; aL = Al; gL = Ga;
            } else if (j < kin - 1) {
                const T cp = rc_[j];
                Y = rd_[j] - cp * Y;
                Al = ra_[j] - cp * Al;
                Ga = -cp * Ga;
            }
        }
        if (kin > 0) { fy = Y; fa = Al; fg = Ga; }
    }
    if (q < Q) {
        FY[q] = fy;
        FA[q] = fa;
        FG[q] = fg;
    }
    __syncthreads();

    // 3. reduced system on the separators S_0..S_{Q-2}: parallel cyclic
    //    reduction on rows normalised to a unit diagonal,
    //    a x_{q-s} + x_q + c x_{q+s} = d, ping-ponging between two LDS buffers
    //    (one reciprocal and one barrier per step).  Finally d = S_q.
    const int R = Q - 1;
    const T *Sv = D0;
    {
        T ra = T(0), rc = T(0), rd = T(0);
        if (q < R) {
            const T nfy = FY[q + 1], nfa = FA[q + 1], nfg = FG[q + 1];
            // chunk 0's left neighbour and the last chunk's right one are the
            // curve's end nodes, whose values are known
            const T a = q > 0 ? sa * aL : T(0);
            const T b = sb + sa * gL + sc * nfa;
            const T c = q + 1 < R ? sc * nfg : T(0);
            const T d = sd - sa * yL - sc * nfy - (q == 0 ? sa * aL * x0 : T(0)) - (q + 1 == R ? sc * nfg * xn : T(0));
            bad |= !(fabs(b) > ptol * (fabs(sb) + fabs(sa * gL) + fabs(sc * nfa)));
            const T ib = recip(b);
            ra = a * ib;
            rc = c * ib;
            rd = d * ib;
        }
        A0[q] = ra; C0[q] = rc; D0[q] = rd;
        __syncthreads();
        T *Ai = A0, *Ci = C0, *Di = D0, *Ao = A1, *Co = C1, *Do = D1;
        for (int st = 1; st < R; st <<= 1) {
            if (q < R) {
                T la = T(0), lc = T(0), ld = T(0), ua = T(0), uc = T(0), ud = T(0);
                if (q - st >= 0) { la = Ai[q - st]; lc = Ci[q - st]; ld = Di[q - st]; }
                if (q + st < R) { ua = Ai[q + st]; uc = Ci[q + st]; ud = Di[q + st]; }
                const T den = T(1) - ra * lc - rc * ua;
                bad |= !(fabs(den) > ptol * (T(1) + fabs(ra * lc) + fabs(rc * ua)));
                const T ib = recip(den);
                const T na = -(ra * la) * ib;
                const T nc = -(rc * uc) * ib;
                const T nd = (rd - ra * ld - rc * ud) * ib;
                ra = na; rc = nc; rd = nd;
            }
            Ao[q] = ra; Co[q] = rc; Do[q] = rd;
            __syncthreads();
            T *t;
            t = Ai; Ai = Ao; Ao = t;
            t = Ci; Ci = Co; Co = t;
            t = Di; Di = Do; Do = t;
        }
        Sv = Di;
    }

    // 4. back-substitution of every chunk into X (P0)
    if (q < Q) {
        const T SL = q > 0 ? Sv[q - 1] : x0;
        const T SR = q < R ? Sv[q] : xn;
        T x = T(0);
#pragma unroll
        for (int j = MAXJ - 1; j >= 0; --j) {
            if (j == kin - 1) {
                x = rd_[j] + ra_[j] * SL - rc_[j] * SR;
                X[rs + j] = x;
            } else if (j < kin - 1) {
                x = rd_[j] + ra_[j] * SL - rc_[j] * x;
                X[rs + j] = x;
            }
        }
        if (has_sep) X[rs + k - 1] = SR;
    }
    __syncthreads();
    if constexpr (DIR) {
        // the update of the curve's interior values (summed per line in a fixed
        // order, and/or kept as the next increment), the state accumulation
        double racc = 0.0;
        for (int j = tid; j < n; j += NT) {
            const T val = j == 0 ? x0 : (j == n - 1 ? xn : X[j - 1]);
            if (j > 0 && j < n - 1) {
                if (a.lpart || a.dout) {
                    const double dlt = static_cast<double>(val) - static_cast<double>(vout[o + j]);
                    racc += dlt * dlt;
                    if (a.dout) a.dout[o + j] = static_cast<float>(dlt);
                }
                if (a.vacc) a.vacc[o + j] += static_cast<double>(val);
                if (a.vacc32) a.vacc32[o + j] += static_cast<float>(val);
            } else if (a.dout) {
                a.dout[o + j] = 0.0f;
            }
            vout[o + j] = val;
        }
        if (a.lpart) {
            double *red = reinterpret_cast<double *>(P1);  // the reduced system is no longer read
            red[tid] = racc;
            __syncthreads();
            for (int w = NT / 2; w > 0; w >>= 1) {
                if (tid < w) red[tid] += red[tid + w];
                __syncthreads();
            }
            if (tid == 0) a.lpart[a.lslot[l]] = red[0];
        }
    } else {
        for (int j = tid; j < n; j += NT) vout[o + j] = j == 0 ? x0 : (j == n - 1 ? xn : X[j - 1]);
    }
    if (bad && a.sing) a.sing[inst] = 1;
}

// One launch for every curve of a family: each workgroup picks the register
// footprint (nodes per thread) of its curve; the kernel's registers are those
// of the largest footprint.  The full list is dealt to the XCDs in chunks of
// neighbouring curves (a.xs); a list compacted to the unfinished instances
// runs in its own order (longest first within each instance's bucket).
template <typename T, int FAM, bool DIR = false>
__global__ __launch_bounds__(kThreads) void k_line(LineArgs<T> a, const T *__restrict__ fin,
                                                   T *__restrict__ vout, const double *__restrict__ par,
                                                   const int *__restrict__ done, int nmax) {
    // the list order (longest first) is the dispatch order, or each XCD takes
    // its share of the list in order
    int pos = static_cast<int>(blockIdx.x);
    if (a.xs) {
        const int p = a.xs[pos & 7] + (pos >> 3);
        if (p >= a.xs[(pos & 7) + 1]) return;
        pos = p;
    }
    const int per = (a.lcnt[a.lidx ? a.lidx[a.lbase + pos] : a.lbase + pos] + kThreads - 1) / kThreads;
    if (per <= 1) line_body<T, FAM, 1, kThreads, DIR>(a, fin, vout, par, done, nmax, pos);
    else if (per <= 2) line_body<T, FAM, 2, kThreads, DIR>(a, fin, vout, par, done, nmax, pos);
    else if (per <= 4) line_body<T, FAM, 4, kThreads, DIR>(a, fin, vout, par, done, nmax, pos);
    else if (per <= 8) line_body<T, FAM, 8, kThreads, DIR>(a, fin, vout, par, done, nmax, pos);
    else line_body<T, FAM, 12, kThreads, DIR>(a, fin, vout, par, done, nmax, pos);
}

// One launch per length bucket: every curve of the launch has at most
// NT * MAXJ nodes, and the kernel has that footprint's registers (more
// resident workgroups for the short curves), its LDS sized by the bucket's
// longest curve.  Short curves take smaller workgroups (128 or 64 threads,
// 4 rows each): fewer idle lanes and a shorter reduced system.
template <typename T, int FAM, int MAXJ, int NT, bool DIR = false>
__global__ __launch_bounds__(NT) void k_line_b(LineArgs<T> a, const T *__restrict__ fin,
                                               T *__restrict__ vout, const double *__restrict__ par,
                                               const int *__restrict__ done, int nmax, int nlist) {
    // the curves of one bucket, dealt to the XCDs in chunks of neighbours
    const int p = xcd_position(static_cast<int>(blockIdx.x), nlist);
    if (p < 0) return;
    line_body<T, FAM, MAXJ, NT, DIR>(a, fin, vout, par, done, nmax, p);
}

// Scatter: out = P v on the interior nodes.  MODE 0: write; MODE 1 (FP64 sweep):
// U <- val, d32 <- val - U_old, partial += (val - U_old)^2; MODE 2 (FP32 sweep):
// U += val, d32 <- val; MODE 3: partial += (val - U)^2, nothing written.
template <typename T, typename TO, int MODE>
__global__ __launch_bounds__(kThreads) void k_scatter(ScatterArgs<T> s, const T *__restrict__ v,
                                                      TO *__restrict__ out, float *__restrict__ d32,
                                                      double *__restrict__ partial,
                                                      const int *__restrict__ done) {
    const int blk = s.blist ? s.blist[blockIdx.x] : static_cast<int>(blockIdx.x);
    const int inst = s.blk_inst[blk];
    if (done[inst]) return;
    const int slot = blk * kThreads + threadIdx.x;
    const int g = s.gidx[slot];
    const int np = s.npad;

    // every load is issued before any is used (no branch between them): the
    // records, then the line values (a missing record reads v[0], v[1] with
    // its contribution dropped), and the old grid value, which depends only
    // on g
    int kk[4];
    T wa[4], wb[4];
    short dk[3];
    kk[0] = s.rk0[slot];
#pragma unroll
    for (int r = 0; r < 3; ++r) dk[r] = s.rd[r * np + slot];
    if constexpr (sizeof(T) == 4) {
        // increment sweeps: the weights from their factors, 12 bytes per slot
        // (quantised to ~3e-5; the FP64 sweeps, with FP64 weights, fix the
        // iterate and its residual)
        const unsigned e = s.sw[slot], t01 = s.rt[slot], t23 = s.rt[np + slot];
        const float wh = static_cast<float>(e & 3u) * 0.5f, wv = 1.0f - wh;
        const float lh = static_cast<float>((e >> 2) & 0x7fffu) * (1.0f / 32767.0f);
        const float lv = static_cast<float>(e >> 17) * (1.0f / 32767.0f);
        const float cf[4] = {wh * lh, wh - wh * lh, wv * lv, wv - wv * lv};
        const float tt[4] = {static_cast<float>(t01 & 0xffffu) * (1.0f / 65535.0f),
                             static_cast<float>(t01 >> 16) * (1.0f / 65535.0f),
                             static_cast<float>(t23 & 0xffffu) * (1.0f / 65535.0f),
                             static_cast<float>(t23 >> 16) * (1.0f / 65535.0f)};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            wb[r] = cf[r] * tt[r];
            wa[r] = cf[r] - wb[r];
        }
    } else {
        // state sweeps: the same factors in FP64 (48 bytes and the weight code)
        const unsigned e = s.sw[slot];
        const double wh = static_cast<double>(e & 3u) * 0.5, wv = 1.0 - wh;
        const double lh = s.rf[slot], lv = s.rf[np + slot];
        const double cf[4] = {wh * lh, wh - wh * lh, wv * lv, wv - wv * lv};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            wb[r] = cf[r] * s.rf[(2 + r) * np + slot];
            wa[r] = cf[r] - wb[r];
        }
    }
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        const short d = dk[r - 1];
        kk[r] = d == kRecMissing ? -1 : d == kRecEscape ? s.rk[r * np + slot] : kk[0] + d;
    }
    TO old = TO(0);
    if constexpr (MODE != 0) old = out[g >= 0 ? g : 0];
    T va[4], vb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = kk[r] >= 0 ? kk[r] : 0;
        va[r] = v[k];
        vb[r] = v[k + 1];
    }
    T val = T(0);
    if constexpr (sizeof(T) == 8) {
        if (s.gb) val = s.gb[slot];  // the Dirichlet data the boundary points carry
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (kk[r] >= 0) val += wa[r] * va[r] + wb[r] * vb[r];
    if constexpr (MODE == 0) {
        if (g >= 0) out[g] = TO(val);
    } else if constexpr (MODE == 2) {
        if (g >= 0) {
            out[g] = old + TO(val);
            d32[g] = float(val);
        }
    } else {
        double r = 0.0;
        if (g >= 0) {
            r = double(val) - double(old);
            if constexpr (MODE == 1) {
                out[g] = TO(val);
                d32[g] = float(r);
            }
        }
        // fixed-order block reduction of r^2
        __shared__ double red[kThreads];
        red[threadIdx.x] = r * r;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[blk] = red[0];
    }
}

// Per-instance norm.  mode 0: rel = sqrt(sum)/cnorm, record, set done at tol.
// mode 1: cnorm = sqrt(sum).  mode 2: rel only (no flags).
__global__ __launch_bounds__(kThreads) void k_norm(const double *__restrict__ partial,
                                                   const int *__restrict__ blk_start, double *__restrict__ cnorm,
                                                   double *__restrict__ rel, int *__restrict__ done,
                                                   int *__restrict__ it_count, int count, double tol, int mode) {
    const int inst = blockIdx.x;
    if (mode == 0 && done[inst]) return;
    const int b0 = blk_start[inst], b1 = blk_start[inst + 1];
    // eight loads in flight per thread (independent accumulators, fixed order)
    double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = b0 + threadIdx.x;
    for (; b + 7 * kThreads < b1; b += 8 * kThreads) {
        double p8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) p8[q] = partial[b + q * kThreads];
#pragma unroll
        for (int q = 0; q < 8; ++q) a8[q] += p8[q];
    }
    for (; b < b1; b += kThreads) a8[0] += partial[b];
    const double acc = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
    __shared__ double red[kThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double nrm = sqrt(red[0]);
    if (mode == 1) {
        cnorm[inst] = nrm;
        return;
    }
    const double cn = cnorm[inst] > 0.0 ? cnorm[inst] : 1.0;
    const double r = nrm / cn;
    rel[inst] = r;
    if (mode == 0) {
        it_count[inst] += count;  // sweeps applied since the previous measurement
        if (!(r <= tol)) return;  // NaN never converges
        done[inst] = 1;
    }
}

// The load of an implicit Euler step solved as a stationary problem: on every
// interior node of every beta-curve, L'_k = L_k + (M G u_n)_k / dt with G the
// bilinear gather of eq. (22) (the curve's ends take their Dirichlet data) and
// M the P1 mass rows.  One workgroup per curve; the gathered values go to LDS.
__global__ __launch_bounds__(kThreads) void k_shift_load(LineArgs<double> a, const double *__restrict__ Lbase,
                                                         const double *__restrict__ un, double *__restrict__ Lout,
                                                         double inv_dt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *su = reinterpret_cast<double *>(smem_raw);
    const int l = static_cast<int>(blockIdx.x);
    const int o = a.loff[l], n = a.lcnt[l], inst = a.linst[l];
    const int nx = a.inst_nx[inst];
    for (int j = threadIdx.x; j < n; j += kThreads) {
        double v;
        if (j == 0 || j == n - 1) {
            v = a.gend ? a.gend[2 * l + (j == 0 ? 0 : 1)] : 0.0;
        } else {
            const int c = a.cell[o + j];
            const int sx = (c & 7) == 7 ? 25 : 1;
            const int cu = c + (((c >> 3) & 3) == 3 ? nx - 24 : 8);
            const double lx = a.lx[o + j], ly = a.ly[o + j];
            v = (1.0 - ly) * ((1.0 - lx) * un[c] + lx * un[c + sx]) + ly * ((1.0 - lx) * un[cu] + lx * un[cu + sx]);
        }
        su[j] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kThreads) {
        double Lk = Lbase[o + j];
        if (j > 0 && j < n - 1) {
            const double hl = a.h[o + j], hr = a.h[o + j + 1];
            Lk += inv_dt * (hl / 6.0 * su[j - 1] + (hl + hr) / 3.0 * su[j] + hr / 6.0 * su[j + 1]);
        }
        Lout[o + j] = Lk;
    }
}

// Curve values from a grid field: ends from gend (or 0), interior nodes the
// bilinear gather of U (eq. (22)), or 0 when U is NULL; zacc, when set, is
// cleared on the same nodes (an accumulator of later curve values).  One
// workgroup per line of the list (a.lidx when set).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_line_values(LineArgs<T> a, const T *__restrict__ U,
                                                          T *__restrict__ v, T *__restrict__ zacc) {
    const int l = a.lidx ? a.lidx[blockIdx.x] : static_cast<int>(blockIdx.x);
    const int o = a.loff[l], n = a.lcnt[l], inst = a.linst[l];
    const int nx = a.inst_nx[inst];
    for (int j = threadIdx.x; j < n; j += kThreads) {
        T val = T(0);
        if (j == 0 || j == n - 1) {
            val = a.gend ? a.gend[2 * l + (j == 0 ? 0 : 1)] : T(0);
        } else if (U) {
            const int c = a.cell[o + j];
            const int sx = (c & 7) == 7 ? 25 : 1;
            const int cu = c + (((c >> 3) & 3) == 3 ? nx - 24 : 8);
            const T lx = a.lx[o + j], ly = a.ly[o + j];
            val = (T(1) - ly) * ((T(1) - lx) * U[c] + lx * U[c + sx]) + ly * ((T(1) - lx) * U[cu] + lx * U[cu + sx]);
        }
        v[o + j] = val;
        if (zacc) zacc[o + j] = T(0);
    }
}

// ------------------------------------------------------------------ compaction
// active items (instance not done), order preserved: per-block counts, one
// workgroup scans them, then every block writes its items' indices
__global__ __launch_bounds__(kThreads) void k_count_active(const int *__restrict__ inst_of, int n,
                                                           const int *__restrict__ done, int *__restrict__ bcnt) {
    __shared__ int red[kThreads];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    red[threadIdx.x] = (i < n && !done[inst_of[i]]) ? 1 : 0;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bcnt[blockIdx.x] = red[0];
}

// in-place exclusive scan of nb counts by one workgroup; *total = their sum
__global__ __launch_bounds__(kThreads) void k_scan_counts(int *__restrict__ bcnt, int nb, int *__restrict__ total) {
    __shared__ int sc[kThreads];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += kThreads) {
        const int b = b0 + threadIdx.x;
        const int v = b < nb ? bcnt[b] : 0;
        sc[threadIdx.x] = v;
        __syncthreads();
        for (int w = 1; w < kThreads; w <<= 1) {  // inclusive Hillis-Steele scan
            const int add = static_cast<int>(threadIdx.x) >= w ? sc[threadIdx.x - w] : 0;
            __syncthreads();
            sc[threadIdx.x] += add;
            __syncthreads();
        }
        const int base = carry;
        if (b < nb) bcnt[b] = base + sc[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kThreads - 1) carry = base + sc[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kThreads) void k_write_active(const int *__restrict__ inst_of, int n,
                                                           const int *__restrict__ done,
                                                           const int *__restrict__ bstart, int *__restrict__ idx) {
    __shared__ int sc[kThreads];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const int f = (i < n && !done[inst_of[i]]) ? 1 : 0;
    sc[threadIdx.x] = f;
    __syncthreads();
    for (int w = 1; w < kThreads; w <<= 1) {
        const int add = static_cast<int>(threadIdx.x) >= w ? sc[threadIdx.x - w] : 0;
        __syncthreads();
        sc[threadIdx.x] += add;
        __syncthreads();
    }
    if (f) idx[bstart[blockIdx.x] + sc[threadIdx.x] - 1] = i;
}

__global__ void k_layout(const int *__restrict__ gr, const int *__restrict__ gb, int npad,
                         const double *__restrict__ src, double *__restrict__ dst, int to_blocked) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad) return;
    const int r = gr[s];
    if (r < 0) return;
    if (to_blocked) dst[gb[s]] = src[r];
    else dst[r] = src[gb[s]];
}

__global__ void k_fill_int(int *p, int v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers
template <typename T>
size_t line_lds_bytes(int fam, int nmax) {
    return sizeof(T) * static_cast<size_t>(line_lds_arrays(fam)) * line_lds_stride(nmax);
}

namespace {
template <typename K>
void set_lds(K *kernel, size_t lds) {
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(lds));
}

template <typename T, int FAM, int MAXJ, int NT, bool DIR>
void launch_b(const LineArgs<T> &a, int n_lines, const T *fin, T *vout, const double *par, const int *done, int nmax,
              hipStream_t st) {
    const size_t lds = sizeof(T) * static_cast<size_t>(line_lds_arrays(FAM)) * line_lds_stride(nmax, NT);
    set_lds(&k_line_b<T, FAM, MAXJ, NT, DIR>, lds);
    hipLaunchKernelGGL((k_line_b<T, FAM, MAXJ, NT, DIR>), dim3(line_grid(n_lines)), dim3(NT), lds, st, a, fin, vout,
                       par, done, nmax, n_lines);
}

// buckets 0..4: curves of at most 3072, 2048, 1024, 512, 256 nodes; each
// bucket's workgroup shapes (rows per thread x threads) cover its longest
// curve, shape 0 first
template <typename T, int FAM, bool DIR>
void launch_line_fam(int bucket, int shape, const LineArgs<T> &a, int n_lines, const T *fin, T *vout,
                     const double *par, const int *done, int nmax, hipStream_t st) {
    switch (bucket * 4 + shape) {
        case 0: launch_b<T, FAM, 12, 256, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 1: launch_b<T, FAM, 6, 512, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 4: launch_b<T, FAM, 8, 256, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 5: launch_b<T, FAM, 4, 512, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 8: launch_b<T, FAM, 4, 256, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 9: launch_b<T, FAM, 8, 128, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 10: launch_b<T, FAM, 2, 512, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 12: launch_b<T, FAM, 4, 128, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 13: launch_b<T, FAM, 2, 256, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 14: launch_b<T, FAM, 8, 64, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 16: launch_b<T, FAM, 4, 64, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 17: launch_b<T, FAM, 2, 128, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        case 18: launch_b<T, FAM, 1, 256, DIR>(a, n_lines, fin, vout, par, done, nmax, st); break;
        default: {
            const size_t lds = line_lds_bytes<T>(FAM, nmax);
            set_lds(&k_line<T, FAM, DIR>, lds);
            hipLaunchKernelGGL((k_line<T, FAM, DIR>), dim3(n_lines), dim3(kThreads), lds, st, a, fin, vout, par, done,
                               nmax);
            break;
        }
    }
}
}  // namespace

int line_bucket(int nodes) {
    const int per = (nodes + kThreads - 1) / kThreads;
    return per <= 1 ? 4 : per <= 2 ? 3 : per <= 4 ? 2 : per <= 8 ? 1 : 0;
}

int line_shapes(int bucket) {
    static const int kShapes[kLineBuckets] = {2, 2, 3, 3, 3};
    return bucket >= 0 && bucket < kLineBuckets ? kShapes[bucket] : 1;
}

template <typename T>
hipError_t launch_line(int fam, int bucket, int shape, const LineArgs<T> &a, int n_lines, const T *fin, T *vout,
                       const double *par, const int *done, int nmax, hipStream_t st) {
    if (n_lines == 0) return hipSuccess;
    if (nmax > 12 * kThreads || bucket > 4) return hipErrorInvalidValue;
    if (bucket >= 0 && line_bucket(nmax) < bucket) return hipErrorInvalidValue;  // curves too long for the bucket
    if (bucket >= 0 && (shape < 0 || shape >= line_shapes(bucket))) return hipErrorInvalidValue;
    if (bucket >= 0 && a.xs) return hipErrorInvalidValue;  // XCD shares serve the single launch
    const int sh = bucket < 0 ? 0 : shape;
    if (a.dk) {
        if (fam == 0) launch_line_fam<T, 0, true>(bucket, sh, a, n_lines, fin, vout, par, done, nmax, st);
        else launch_line_fam<T, 1, true>(bucket, sh, a, n_lines, fin, vout, par, done, nmax, st);
    } else if (fam == 0) {
        launch_line_fam<T, 0, false>(bucket, sh, a, n_lines, fin, vout, par, done, nmax, st);
    } else {
        launch_line_fam<T, 1, false>(bucket, sh, a, n_lines, fin, vout, par, done, nmax, st);
    }
    return hipGetLastError();
}

template <typename T, typename TO>
hipError_t launch_scatter(int mode, const ScatterArgs<T> &s, const T *v, TO *out, float *d32, double *partial,
                          const int *done, hipStream_t st) {
    const int nb = s.blist ? s.nblist : s.npad / kThreads;
    if (nb == 0) return hipSuccess;
    switch (mode) {
        case 0: hipLaunchKernelGGL((k_scatter<T, TO, 0>), dim3(nb), dim3(kThreads), 0, st, s, v, out, d32, partial, done); break;
        case 1: hipLaunchKernelGGL((k_scatter<T, TO, 1>), dim3(nb), dim3(kThreads), 0, st, s, v, out, d32, partial, done); break;
        case 2: hipLaunchKernelGGL((k_scatter<T, TO, 2>), dim3(nb), dim3(kThreads), 0, st, s, v, out, d32, partial, done); break;
        default: hipLaunchKernelGGL((k_scatter<T, TO, 3>), dim3(nb), dim3(kThreads), 0, st, s, v, out, d32, partial, done); break;
    }
    return hipGetLastError();
}

hipError_t launch_norm(int n_inst, const double *partial, const int *blk_start, double *cnorm, double *rel, int *done,
                       int *it_count, int count, double tol, int mode, hipStream_t st) {
    hipLaunchKernelGGL(k_norm, dim3(n_inst), dim3(kThreads), 0, st, partial, blk_start, cnorm, rel, done, it_count,
                       count, tol, mode);
    return hipGetLastError();
}

hipError_t launch_layout(const int *gr, const int *gb, int npad, const double *src, double *dst, bool to_blocked,
                         hipStream_t st) {
    if (npad <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_layout, dim3((npad + kThreads - 1) / kThreads), dim3(kThreads), 0, st, gr, gb, npad, src, dst,
                       to_blocked ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_compact(const int *inst_of, int n, const int *done, int *bcnt, int *idx, int *count, hipStream_t st) {
    const int nb = (n + kThreads - 1) / kThreads;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_active, dim3(nb), dim3(kThreads), 0, st, inst_of, n, done, bcnt);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kThreads), 0, st, bcnt, nb, count);
    hipLaunchKernelGGL(k_write_active, dim3(nb), dim3(kThreads), 0, st, inst_of, n, done, bcnt, idx);
    return hipGetLastError();
}

hipError_t launch_shift_load(const LineArgs<double> &a, int n_lines, int nmax, const double *Lbase, const double *un,
                             double *Lout, double inv_dt, hipStream_t st) {
    if (n_lines == 0) return hipSuccess;
    const size_t lds = sizeof(double) * static_cast<size_t>(nmax);
    set_lds(&k_shift_load, lds);
    hipLaunchKernelGGL(k_shift_load, dim3(n_lines), dim3(kThreads), lds, st, a, Lbase, un, Lout, inv_dt);
    return hipGetLastError();
}

hipError_t launch_line_values(const LineArgs<double> &a, int n_lines, const double *U, double *v, hipStream_t st) {
    if (n_lines == 0) return hipSuccess;
    hipLaunchKernelGGL(k_line_values<double>, dim3(n_lines), dim3(kThreads), 0, st, a, U, v, nullptr);
    return hipGetLastError();
}

hipError_t launch_line_values32(const LineArgs<float> &a, int n_lines, const float *U, float *v, float *zacc,
                                hipStream_t st) {
    if (n_lines == 0) return hipSuccess;
    hipLaunchKernelGGL(k_line_values<float>, dim3(n_lines), dim3(kThreads), 0, st, a, U, v, zacc);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int v, int n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

template size_t line_lds_bytes<double>(int, int);
template size_t line_lds_bytes<float>(int, int);
template hipError_t launch_line<double>(int, int, int, const LineArgs<double> &, int, const double *, double *,
                                        const double *, const int *, int, hipStream_t);
template hipError_t launch_line<float>(int, int, int, const LineArgs<float> &, int, const float *, float *,
                                       const double *, const int *, int, hipStream_t);
template hipError_t launch_scatter<double, double>(int, const ScatterArgs<double> &, const double *, double *,
                                                   float *, double *, const int *, hipStream_t);
template hipError_t launch_scatter<float, float>(int, const ScatterArgs<float> &, const float *, float *, float *,
                                                 double *, const int *, hipStream_t);
template hipError_t launch_scatter<float, double>(int, const ScatterArgs<float> &, const float *, double *, float *,
                                                  double *, const int *, hipStream_t);

}  // namespace adr
