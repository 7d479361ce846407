// Run/sheet back projection for ordered ray lists (presorted listmode events,
// radial-view-plane sinograms).
//
// Float atomic adds on this GPU are priced per cache-line request at the
// memory side, so the direct scatter (4 atomics per plane sample) is bound by
// request count.  In an ordered ray list, consecutive rays very often lie on
// the same transaxial line: same principal axis p (0 or 1) and identical
// in-plane coordinate U(k) = U0 + k dU at every plane k -- they differ only in
// their axial coordinate W(k) and in their value.  All contributions of such a
// run then fall into a "sheet" of the image: at plane k the two columns
// (k, i0(k), :) and (k, i0(k) + 1, :) along the fastest axis (2).
//
// A workgroup takes 256 consecutive rays of the processing order and splits
// them into runs (bitwise-equal p, U0, dU).  For every run of >= kRunMin rays
// each thread becomes a plane k: it walks the run's rays and accumulates the
// W-interpolated values into its own LDS column (thread-private addresses: no
// atomics, no bank conflicts; the current pair of z entries is kept in
// registers, its column values read when z moves to it and written back when z
// moves on), then the waves flush the sheet with contiguous, duplicate-free
// atomics -- one memory request per ~16 values instead of one per value.  The
// column stride is the grid's longest line + 1, so that two workgroups fit a
// CU's LDS on clinical grids: the loop needs the second workgroup's waves.  The
// u-weights (1 - fu, fu) are shared by the run and applied at the flush.  Rays
// in short runs (or with p == 2, or grids whose axis 2 exceeds the LDS column)
// take the direct wave-synchronous, run-combined scatter.  The arithmetic per
// (ray, plane) sample is the same as in the direct path; only the order of
// float additions differs.
#pragma once

#include "joseph.hpp"

namespace ppmi {

constexpr int kSheetBlock = 256;
constexpr int kRunMin = 2;
constexpr int kSheetMaxW = 128;  // largest axis-2 size with an LDS sheet
constexpr int kSheetGroups = 8;  // groups of 256 rays per workgroup (a sheet persists across them)
constexpr int kNoEntry = -(1 << 30);  // "no z entry cached": no ray's floor(W) comes near it

// LDS layout of k_back_runs (bytes): per-ray arrays, then the column buffer.
struct SheetLayout {
    static constexpr int kDoubles = 6;  // W0 dW s0 ds U0 dU
    static constexpr int kWords = 7;    // cv, lohi, pax, start, cnt, list, aux; + 24 words
    static size_t ray_bytes() { return (size_t)kSheetBlock * (kDoubles * 8 + kWords * 4) + 24 * 4; }
    // column stride: the longest line a sheet can hold (planes along axis 0 or 1, at most one
    // per thread) + 1; sized to the grid so that two workgroups share a CU's LDS on the
    // clinical grid (215 planes, 71 z entries: 79.8 KB)
    __host__ __device__ static int col_stride(const GeomK& g) {
        const int np = g.n[0] > g.n[1] ? g.n[0] : g.n[1];
        return (np < kSheetBlock ? np : kSheetBlock) + 1;
    }
    // nw rows of the sheet plus one spare row that absorbs the out-of-grid entries of a z pair
    // (216-entry rows on the clinical grid: 81,760 bytes, two workgroups per CU)
    static size_t bytes(int nw, const GeomK& g) { return ray_bytes() + (size_t)(nw + 1) * col_stride(g) * 4; }
};

// Per-ray value hooks:
//   setup(l, r, cv, aux): prepare ray l (false = no contribution); cv = ell * p (the constant
//                    factor of every sample); for listmode TOF, r.s0 is made relative to the bin
//                    centre; aux: a per-ray word the mode keeps (kAux)
//   sample(x, cv, aux): the value scattered at the plane sample with TOF coordinate
//                    x = fma(k, r.ds, r.s0)
struct ModeNonTof {
    static constexpr bool kAux = false;
    const float* __restrict__ p;
    __device__ bool setup(int64_t l, const RaySrc& src, const GeomK& g, RayK& r, float& cv,
                          int& /*aux*/) const {
        const float pl = p[l];
        if (pl == 0.0f || !ray_setup(src, l, g, r)) return false;
        cv = r.ell * pl;
        return true;
    }
    __device__ float sample(double /*x*/, float cv, int /*aux*/) const { return cv; }
};

// Listmode TOF, the weight in form Form (TofForm).  With per-ray TOF parameters (PerRay) the ray's
// offset is folded into its TOF coordinate at setup and aux carries the bits of its erf argument
// per mm (TofRay::inv).
template <int Form, bool PerRay = false>
struct ModeTofLm {
    static constexpr bool kAux = PerRay;
    const float* __restrict__ p;
    const int16_t* __restrict__ bins;
    TofK t;
    __device__ bool setup(int64_t l, const RaySrc& src, const GeomK& g, RayK& r, float& cv,
                          int& aux) const {
        const int b = bins[l];
        const float pl = p[l];
        TofRay q;
        if (b < 0 || b >= t.nb || pl == 0.0f || !tof_ray<PerRay>(t, l, q) || !ray_setup(src, l, g, r))
            return false;
        if (PerRay) r.s0 -= q.shift;
        if (!tof_window_rel(r, t.c0 + b * t.bw, q.lo, q.hi)) return false;
        cv = r.ell * pl * kTofScale<Form>;
        if (PerRay) aux = __float_as_int(q.inv);
        return true;
    }
    __device__ float sample(double x, float cv, int aux) const {
        return tof_weight_unscaled<Form>(x, t, PerRay ? __int_as_float(aux) : t.u_per_mm) * cv;
    }
};

// Sinogram TOF: the value at a plane sample is ell * sum over the bins b of its TOF window of
// w_b(s) p[l][b] (neighbouring bins share their erf edge).  aux carries the ray index l (the
// sheet path is used for fewer than 2^31 rays); all lanes of a wave read the same ray's bin
// values, so those loads hit one or two cache lines.  With per-ray TOF parameters (PerRay) the
// ray's offset is folded into its TOF coordinate at setup and its sigma is read per sample.
template <bool Lut, bool PerRay = false>
struct ModeTofSino {
    static constexpr bool kAux = true;
    const float* __restrict__ p;  // [n][n_bins]
    TofK t;
    __device__ bool setup(int64_t l, const RaySrc& src, const GeomK& g, RayK& r, float& cv,
                          int& aux) const {
        const float* pr = p + l * t.nb;
        bool any = false;
        for (int b = 0; b < t.nb; ++b) any |= (pr[b] != 0.0f);
        TofRay q;
        if (!any || !tof_ray<PerRay>(t, l, q) || !ray_setup(src, l, g, r)) return false;
        if (PerRay) r.s0 -= q.shift;
        cv = r.ell;
        aux = (int)l;
        return true;
    }
    __device__ float sample(double s, float cv, int aux) const {
        const float* pr = p + (int64_t)aux * t.nb;
        TofRay q;
        tof_ray<PerRay>(t, aux, q);  // usable: checked at setup
        int b_lo, b_hi;
        tof_bin_range(s, t, q.lo, q.hi, b_lo, b_hi);
        float c = 0.0f;
        if (Lut) {
            for (int b = b_lo; b <= b_hi; ++b) c += tof_lut(s - (t.c0 + b * t.bw), t) * pr[b];
        } else {
            const float x_hi0 = (float)(s - (t.c0 + b_lo * t.bw) + 0.5 * t.bw), bwf = (float)t.bw;
            float e_hi = tof_erf(x_hi0, q.inv, t);
            for (int b = b_lo; b <= b_hi; ++b) {
                const float e_lo = tof_erf(x_hi0 - (float)(b - b_lo + 1) * bwf, q.inv, t);
                c += 0.5f * (e_hi - e_lo) * pr[b];
                e_hi = e_lo;
            }
        }
        return c * cv;
    }
};

// Row of z entry j in a thread's column: entries outside the grid (j = -1, j = nw, or no entry yet)
// go to the spare row nw, which is never flushed, so that a pair's LDS accesses need no branch.
__device__ __forceinline__ int col_row(int j, int nw) { return ((unsigned)j < (unsigned)nw) ? j : nw; }

// Flush the sheet of line (p, U0, dU) with contiguous atomics and clear it: only the planes
// whose thread accumulated something (touched), listed in tl[], only the z entries between the
// lowest and the highest any of them wrote ([zlo, zhi] of each thread, united over the
// workgroup), and with the (plane, z) entries spread over all threads (consecutive threads take
// consecutive z of a plane).  Every thread of the workgroup calls it; the caller synchronises
// before and after.
__device__ __forceinline__ void sheet_flush(float* __restrict__ img, float* col, const GeomK& g, int p, double U0,
                                            double dU, bool touched, int zlo, int zhi, int nw, int cs, int* tl,
                                            int* tcount) {
    constexpr int B = kSheetBlock;
    const int tid = threadIdx.x, lane = (int)__lane_id(), wave = tid >> 6;
    const unsigned long long bal = __ballot(touched);
    // per wave: touched count (bits 0-7), lowest z (bits 8-15), highest z (bits 16-23); nw <= 128.
    // Both ends are clamped to [0, nw - 1] per lane: a thread whose writes all went to out-of-grid
    // entries (a pair below z = 0 at the conservative end plane of a window, or above nw - 1) has
    // zhi < 0 or zlo >= nw, and an unclamped negative value would sign-extend into the packed word.
    const int wlo = wave_min(touched ? min(max(zlo, 0), nw - 1) : 255);
    const int whi = wave_max(touched ? max(min(zhi, nw - 1), 0) : 0);
    if (lane == 0) tcount[wave] = __popcll(bal) | (wlo << 8) | (whi << 16);
    __syncthreads();
    int off = 0, nt = 0, z0 = 255, z1 = 0;
    for (int w = 0; w < B / 64; ++w) {
        const int c = tcount[w];
        off += (w < wave) ? (c & 0xff) : 0;
        nt += c & 0xff;
        z0 = min(z0, (c >> 8) & 0xff);
        z1 = max(z1, (c >> 16) & 0xff);
    }
    if (touched) tl[off + __popcll(bal & ((1ull << lane) - 1ull))] = tid;
    __syncthreads();
    const int su = (p == 0) ? g.stride[1] : g.stride[0];
    const int sp = g.stride[p];
    const int nu = (p == 0) ? g.n[1] : g.n[0];
    const int nz = max(z1 - z0 + 1, 0);
    const int total = nt * nz;
    const float inv_nz = 1.0f / (float)max(nz, 1);
    for (int e = tid; e < total; e += B) {
        // e / nz: (e + 1/2) / nz stays >= 1/(2 nz) away from an integer, far above float error
        const int pi = (int)(((float)e + 0.5f) * inv_nz), j = z0 + e - pi * nz;
        const int k = tl[pi];
        float* cp = col + j * cs + k;
        const float v = *cp;
        if (v != 0.0f) {
            *cp = 0.0f;
            const double U = fma((double)k, dU, U0);
            const double fi = floor(U);
            const int i0 = (int)fi;
            const float fu = (float)(U - fi);
            const int base = k * sp + i0 * su;
            if ((unsigned)i0 < (unsigned)nu) unsafeAtomicAdd(img + base + j, (1.0f - fu) * v);
            if ((unsigned)(i0 + 1) < (unsigned)nu) unsafeAtomicAdd(img + base + su + j, fu * v);
        }
    }
}

// One workgroup walks `groups` consecutive groups of 256 rays of the processing
// order.  The sheet of the current line persists across groups (thread t holds
// the column of absolute plane t, so lines need n_p <= 256); it is flushed when a
// run of another line starts, and at the end.
template <class Mode>
__device__ void back_runs_chunk(const Mode& m, RaySrc src, int64_t n,
                                const GeomK& g, float* __restrict__ img, const int32_t* __restrict__ order,
                                int nw_lds, int groups, int64_t chunk0, double* smem) {
    constexpr int B = kSheetBlock;
    double* W0 = smem;
    double* dW = W0 + B;
    double* s0 = dW + B;
    double* ds = s0 + B;
    double* U0 = ds + B;
    double* dU = U0 + B;
    float* cvs = reinterpret_cast<float*>(dU + B);
    int* lohi = reinterpret_cast<int*>(cvs + B);  // k_lo | k_hi << 16 (sheet rays: planes < 256)
    int* pax = lohi + B;
    int* start = pax + B;
    int* cnt = start + B;
    int* masks = cnt + B;  // 8 words: run-boundary ballots of the 4 waves
    int* list = masks + 8;  // sheet-run heads; count at list[B]; per-wave counts at list[B + 4 ..]
    int* aux = list + B + 8;  // per-ray word of the mode (sinogram TOF: the ray index)
    // the flush's list of touched planes reuses start[] and masks[], which only the run
    // detection before the sheet loop uses
    int* tl = start;
    float* col = reinterpret_cast<float*>(aux + B + 8);  // [nw][cs]
    const int cs = SheetLayout::col_stride(g);

    const int tid = threadIdx.x;
    const int lane = (int)__lane_id();
    const int wave = tid >> 6;
    const int nw = g.n[2];
    const bool sheets = nw_lds > 0 && nw <= nw_lds;
    if (sheets)
        for (int q = tid; q < nw * cs; q += B) col[q] = 0.0f;
    // current sheet (block-uniform copies in registers, updated after barriers)
    bool sh_on = false, touched = false;  // touched: this thread's plane holds sheet values
    int zlo = INT_MAX, zhi = INT_MIN;      // z entries it wrote since the last flush (pairs jc, jc + 1)
    int sh_p = -1, sh_kmax = -1;
    double sh_U0 = 0.0, sh_dU = 0.0;
    for (int grp = 0; grp < groups; ++grp) {
        const int64_t i = chunk0 + (int64_t)grp * B + tid;
        if (chunk0 + (int64_t)grp * B >= n) break;  // block-uniform
        int64_t l = -1;
        if (i < n) {
            l = order ? (int64_t)order[i] : i;
            if (l < 0 || l >= n) l = -1;
        }
        RayK r;
        float cv = 0.0f;
        int ax = 0;
        const bool ok = l >= 0 && m.setup(l, src, g, r, cv, ax);
        // compact the valid rays to the front of the group (stable order), so that rays
        // without a contribution do not break runs
        const unsigned long long vb = __ballot(ok);
        __syncthreads();  // previous group's LDS readers are done
        if (lane == 0) list[B + 4 + wave] = __popcll(vb);
        __syncthreads();
        int voff = 0, nvalid = 0;
        for (int w = 0; w < B / 64; ++w) {
            const int c_w = list[B + 4 + w];
            voff += (w < wave) ? c_w : 0;
            nvalid += c_w;
        }
        const int cp = ok ? voff + __popcll(vb & ((1ull << lane) - 1ull)) : -1;
        if (ok) {
            W0[cp] = r.W0;
            dW[cp] = r.dW;
            s0[cp] = r.s0;
            ds[cp] = r.ds;
            U0[cp] = r.U0;
            dU[cp] = r.dU;
            cvs[cp] = cv;
            aux[cp] = ax;
            lohi[cp] = (r.k_lo & 0xffff) | (r.k_hi << 16);
            pax[cp] = r.p;
        }
        __syncthreads();
        // runs over the compacted entries (thread t examines entry t): maximal stretches with
        // bitwise-equal (p, U0, dU)
        const bool e_ok = tid < nvalid;
        const bool same =
            e_ok && tid > 0 && pax[tid - 1] == pax[tid] && U0[tid - 1] == U0[tid] && dU[tid - 1] == dU[tid];
        int st = (e_ok && !same) ? tid : -1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(st, off, 64);
            if (lane >= off) st = max(st, o);
        }
        // carry across waves: latest head position of each earlier wave; boundary masks for lengths
        const bool bnd = !(e_ok && same);  // a run head, or an entry past the valid ones
        const unsigned long long bmask = __ballot(bnd);
        if (lane == 63) start[wave] = st;
        if (lane == 0) {
            masks[2 * wave] = (int)(bmask & 0xffffffffull);
            masks[2 * wave + 1] = (int)(bmask >> 32);
        }
        __syncthreads();
        int carry = -1;
        for (int w = 0; w < wave; ++w) carry = max(carry, start[w]);
        // run length of a head: distance to the next boundary after it
        int len = 0;
        if (e_ok && !same) {
            int w = wave;
            unsigned long long mk = (lane == 63) ? 0ull : (bmask & (~0ull << (lane + 1)));
            int nxt = B;
            while (true) {
                if (mk) {
                    nxt = w * 64 + __ffsll((long long)mk) - 1;
                    break;
                }
                if (++w >= B / 64) break;
                mk = ((unsigned long long)(unsigned)masks[2 * w + 1] << 32) | (unsigned)masks[2 * w];
            }
            len = nxt - tid;
        }
        __syncthreads();
        if (e_ok && same && st < 0) st = carry;
        if (!e_ok) st = -1;
        start[tid] = st;
        cnt[tid] = len;
        __syncthreads();
        // a run goes to the sheet if it is long, or if it continues the current sheet's line
        auto sheet_run = [&](int h) {
            if (!sheets || cnt[h] == 0 || pax[h] == 2 || g.n[pax[h]] > B) return false;
            if (cnt[h] >= kRunMin) return true;
            return sh_on && pax[h] == sh_p && U0[h] == sh_U0 && dU[h] == sh_dU;
        };
        const bool in_sheet = ok && sheet_run(start[cp]);
        // parallel compaction of the sheet-run heads (in order): ballot + prefix popcount
        {
            const bool f = sheet_run(tid);
            const unsigned long long bal = __ballot(f);
            if (lane == 0) list[B + 4 + wave] = __popcll(bal);
            __syncthreads();
            int off = 0, total = 0;
            for (int w = 0; w < B / 64; ++w) {
                const int c_w = list[B + 4 + w];
                off += (w < wave) ? c_w : 0;
                total += c_w;
            }
            if (f) list[off + __popcll(bal & ((1ull << lane) - 1ull))] = tid;
            if (tid == 0) list[B] = total;
        }
        // direct path for the other rays: wave-synchronous, run-combined atomics
        {
            const bool d = ok && !in_sheet;
            const int dlo = d ? r.k_lo : (1 << 30), dhi = d ? r.k_hi : -(1 << 30);
            const int k0 = wave_min(dlo), k1 = wave_max(dhi);
            for (int k = k0; k <= k1; ++k) {
                const bool act = k >= dlo && k <= dhi;
                Stencil stn{};
                float v = 0.0f;
                if (act) {
                    stn = stencil_at(r, k);
                    v = m.sample(fma((double)k, r.ds, r.s0), cv, ax);
                }
                wave_stencil_scatter(img, act && v != 0.0f, r, stn, v);
            }
        }
        __syncthreads();
        const int n_long = list[B];
        for (int li = 0; li < n_long; ++li) {
            const int h = list[li];
            const bool same_line = sh_on && pax[h] == sh_p && U0[h] == sh_U0 && dU[h] == sh_dU;
            if (sh_on && !same_line) {
                sheet_flush(img, col, g, sh_p, sh_U0, sh_dU, touched, zlo, zhi, nw, cs, tl, masks);
                touched = false;
                zlo = INT_MAX;
                zhi = INT_MIN;
                __syncthreads();
                sh_on = false;
            }
            if (!sh_on) {
                sh_on = true;
                sh_p = pax[h];
                sh_U0 = U0[h];
                sh_dU = dU[h];
                sh_kmax = g.n[sh_p] - 1;
            }
            // thread tid accumulates the column of absolute plane k = tid.  Each wave walks the run's
            // rays whose plane window meets its 64 planes, one ray per step (evaluating 2 or 4 rays
            // per step measured slower), and the current pair of z entries stays in registers until
            // z changes.
            const int k = tid;
            const int len = cnt[h];
            const bool kin = k <= sh_kmax;
            int jc = kNoEntry;
            float accA = 0.0f, accB = 0.0f;
            float preA = 0.0f, preB = 0.0f;  // column values of the pair jc, read when z moved to it
            // the column this thread writes: its own plane's, or for threads past the line's last plane
            // the unused last column (cs - 1 is never a plane of a sheet line), whose spare-row entry
            // takes their (zero) write-backs
            const int kc = kin ? k : cs - 1;
            // byte offsets into the column buffer of the pair's two entries (rows col_row(jc) and
            // col_row(jc + 1)), recomputed from jc on every step
            typedef __attribute__((address_space(3))) char lds_char;
            typedef __attribute__((address_space(3))) float lds_float;
            lds_char* colb = (lds_char*)col;
            // LDS byte addresses (the buffer's own address folded into the per-thread term, so that
            // an address is one multiply-add of the row)
            const unsigned cs4 = 4u * (unsigned)cs;
            const unsigned kc4 = 4u * (unsigned)kc + (unsigned)(uintptr_t)colb;
            auto row_off = [&](int j) { return (int)(__umul24((unsigned)col_row(j, nw), cs4) + kc4); };
            auto at = [&](int addr) { return (lds_float*)(uintptr_t)(unsigned)addr; };
            int ia = row_off(nw), ib = ia;
            for (int b0 = h; b0 < h + len; b0 += 64) {
                const int nb = min(64, h + len - b0);
                const int qlh = lohi[b0 + min(lane, nb - 1)];
                // rays whose plane window meets this wave's 64 planes (wave-uniform bit mask)
                const int kw0 = wave * 64, kw1 = min(kw0 + 63, sh_kmax);
                unsigned long long todo =
                    __ballot(lane < nb && (qlh & 0xffff) <= kw1 && (qlh >> 16) >= kw0);
                if (!todo) continue;
                // Each ray's parameters are read from LDS at a wave-uniform address (a broadcast,
                // no bank conflict), one ray ahead of its evaluation so that the read latency
                // overlaps the current ray's arithmetic; two records alternate (no copies).
                struct Rec {
                    double W0, dW, s0, ds;
                    float cv;
                    int ax, lh;
                };
                auto load = [&](int e) {
                    return Rec{W0[e], dW[e], s0[e], ds[e], cvs[e], aux[e], lohi[e]};
                };
                auto next = [&](int fallback) {
                    const int en = todo ? b0 + __ffsll((long long)todo) - 1 : fallback;
                    todo &= todo - 1ull;
                    return en;
                };
                // Every step writes the current pair back (its column values plus what the previous
                // step added) and reads the pair of this step's z -- the same pair again when z did not
                // change or the lane contributes nothing.  The same LDS accesses on every step and no
                // branch: the wait for a pair's values comes a whole step after their read, at the next
                // write-back, and the record loads of the next rays are never held up behind a read
                // issued late in a step.  (A write-back followed by the read of an overlapping pair is
                // seen by that read: one wave's LDS accesses complete in order.)
                auto step = [&](const Rec& c) {
                    const bool act = kin && k >= (c.lh & 0xffff) && k <= (c.lh >> 16);
                    const double W = fma((double)k, c.dW, c.W0);
                    const double fj = floor(W);
                    const int j0 = (int)fj;
                    const float fw = (float)(W - fj);
                    const float v0 = m.sample(fma((double)k, c.ds, c.s0), c.cv, Mode::kAux ? c.ax : 0);
                    const float v = act ? v0 : 0.0f;
                    *at(ia) = preA + accA;
                    *at(ib) = preB + accB;
                    const bool move = v != 0.0f && j0 != jc;
                    jc = move ? j0 : jc;
                    zlo = move ? min(zlo, j0) : zlo;
                    zhi = move ? max(zhi, j0 + 1) : zhi;
                    ia = row_off(jc);
                    ib = row_off(jc + 1);
                    preA = *at(ia);
                    preB = *at(ib);
                    accA = (1.0f - fw) * v;
                    accB = fw * v;
                };
                // A compiler-only barrier after each prefetch keeps the loads where they are: the
                // column accesses of step() are float and the records double / int, so without it the
                // compiler may sink the loads to their first use and wait on them there.
                int e = next(0);
                Rec ra = load(e);
                asm volatile("" ::: "memory");
                {   // a step without a ray (write the pair back, read it again): the LDS accesses
                    // entering the loop then follow the same pattern as from one step to the next,
                    // so the waits at the top of the loop are as exact as inside it
                    volatile lds_float* va = at(ia);
                    volatile lds_float* vb = at(ib);
                    *va = preA + accA;
                    *vb = preB + accB;
                    preA = *va;
                    preB = *vb;
                    accA = 0.0f;
                    accB = 0.0f;
                }
                while (true) {
                    bool more = todo != 0ull;
                    e = next(e);
                    const Rec rb = load(e);
                    asm volatile("" ::: "memory");
                    step(ra);
                    if (!more) break;
                    more = todo != 0ull;
                    e = next(e);
                    ra = load(e);
                    asm volatile("" ::: "memory");
                    step(rb);
                    if (!more) break;
                }
            }
            *at(ia) = preA + accA;
            *at(ib) = preB + accB;
            touched = touched || jc != kNoEntry;  // jc may be an out-of-grid entry after writes
            // no barrier between runs: a run writes only the thread's own column; other threads read
            // the columns only in a flush, whose first barrier follows every wave's last write here
        }
    }
    if (sh_on) sheet_flush(img, col, g, sh_p, sh_U0, sh_dU, touched, zlo, zhi, nw, cs, tl, masks);
    __syncthreads();  // the LDS may be reused by the caller
}

template <class Mode>
__global__ void __launch_bounds__(kSheetBlock) k_back_runs(Mode m, RaySrc src, int64_t n, GeomK g,
                                                          float* __restrict__ img, const int32_t* __restrict__ order,
                                                          int nw_lds, int groups) {
    extern __shared__ double smem[];
    const int64_t chunk0 = (int64_t)blockIdx.x * groups * kSheetBlock;
    back_runs_chunk(m, src, n, g, img, order, nw_lds, groups, chunk0, smem);
}

}  // namespace ppmi
