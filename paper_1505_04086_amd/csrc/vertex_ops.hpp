// vertex_ops.hpp -- the per-vertex work of a colouring round, in three shapes
// chosen by degree: a group of kGroup lanes, one wavefront, or one workgroup
// per vertex.
//
// Every shape computes, for vertex v with row [b, e) of col_idx:
//   * detection (the test of Algorithm 3, Section 3): does a neighbour u != v
//     that v loses to (by the tie rule) hold v's colour?
//   * First-Fit (Algorithm 1, Section 2.1): the smallest colour absent among
//     all neighbours u != v.  Colours < 0 (uncoloured) are ignored.  Since v
//     has at most e-b neighbours, the answer is at most e-b, so a window of
//     colours [base, base+W) with W > e-b always contains it.
// Phase kAssign computes First-Fit only; kRecolor detects and, if defective,
// computes First-Fit; kDetect only detects.  A vertex whose own colour is
// negative or above its degree counts as defective (only a recolouring that
// starts from a given colouring meets one).
#pragma once

#include <limits.h>

#include "device_common.hpp"

namespace rsoc {

// ------------------------------------------------------------ lane group --
// Rows of at most kThreadBinMax entries.  The G lanes of a group first load
// the whole row (load_row: one aligned 16-byte piece per lane), then gather neighbour colours from the byte-wide colour shadow col8
// (min(colour, 255); 255 also marks "uncoloured").  A thread-bin vertex has a
// colour <= its degree < 64, so only shadow values < 64 can equal it or block
// its First-Fit, and the byte shadow loses nothing.  In detect phases only
// the neighbours v loses to are gathered first; the rest only when v turns out
// defective.  The forbidden set is one 64-bit mask OR-reduced over the group.
// Every lane of the group gets the same result.
// NV vertices per group are handled together so that their loads overlap.
// In kAssign, WIN_ONLY restricts First-Fit to the neighbours v loses to plus
// the neighbours it wins against whose id lies within `look` of v's (those
// the sweep may already have coloured); unc[i] gets one bit per row position
// (bit p for row entry b+p) of the neighbours v loses to that were still
// uncoloured when read (zero: none was).  When keep is given (kAssign only),
// keep[i] = {ids of the first three such neighbours (-1 past the last), unc[i]}.
// ci[i] / col8[i] / col4[i] are the (per-graph) bases vertex i's ids refer to.
//
// NIB: colours are first read from a 4-bit shadow (eight vertices per 32-bit
// word): 0..13 are the colour, 14 means "coloured, 14 or more", 15 "not
// coloured yet" in round 0 and "consult the byte shadow" after it (a vertex
// recoloured later gets 15 back).  Where exact[s] is set, 14 and 15 fall back
// to the byte shadow; elsewhere they read as uncoloured (255), except that
// with `big` a 14 is settled from the byte shadow too (round 0 after the
// hub-first pass: a hub among the neighbours v wins against must be seen).
// The 4-bit array is half the size of the byte one, so far more of it stays
// in each XCD's L2 under random gathers.
// Colour reads are agent-scope relaxed loads: a kernel that colours in place
// must not be served a line its compute unit's L1 cached before another
// compute unit wrote the colour (a stale "uncoloured" costs conflicts).
__device__ __forceinline__ uint32_t colour_word(const RSOC_GLOBAL uint32_t *p) {
    return __hip_atomic_load((const uint32_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int colour_byte(const RSOC_GLOBAL uint8_t *p) {
    return (int)__hip_atomic_load((const uint8_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool NIB, int S>
__device__ __forceinline__ void gather_colours(const int (&u)[S], const bool (&take)[S], const bool (&exact)[S],
                                               const RSOC_GLOBAL uint8_t *col8, const RSOC_GLOBAL uint32_t *col4,
                                               int (&out)[S], bool big = false) {
    if (!NIB) {
#pragma unroll
        for (int s = 0; s < S; ++s) out[s] = take[s] ? colour_byte(col8 + u[s]) : 255;
        return;
    }
    uint32_t w[S];
#pragma unroll
    for (int s = 0; s < S; ++s) w[s] = take[s] ? colour_word(col4 + (u[s] >> 3)) : 0xffffffffu;
#pragma unroll
    for (int s = 0; s < S; ++s) out[s] = (int)((w[s] >> ((u[s] & 7) << 2)) & 15u);
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (out[s] >= 14) out[s] = (take[s] && (exact[s] || (big && out[s] == 14))) ? colour_byte(col8 + u[s]) : 255;
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (!take[s]) out[s] = 255;
}

template <bool NIB, int S>
__device__ __forceinline__ void gather_colours(const int (&u)[S], const bool (&take)[S],
                                               const RSOC_GLOBAL uint8_t *col8, const RSOC_GLOBAL uint32_t *col4,
                                               int (&out)[S]) {
    gather_colours<NIB, S>(u, take, take, col8, col4, out);
}

// Row layout in a lane group (G = 8 lanes, rows of at most 32 entries): the
// row [b, e) is read as the 16-byte-aligned pieces that overlap it.  With
// off = (address of row entry 0 / 4) mod 4, lane k loads piece k of the
// 128-byte window that starts off entries before the row (slots 0..3 = row
// positions 4k - off .. 4k - off + 3), and lanes k < off load row position
// 32 + k - off into slot 4 when the row reaches past the window.  A piece is
// loaded only if it holds an entry of the row, so no load leaves the pages
// the row occupies.  One instruction fetches the whole row (one or two cache
// lines) instead of one per slot.
constexpr int kRowSlots = 5;

template <int G>
__device__ __forceinline__ void load_row(int v, int b, int e, const RSOC_GLOBAL int32_t *ci, int (&u)[kRowSlots],
                                         int (&pos)[kRowSlots], int &off) {
    static_assert(G == 8, "row layout assumes 8 lanes of 4 entries");
    typedef int v4i __attribute__((ext_vector_type(4)));
    const int k = lane_id() & (G - 1);
    const int deg = e - b;
    const RSOC_GLOBAL int32_t *row = ci + b;
    off = (int)(((uintptr_t)row >> 2) & 3);
    const RSOC_GLOBAL int32_t *win = row - off;
    const int p0 = 4 * k - off;
    v4i q = {v, v, v, v};
    if (p0 + 3 >= 0 && p0 < deg) q = __builtin_nontemporal_load((const RSOC_GLOBAL v4i *)win + k);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        pos[s] = p0 + s;
        u[s] = (pos[s] >= 0 && pos[s] < deg) ? q[s] : v;
    }
    pos[4] = 32 + k - off;
    u[4] = (pos[4] < deg) ? __builtin_nontemporal_load(win + 32 + k) : v;
}

template <int PHASE, int TIE, int G, int S, bool WIN_ONLY, int NV, bool NIB = false>
__device__ __forceinline__ void group_vertices(const int (&v)[NV], const int (&b)[NV], const int (&e)[NV],
                                               const RSOC_GLOBAL int32_t *const (&ci)[NV],
                                               const RSOC_GLOBAL uint8_t *const (&col8)[NV], const int (&cv)[NV],
                                               int look, int (&newc)[NV], bool (&act)[NV], uint32_t (&unc)[NV],
                                               const RSOC_GLOBAL uint32_t *const *col4 = nullptr,
                                               int (*keep)[4] = nullptr, bool big = false) {
    static_assert(G == 8 && S == 4, "rows of at most 32 entries over 8 lanes");
    constexpr int T = kRowSlots;
    int u[NV][T], pos[NV][T], off[NV];
    int cu[NV][T];
#pragma unroll
    for (int i = 0; i < NV; ++i) load_row<G>(v[i], b[i], e[i], ci[i], u[i], pos[i], off[i]);
    if (PHASE != kAssign) {
        bool def[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            bool w[T];
#pragma unroll
            for (int s = 0; s < T; ++s) w[s] = (u[i][s] != v[i]) && loses<TIE>(v[i], u[i][s]);
            gather_colours<NIB, T>(u[i], w, col8[i], NIB ? col4[i] : nullptr, cu[i]);
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            bool c = false;
#pragma unroll
            for (int s = 0; s < T; ++s) c |= (cu[i][s] == cv[i]);
            // a vertex without a valid First-Fit colour (none, shadow 255, or
            // one above its degree; only a recolouring from a given colouring
            // meets such a vertex) is defective too
            def[i] = group_any<G>(c) || (v[i] >= 0 && cv[i] > e[i] - b[i]);
            act[i] = def[i];
        }
        if (PHASE == kDetect) return;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            bool rest[T];
            int c2[T];
#pragma unroll
            for (int s = 0; s < T; ++s) rest[s] = def[i] && u[i][s] != v[i] && !loses<TIE>(v[i], u[i][s]);
            gather_colours<NIB, T>(u[i], rest, col8[i], NIB ? col4[i] : nullptr, c2);
#pragma unroll
            for (int s = 0; s < T; ++s)
                if (rest[s]) cu[i][s] = c2[s];
        }
    } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            bool take[T], win[T];
#pragma unroll
            for (int s = 0; s < T; ++s) {
                win[s] = (u[i][s] != v[i]) && loses<TIE>(v[i], u[i][s]);
                const int dist = u[i][s] > v[i] ? u[i][s] - v[i] : v[i] - u[i][s];
                take[s] = WIN_ONLY ? (win[s] || (u[i][s] != v[i] && dist < look)) : (u[i][s] != v[i]);
            }
            // a nibble of 14 or 15 is settled from the byte shadow for every
            // neighbour of a First-Fit over all of them, and in round 0
            // (WIN_ONLY) for the neighbours v loses to: otherwise every such
            // neighbour with a colour of 14 or more, or coloured but not yet
            // published, would look uncoloured and send v to U^0.  Round 0
            // reads the others only as far as the nibble tells (their colours
            // are optional to it; after the hub-first pass a 14 is settled,
            // for the hubs)
            bool exact[T];
#pragma unroll
            for (int s = 0; s < T; ++s) exact[s] = WIN_ONLY ? win[s] : take[s];
            gather_colours<NIB, T>(u[i], take, exact, col8[i], NIB ? col4[i] : nullptr, cu[i], big);
            uint32_t bits = 0;
#pragma unroll
            for (int s = 0; s < T; ++s)
                if (win[s] && cu[i][s] == 255) bits |= 1u << pos[i][s];
            const uint32_t um = group_or32<G>(bits);
            unc[i] = um;
            act[i] = true;
            if (keep) {
                // row position p sits in window entry q = p + off: slot q % 4
                // of lane q / 4, or slot 4 of lane q - 32 past the window
                const int g0 = lane_id() & ~(G - 1);
                uint32_t mm = um;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int q = (mm ? __builtin_ctz(mm) : 0) + off[i];
                    mm &= mm - 1;
                    const int slot = q < 32 ? (q & 3) : 4;
                    int cand = u[i][0];
#pragma unroll
                    for (int s = 1; s < T; ++s) cand = (slot == s) ? u[i][s] : cand;
                    const int got = __shfl(cand, g0 + (q < 32 ? (q >> 2) : q - 32));
                    keep[i][j] = (j < __popc(um)) ? got : -1;
                }
                keep[i][3] = (int)um;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        uint64_t mask = 0;
#pragma unroll
        for (int s = 0; s < T; ++s) mask |= (cu[i][s] < 64) ? (1ull << cu[i][s]) : 0ull;
        mask = group_or64<G>(mask);
        newc[i] = (int)__builtin_ctzll(~mask);
    }
}

// Detection of the first worklist round after the pruned round 0, one lane per
// vertex, for a v with at most three kept neighbours.  x is what round 0 kept
// for v: the ids of the neighbours v loses to that were uncoloured when read
// (x.x, x.y, x.z; -1 past the last) and in x.w their row positions (see
// group_vertices).  Every other neighbour v loses to was already coloured
// when v chose its colour, so v's First-Fit avoided that colour, and neither
// has been recoloured since: only the kept neighbours can hold v's colour.
template <bool NIB>
__device__ __forceinline__ bool lane_detect_kept(int v, int4 x, int cv, const RSOC_GLOBAL uint8_t *col8,
                                                 const RSOC_GLOBAL uint32_t *col4) {
    const int cnt = __popc((uint32_t)x.w);
    int u[3] = {x.x, x.y, x.z}, cu[3];
    bool t[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        t[s] = s < cnt;
        if (!t[s]) u[s] = v;
    }
    gather_colours<NIB, 3>(u, t, col8, col4, cu);
    bool def = false;
#pragma unroll
    for (int s = 0; s < 3; ++s) def |= t[s] && cu[s] == cv;
    return def;
}

// Colours of long rows (wavefront and workgroup shapes) are gathered from the
// byte shadow col8 (min(colour, 255); 4 bytes per vertex less to pull through
// L2 than col), and from col only where the shadow saturates (255: uncoloured,
// or 255 and above).  Entries with take[s] false read as uncoloured (-1).
// LOOSE (round 0 over the neighbours v loses to, optimistic): a saturated
// shadow reads as uncoloured without the second load.  Round 0 may read any
// neighbour before it is coloured, so this is one of its interleavings: First-Fit
// ignores that neighbour and, if v loses to it, v enters U^0 with it.
template <bool LOOSE, int U>
__device__ __forceinline__ void hub_gather(const int (&u)[U], const bool (&take)[U], const RSOC_GLOBAL int32_t *col,
                                           const RSOC_GLOBAL uint8_t *col8, int (&x)[U]) {
    int y[U];
#pragma unroll
    for (int s = 0; s < U; ++s) y[s] = take[s] ? (int)col8[u[s]] : -1;
#pragma unroll
    for (int s = 0; s < U; ++s) x[s] = (y[s] == 255) ? (LOOSE ? -1 : col[u[s]]) : y[s];
}

// The same, except that entries with exact[s] are read from col directly (one
// exact load, -1 when uncoloured), whatever LOOSE says: round 0 after the
// hub-first pass must see every hub's colour, also one of 255 or more.
template <bool LOOSE, int U>
__device__ __forceinline__ void hub_gather(const int (&u)[U], const bool (&take)[U], const bool (&exact)[U],
                                           const RSOC_GLOBAL int32_t *col, const RSOC_GLOBAL uint8_t *col8,
                                           int (&x)[U]) {
    int y[U];
#pragma unroll
    for (int s = 0; s < U; ++s) y[s] = take[s] ? (exact[s] ? col[u[s]] : (int)col8[u[s]]) : -1;
#pragma unroll
    for (int s = 0; s < U; ++s) x[s] = (!exact[s] && y[s] == 255) ? (LOOSE ? -1 : col[u[s]]) : y[s];
}

// Round 0 after the hub-first pass (optimistic): entries with up[s] (the
// neighbours v wins against, which round 0 reads only for the hubs' sake) are
// read from the 4-bit shadow first: 15 (not coloured yet) reads as
// uncoloured, 0..13 are the colour, and 14 (14 or more: every hub of such a
// colour) is settled from the byte shadow and, where that saturates, from
// col.  The other taken entries are read as hub_gather<LOOSE> reads them.
template <bool LOOSE, int U>
__device__ __forceinline__ void hub_gather_up(const int (&u)[U], const bool (&take)[U], const bool (&up)[U],
                                              const RSOC_GLOBAL int32_t *col, const RSOC_GLOBAL uint8_t *col8,
                                              const RSOC_GLOBAL uint32_t *col4, int (&x)[U]) {
    int y[U];
#pragma unroll
    for (int s = 0; s < U; ++s)
        y[s] = take[s] ? (up[s] ? (int)((colour_word(col4 + (u[s] >> 3)) >> ((u[s] & 7) << 2)) & 15u)
                                : (int)col8[u[s]])
                       : -1;
#pragma unroll
    for (int s = 0; s < U; ++s) {
        if (up[s] && take[s]) y[s] = y[s] == 15 ? -1 : (y[s] == 14 ? (int)col8[u[s]] : y[s]);
        else if (take[s] && y[s] == 255) y[s] = LOOSE ? -1 : 255;
    }
#pragma unroll
    for (int s = 0; s < U; ++s) x[s] = (take[s] && y[s] == 255) ? col[u[s]] : y[s];
}

// Row entries each lane of a wavefront or workgroup holds per step: all the
// loads of a step are in flight together, and so are its gathers.
constexpr int kWaveSlots = 8;
constexpr int kBlockSlots = 8;

// ------------------------------------------------------------- wavefront --
// One wavefront per vertex: lanes stride the row kWaveSlots entries at a time;
// forbidden colours go into an LDS bitmap window of kWaveWindowBits bits.
// Rows of at most kWaveSlots * kWave entries (every row of the default bins)
// are read once: the detection keeps the row and the colours it gathered, and
// the recolouring gathers only the remaining neighbours' colours.  Its colour
// is at most its degree, below the window, so one window pass settles it.
template <int PHASE, int TIE, bool WIN_ONLY>
__device__ __forceinline__ bool wave_vertex(int v, int b, int e, const RSOC_GLOBAL int32_t *ci,
                                            const RSOC_GLOBAL int32_t *col, const RSOC_GLOBAL uint8_t *col8,
                                            uint32_t *bm, int look, int &newc, bool &unc_win, bool exact_up = false,
                                            const RSOC_GLOBAL uint32_t *col4 = nullptr) {
    const int lane = lane_id();
    constexpr int U = kWaveSlots;
    constexpr bool kLoose = PHASE == kAssign && WIN_ONLY;
    static_assert(kWaveSlots * kWave <= kWaveWindowBits, "a one-step row must fit the window");
    if (e - b <= U * kWave) {
        int u[U], x[U];
        bool w[U];
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const int j = b + s * kWave + lane;
            u[s] = (j < e) ? __builtin_nontemporal_load(ci + j) : v;
        }
#pragma unroll
        for (int s = 0; s < U; ++s) w[s] = (u[s] != v) && loses<TIE>(v, u[s]);
        if (PHASE != kAssign) {
            const int cv = col[v];
            hub_gather<false, U>(u, w, col, col8, x);
            bool c = false;
#pragma unroll
            for (int s = 0; s < U; ++s) c |= w[s] && x[s] == cv;
            const bool any = cv < 0 || cv > e - b || ballot(c) != 0;
            if (!any) return false;
            if (PHASE == kDetect) return true;
            bool r[U];
            int x2[U];
#pragma unroll
            for (int s = 0; s < U; ++s) r[s] = (u[s] != v) && !w[s];
            hub_gather<false, U>(u, r, col, col8, x2);
#pragma unroll
            for (int s = 0; s < U; ++s)
                if (r[s]) x[s] = x2[s];
        } else {
            bool take[U], ex[U];
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int dist = u[s] > v ? u[s] - v : v - u[s];
                take[s] = WIN_ONLY ? (w[s] || (u[s] != v && dist < look)) : (u[s] != v);
                ex[s] = exact_up && take[s] && !w[s];
            }
            if (exact_up) hub_gather_up<kLoose, U>(u, take, ex, col, col8, col4, x);
            else hub_gather<kLoose, U>(u, take, col, col8, x);
            bool unc = false;
#pragma unroll
            for (int s = 0; s < U; ++s) unc |= w[s] && x[s] < 0;
            unc_win = ballot(unc) != 0;
        }
        for (int q = lane; q < kWaveWindowWords; q += kWave) bm[q] = 0u;
        wave_lds_sync();
#pragma unroll
        for (int s = 0; s < U; ++s)
            if (x[s] >= 0 && x[s] < kWaveWindowBits) lds_or(&bm[x[s] >> 5], 1u << (x[s] & 31));
        wave_lds_sync();
        // at most e - b <= kWaveSlots * kWave bits are set, so a clear one
        // lies within the first kWave words
        const uint32_t word = bm[lane];
        const uint64_t m = ballot(word != 0xffffffffu);
        const int l = __ffsll((unsigned long long)m) - 1;
        const uint32_t wl = __shfl(word, l);
        newc = l * 32 + __builtin_ctz(~wl);
        wave_lds_sync();
        return true;
    }
    // longer rows (a wavefront bin raised past kWaveSlots * kWave): one pass
    // for the detection, then a pass per colour window
    bool unc = false;
    if (PHASE != kAssign) {
        const int cv = col[v];
        bool any = cv < 0 || cv > e - b;  // no valid First-Fit colour: defective
        for (int j0 = b; j0 < e && !any; j0 += U * kWave) {
            int u[U], x[U];
            bool w[U];
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int j = j0 + s * kWave + lane;
                u[s] = (j < e) ? __builtin_nontemporal_load(ci + j) : v;
            }
#pragma unroll
            for (int s = 0; s < U; ++s) w[s] = (u[s] != v) && loses<TIE>(v, u[s]);
            hub_gather<false, U>(u, w, col, col8, x);
            bool c = false;
#pragma unroll
            for (int s = 0; s < U; ++s) c |= w[s] && x[s] == cv;
            any = ballot(c) != 0;
        }
        if (!any) return false;
        if (PHASE == kDetect) return true;
    }
    for (int base = 0;; base += kWaveWindowBits) {
        for (int q = lane; q < kWaveWindowWords; q += kWave) bm[q] = 0u;
        wave_lds_sync();
        for (int j0 = b; j0 < e; j0 += U * kWave) {
            int u[U], x[U];
            bool take[U], w[U], ex[U];
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int j = j0 + s * kWave + lane;
                u[s] = (j < e) ? __builtin_nontemporal_load(ci + j) : v;
            }
#pragma unroll
            for (int s = 0; s < U; ++s) {
                w[s] = (u[s] != v) && loses<TIE>(v, u[s]);
                const int dist = u[s] > v ? u[s] - v : v - u[s];
                take[s] = (PHASE == kAssign && WIN_ONLY) ? (w[s] || (u[s] != v && dist < look)) : (u[s] != v);
                ex[s] = PHASE == kAssign && exact_up && take[s] && !w[s];
            }
            if (PHASE == kAssign && exact_up) hub_gather_up<kLoose, U>(u, take, ex, col, col8, col4, x);
            else hub_gather<kLoose, U>(u, take, col, col8, x);
#pragma unroll
            for (int s = 0; s < U; ++s) {
                if (PHASE == kAssign) unc |= w[s] && x[s] < 0;
                const int rel = x[s] - base;
                if (x[s] >= 0 && (unsigned)rel < (unsigned)kWaveWindowBits) lds_or(&bm[rel >> 5], 1u << (rel & 31));
            }
        }
        if (PHASE == kAssign) unc_win = ballot(unc) != 0;
        wave_lds_sync();
        for (int w0 = 0; w0 < kWaveWindowWords; w0 += kWave) {
            const uint32_t word = bm[w0 + lane];
            const uint64_t m = ballot(word != 0xffffffffu);
            if (m) {
                const int l = __ffsll((unsigned long long)m) - 1;
                const uint32_t wl = __shfl(word, l);
                newc = base + (w0 + l) * 32 + __builtin_ctz(~wl);
                wave_lds_sync();
                return true;
            }
        }
        wave_lds_sync();
    }
}

// -------------------------------------------------------------- workgroup --
// One workgroup per vertex (hubs): threads stride the row kBlockSlots entries
// at a time, the conflict flag is a workgroup OR per step, forbidden colours
// go into an LDS bitmap window of kBlockWindowBits bits; the first clear word
// is found with an LDS atomicMin.  Must be called by the whole workgroup;
// newc valid in every thread.
template <int PHASE, int TIE, bool WIN_ONLY>
__device__ __forceinline__ bool block_vertex(int v, int b, int e, const RSOC_GLOBAL int32_t *ci,
                                             const RSOC_GLOBAL int32_t *col, const RSOC_GLOBAL uint8_t *col8,
                                             uint32_t *bm, int *sh_min, int look, int &newc, bool &unc_win,
                                             bool exact_up = false, const RSOC_GLOBAL uint32_t *col4 = nullptr) {
    const int t = threadIdx.x;
    constexpr int U = kBlockSlots;
    constexpr bool kLoose = PHASE == kAssign && WIN_ONLY;
    bool unc = false;
    if (PHASE != kAssign) {
        const int cv = col[v];
        int any = cv < 0 || cv > e - b;  // no valid First-Fit colour: defective
        for (int j0 = b; j0 < e && !any; j0 += kBlock * U) {
            int u[U], x[U];
            bool w[U];
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int j = j0 + s * kBlock + t;
                u[s] = (j < e) ? __builtin_nontemporal_load(ci + j) : v;
            }
#pragma unroll
            for (int s = 0; s < U; ++s) w[s] = (u[s] != v) && loses<TIE>(v, u[s]);
            hub_gather<false, U>(u, w, col, col8, x);
            bool c = false;
#pragma unroll
            for (int s = 0; s < U; ++s) c |= w[s] && x[s] == cv;
            any = __syncthreads_or(c);
        }
        if (!any) return false;
        if (PHASE == kDetect) return true;
    }
    for (int base = 0;; base += kBlockWindowBits) {
        for (int q = t; q < kBlockWindowWords; q += kBlock) bm[q] = 0u;
        if (t == 0) *sh_min = INT_MAX;
        __syncthreads();
        for (int j0 = b; j0 < e; j0 += kBlock * U) {
            int u[U], x[U];
            bool take[U], w[U], ex[U];
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int j = j0 + s * kBlock + t;
                u[s] = (j < e) ? __builtin_nontemporal_load(ci + j) : v;
            }
#pragma unroll
            for (int s = 0; s < U; ++s) {
                w[s] = (u[s] != v) && loses<TIE>(v, u[s]);
                const int dist = u[s] > v ? u[s] - v : v - u[s];
                take[s] = (PHASE == kAssign && WIN_ONLY) ? (w[s] || (u[s] != v && dist < look)) : (u[s] != v);
                ex[s] = PHASE == kAssign && exact_up && take[s] && !w[s];
            }
            if (PHASE == kAssign && exact_up) hub_gather_up<kLoose, U>(u, take, ex, col, col8, col4, x);
            else hub_gather<kLoose, U>(u, take, col, col8, x);
#pragma unroll
            for (int s = 0; s < U; ++s) {
                if (PHASE == kAssign) unc |= w[s] && x[s] < 0;
                const int rel = x[s] - base;
                if (x[s] >= 0 && (unsigned)rel < (unsigned)kBlockWindowBits) lds_or(&bm[rel >> 5], 1u << (rel & 31));
            }
        }
        if (PHASE == kAssign) unc_win = __syncthreads_or(unc) != 0;
        __syncthreads();
        for (int q = t; q < kBlockWindowWords; q += kBlock)
            if (bm[q] != 0xffffffffu) { atomicMin(sh_min, q); break; }
        __syncthreads();
        const int q = *sh_min;
        if (q != INT_MAX) {
            newc = base + q * 32 + __builtin_ctz(~bm[q]);
            __syncthreads();
            return true;
        }
        __syncthreads();
    }
}

}  // namespace rsoc
