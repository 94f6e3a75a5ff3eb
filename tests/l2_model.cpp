// Cache model of the gather's image reads on one XCD, for the design analysis of the
// work order and the data layout (run by tests/test_l2_model_cpu.py).
//
// What each lane reads comes from running the kernels' own per-pixel code on the host
// (ssvb_pixel.h, the host build, with its read observer), with the frame constants and
// tables the library derives (fill_frame, fill_tables), and the work items from the
// kernels' own XCD runs, tile walk and tile -> pixel mapping (ssvb_internal.h).  A lane's
// reads are labelled with the load instruction that issues them: the centre depth and
// normal, then per slice and step the depth read of each side and, for a side whose
// sample covers new sectors, its normal read and (with a positive weight) its radiance
// read.  Timing is modelled: the XCD's 32 CUs each hold `wg_per_cu` workgroups of 4 waves;
// every resident wave issues its next load instruction in turn (round robin over the
// XCD's waves); a workgroup takes the next work item of the XCD's queue once its four
// waves are done.  An instruction's distinct 128-byte lines go to the CU's L1 (LRU, 32 KB)
// and its misses to the XCD's L2 (LRU, 16-way, 4 MB).  Output writes are not modelled.
//
// Orders: "strip" (the library's default), "interleaved" (strips 0, 8, 16, ... then 1, 9,
// ...), "slice<C>" (the library's slice-major order, ssvb_set_slice_order: work items are
// (tile, slice) pairs, for each chunk of C tiles of the XCD's run slice 0 of every tile,
// then slice 1, ...; the partial-sum writes and their reduction are not modelled),
// "pair<C>" (the same with two slices per work item),
// "block<X>x<Y>" (the tiles cut into an X x Y grid of blocks, one per XCD, each walked in
// vertical strips).  The replayed share is XCD 0's unless an XCD is named (a share at the
// frame's edge loses the samples that fall off it).  Layout "packed" puts a texel's normal
// and radiance in one 16-byte (FP16) or 32-byte (FP32) record, so one sample's two reads
// share a line.
// A layout suffix "+d<w>x<h>" (w h = 32, e.g. "planar+d8x4") stores depth in 2D blocks, a
// 128-byte line holding w x h texels instead of 32 texels of one row.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "ssvb_host.h"
#include "ssvb_pixel.h"

using namespace ssvb;

namespace {

// set index: the line number modulo the set count (plain address bits), or a
// multiplicative hash of it (sets used uniformly whatever the stride)
bool g_hash_sets = false;

struct SetAssoc {
    int sets, ways;
    std::vector<uint64_t> tag, stamp;
    uint64_t clock = 0, hits = 0, misses = 0;
    SetAssoc(int bytes, int line, int ways_) : sets(bytes / line / ways_), ways(ways_) {
        tag.assign((size_t)sets * ways, ~0ull);
        stamp.assign((size_t)sets * ways, 0);
    }
    bool access(uint64_t line) {
        const size_t s = g_hash_sets ? (size_t)((line * 0x9E3779B97F4A7C15ull) >> 40) % (size_t)sets
                                     : (size_t)(line % (uint64_t)sets);
        uint64_t* t = &tag[s * ways];
        uint64_t* st = &stamp[s * ways];
        ++clock;
        int victim = 0;
        for (int w = 0; w < ways; ++w) {
            if (t[w] == line) {
                st[w] = clock;
                ++hits;
                return true;
            }
            if (st[w] < st[victim]) victim = w;
        }
        t[victim] = line;
        st[victim] = clock;
        ++misses;
        return false;
    }
};

enum Kind { DEPTH = 0, NORMAL = 1, RADIANCE = 2 };

struct Read {
    uint32_t instr;  // load instruction of the lane's program
    uint8_t kind;
    uint64_t addr;   // byte address in a flat model space (kinds in disjoint ranges)
    int bytes;
};

// the lane being traced (the observer is a plain function pointer)
std::vector<Read>* g_reads = nullptr;
const char *g_depth = nullptr, *g_normal = nullptr, *g_radiance = nullptr;
size_t g_depth_bytes = 0, g_normal_bytes = 0, g_radiance_bytes = 0;

void observe(const void* p, int bytes) {
    const char* c = (const char*)p;
    Read r{0, 0, 0, bytes};
    if (c >= g_depth && c < g_depth + g_depth_bytes) {
        r.kind = DEPTH;
        r.addr = (uint64_t)(c - g_depth);
    } else if (c >= g_normal && c < g_normal + g_normal_bytes) {
        r.kind = NORMAL;
        r.addr = (1ull << 40) + (uint64_t)(c - g_normal);
    } else {
        r.kind = RADIANCE;
        r.addr = (2ull << 40) + (uint64_t)(c - g_radiance);
    }
    g_reads->push_back(r);
}

struct Config {
    int W, H, nd, ns, fp16;
    std::string order, layout;
    int chunk = 0;
    int per_item = 1;      // slices per work item in a slice-major order ("pair<C>": 2)
    int dlw = 0, dlh = 0;  // depth line shape in texels ("...+d<w>x<h>" layouts), 0: rows
};

// The reads of one pixel, labelled with their load instruction: 0 centre depth, 1 centre
// normal, then 2 + 3 ((i N_s + j) 2 + side) + kind.
std::vector<Read> trace_pixel(const FrameArgs& A, ExactLds& L, int x, int y) {
    std::vector<Read> rd;
    g_reads = &rd;
    if (A.normal_f16) gather_pixel<SSVB_HIT_ROUND, MODE_COMPUTE, false, 3, 32>(A, L, x, y, 0, 1, nullptr, nullptr);
    else gather_pixel<SSVB_HIT_ROUND, MODE_COMPUTE, false, 0, 32>(A, L, x, y, 0, 1, nullptr, nullptr);
    g_reads = nullptr;
    // label
    const int es = A.normal_f16 ? 2 : 4;
    int m = -1;          // index of the last sample depth read
    uint64_t tex[2] = {~0ull, ~0ull};  // texels of the current step's two depth reads
    for (size_t k = 0; k < rd.size(); ++k) {
        Read& r = rd[k];
        if (k == 0) {
            r.instr = 0;
            continue;
        }
        if (k == 1 && r.kind == NORMAL) {
            r.instr = 1;
            continue;
        }
        if (r.kind == DEPTH) {
            ++m;
            tex[m % 2] = r.addr / 4;
            const int i = m / (2 * A.ns), j = (m / 2) % A.ns, side = m % 2;
            r.instr = 2 + 3 * (uint32_t)((i * A.ns + j) * 2 + side);
            continue;
        }
        // a GI read: its texel is one of the step's two samples
        const uint64_t off = r.addr & ((1ull << 40) - 1);
        const uint64_t t = off / (uint64_t)(3 * es);
        const int side = t == tex[1] ? 1 : 0;
        const int step0 = m - (m % 2);  // the step's side-0 depth read
        const int i = step0 / (2 * A.ns), j = (step0 / 2) % A.ns;
        r.instr = 2 + 3 * (uint32_t)((i * A.ns + j) * 2 + side) + (r.kind == NORMAL ? 1 : 2);
    }
    return rd;
}

struct Model {
    const FrameArgs& A;
    const Config& C;
    SetAssoc L2{4 << 20, 128, 16};
    std::vector<SetAssoc> L1;
    uint64_t instrs[3] = {}, lines[3] = {}, l2_access[3] = {}, l2_miss[3] = {}, samples = 0;
    Model(const FrameArgs& a, const Config& c) : A(a), C(c) {
        for (int k = 0; k < 32; ++k) L1.emplace_back(32 << 10, 128, 64);
    }
    // the model-space address of a read under the layout
    void lines_of(const Read& r, uint64_t out[2], int& n) const {
        uint64_t a = r.addr;
        int bytes = r.bytes;
        if (r.kind == DEPTH && C.dlw > 0) {
            // depth in 2D blocks: one 128-byte line holds dlw x dlh texels (dlw * dlh = 32),
            // lines row-major over the grid of blocks
            const uint64_t t = r.addr / 4;
            const uint64_t x = t % (uint64_t)A.W, y = t / (uint64_t)A.W;
            const uint64_t bw = ((uint64_t)A.W + C.dlw - 1) / C.dlw;
            out[0] = (y / C.dlh) * bw + x / C.dlw;
            n = 1;
            return;
        }
        if (C.layout.rfind("packed", 0) == 0 && r.kind != DEPTH) {
            const int es = A.normal_f16 ? 2 : 4;
            const uint64_t t = (r.addr & ((1ull << 40) - 1)) / (uint64_t)(3 * es);
            const int rec = A.normal_f16 ? 16 : 32;
            a = (1ull << 40) + t * rec + (r.kind == RADIANCE ? rec / 2 : 0);
            bytes = 3 * es;
        }
        n = 0;
        for (uint64_t l = a >> 7; l <= (a + bytes - 1) >> 7; ++l) out[n++] = l;
    }
};

struct Lane {
    std::vector<Read> reads;
    size_t pos = 0;
};

struct Wave {
    std::vector<Lane> lanes;
    uint32_t slice_lo = 0, slice_hi = 0;  // instruction range of the item
    bool active = false;
};

uint32_t instr_lo(const FrameArgs& A, int s) { return 2 + 3 * (uint32_t)(s * A.ns * 2); }

// Issue wave w's next instruction on CU cu; false once it has none left.
bool issue(Model& M, Wave& w, int cu) {
    if (!w.active) return false;
    uint32_t next = ~0u;
    for (auto& l : w.lanes) {
        while (l.pos < l.reads.size() && l.reads[l.pos].instr < w.slice_lo && l.reads[l.pos].instr >= 2) ++l.pos;
        if (l.pos < l.reads.size() && l.reads[l.pos].instr < w.slice_hi) next = std::min(next, l.reads[l.pos].instr);
    }
    if (next == ~0u) {
        w.active = false;
        return false;
    }
    uint64_t lines[128];
    int nl = 0, kind = 0, active = 0;
    for (auto& l : w.lanes) {
        if (l.pos < l.reads.size() && l.reads[l.pos].instr == next) {
            const Read& r = l.reads[l.pos++];
            kind = r.kind;
            ++active;
            uint64_t ls[2];
            int n;
            M.lines_of(r, ls, n);
            for (int k = 0; k < n; ++k) {
                bool seen = false;
                for (int m = 0; m < nl; ++m) seen |= lines[m] == ls[k];
                if (!seen) lines[nl++] = ls[k];
            }
        }
    }
    M.instrs[kind]++;
    M.lines[kind] += (uint64_t)nl;
    if (kind == DEPTH && next >= 2) M.samples += (uint64_t)active;
    for (int m = 0; m < nl; ++m) {
        if (M.L1[cu].access(lines[m])) continue;
        M.l2_access[kind]++;
        if (!M.L2.access(lines[m])) M.l2_miss[kind]++;
    }
    return true;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 14) {
        fprintf(stderr, "usage: l2_model depth normal radiance W H fp16 slices steps radius thickness seed order fraction "
                        "[layout] [wg_per_cu] [hash|plain] [xcd] [r2|hash|fixed]\n");
        return 2;
    }
    Config C;
    C.W = atoi(argv[4]);
    C.H = atoi(argv[5]);
    C.fp16 = atoi(argv[6]);
    C.nd = atoi(argv[7]);
    C.ns = atoi(argv[8]);
    const float radius = (float)atof(argv[9]), thickness = (float)atof(argv[10]);
    const uint32_t seed = (uint32_t)strtoul(argv[11], nullptr, 10);
    C.order = argv[12];
    const double fraction = atof(argv[13]);
    C.layout = argc > 14 ? argv[14] : "planar";
    {
        const size_t at = C.layout.find("+d");
        if (at != std::string::npos && sscanf(C.layout.c_str() + at + 2, "%dx%d", &C.dlw, &C.dlh) == 2 &&
            C.dlw * C.dlh != 32) {
            fprintf(stderr, "a depth line holds 32 texels: %dx%d\n", C.dlw, C.dlh);
            return 2;
        }
    }
    const int wg_per_cu = argc > 15 ? atoi(argv[15]) : 4;
    g_hash_sets = argc > 16 && !strcmp(argv[16], "hash");
    const int xcd = argc > 17 ? atoi(argv[17]) : 0;  // which XCD's share to replay (0..7)
    const char* noise = argc > 18 ? argv[18] : "r2";   // r2 (the workloads'), hash or fixed
    if (C.order.rfind("slice", 0) == 0) C.chunk = atoi(C.order.c_str() + 5);
    if (C.order.rfind("pair", 0) == 0) C.chunk = atoi(C.order.c_str() + 4), C.per_item = 2;
    const size_t px = (size_t)C.W * C.H, es = C.fp16 ? 2 : 4;
    std::vector<char> depth(px * 4), normal(px * 3 * es), radiance(px * 3 * es);
    const char* files[3] = {argv[1], argv[2], argv[3]};
    std::vector<char>* bufs[3] = {&depth, &normal, &radiance};
    for (int k = 0; k < 3; ++k) {
        FILE* f = fopen(files[k], "rb");
        if (!f || fread(bufs[k]->data(), 1, bufs[k]->size(), f) != bufs[k]->size()) {
            fprintf(stderr, "cannot read %s\n", files[k]);
            return 2;
        }
        fclose(f);
    }
    g_depth = depth.data(), g_normal = normal.data(), g_radiance = radiance.data();
    g_depth_bytes = depth.size(), g_normal_bytes = normal.size(), g_radiance_bytes = radiance.size();
    std::vector<float> ao(px), gi(px * 3), amb(px * 3);
    static int2 lut[kLutSize];
    static double2 half[129], half128[513];
    fill_tables(lut, half, half128);
    FrameTables tab;
    tab.d_lut = lut;
    tab.d_half = half;
    tab.d_half128 = half128;
    ssvb_camera cam{C.W, C.H, 0.5f * C.H, 0.5f * C.H, 0.5f * C.W, 0.5f * C.H, {1, 0, 0, 0, 1, 0, 0, 0, 1}};
    ssvb_params p;
    ssvb_default_params(&p);
    p.slices = C.nd;
    p.steps = C.ns;
    p.radius = radius;
    p.thickness = thickness;
    p.noise = !strcmp(noise, "fixed") ? SSVB_NOISE_FIXED : !strcmp(noise, "hash") ? SSVB_NOISE_HASH : SSVB_NOISE_R2;
    p.seed = seed;
    const ssvb_dtype dt = C.fp16 ? SSVB_F16 : SSVB_F32;
    ssvb_image d{depth.data(), 0, SSVB_F32, 1}, n{normal.data(), 0, dt, 3}, r{radiance.data(), 0, dt, 3};
    ssvb_outputs o{ao.data(), gi.data(), amb.data(), nullptr, 0, 0, 0, 0};
    FrameArgs A;
    fill_frame(A, &tab, &d, &n, &r, &cam, &p, &o);
    host_read_observer = observe;
    static ExactLds L;

    const uint32_t nt = (uint32_t)A.tiles_x * (uint32_t)A.tiles_y;
    uint32_t first, count;
    xcd_run(nt, xcd, first, count);
    const uint32_t take = std::max<uint32_t>(1, (uint32_t)(count * fraction));
    struct Item {
        int tx, ty, slice;
    };
    std::vector<Item> items;
    auto tile_of = [&](uint32_t ord, int& tx, int& ty) {
        if (C.order == "interleaved") {
            const uint32_t S = (uint32_t)A.strip, TY = (uint32_t)A.tiles_y, TX = (uint32_t)A.tiles_x;
            const uint32_t nstrips = (TX + S - 1) / S, full = TX / S, wl = TX - full * S;
            uint32_t base = 0;
            for (uint32_t g = 0; g < (uint32_t)kXcds && g < nstrips; ++g) {
                const uint32_t in_group = (nstrips - g + kXcds - 1) / kXcds;
                uint32_t tiles = in_group * S * TY;
                if (wl != 0 && (nstrips - 1) % kXcds == g) tiles -= (S - wl) * TY;
                if (ord < base + tiles) {
                    const uint32_t rr0 = ord - base, st = g + (uint32_t)kXcds * (rr0 / (S * TY)), rr = rr0 % (S * TY);
                    const uint32_t width = (wl != 0 && st == nstrips - 1) ? wl : S;
                    ty = (int)(rr / width);
                    tx = (int)(st * S + rr % width);
                    return;
                }
                base += tiles;
            }
        }
        walk_tile(A, ord, tx, ty);
    };
    if (C.order.rfind("block", 0) == 0) {
        // the frame's tiles cut into a bx x by grid of blocks, one per XCD; this XCD's block
        // (the top-left one) walked in vertical strips of `strip` tiles, top to bottom
        int bx = 4, by = 2;
        sscanf(C.order.c_str() + 5, "%dx%d", &bx, &by);
        const int bw = (A.tiles_x + bx - 1) / bx, bh = (A.tiles_y + by - 1) / by, S = A.strip;
        const int x0 = (xcd % bx) * bw, y0 = (xcd / bx) * bh;  // this XCD's block
        const uint32_t in_block = (uint32_t)bw * (uint32_t)bh;
        const uint32_t tk = std::max<uint32_t>(1, (uint32_t)(in_block * fraction));
        for (uint32_t k = 0; k < tk; ++k) {
            const int strip = (int)(k / (uint32_t)(S * bh)), r = (int)(k % (uint32_t)(S * bh));
            const int w = std::min(S, bw - strip * S);
            const int tx = x0 + strip * S + r % w, ty = y0 + r / w;
            if (tx < A.tiles_x && ty < A.tiles_y) items.push_back({tx, ty, -1});
        }
    } else if (C.chunk > 0) {
        // the library's slice-major items (slice_item) over the replayed tiles of the run;
        // with two slices per item, item slice s stands for slices 2s and 2s + 1
        const int groups = (A.nd + C.per_item - 1) / C.per_item;
        for (uint32_t j = 0; j < take * (uint32_t)groups; ++j) {
            uint32_t tile;
            int s, tx, ty;
            slice_item((uint32_t)C.chunk, groups, take, j, tile, s);
            walk_tile(A, first + tile, tx, ty);
            items.push_back({tx, ty, s * C.per_item});
        }
    } else {
        for (uint32_t k = 0; k < take; ++k) {
            int tx, ty;
            tile_of(first + k, tx, ty);
            items.push_back({tx, ty, -1});
        }
    }
    // per-tile traces, kept while a tile has items in flight or ahead in its chunk
    std::map<std::pair<int, int>, std::vector<std::vector<Read>>> traces;
    std::map<std::pair<int, int>, int> uses;
    for (const Item& it : items) uses[{it.tx, it.ty}]++;
    auto tile_traces = [&](int tx, int ty) -> std::vector<std::vector<Read>>& {
        auto key = std::make_pair(tx, ty);
        auto f = traces.find(key);
        if (f != traces.end()) return f->second;
        auto& v = traces[key];
        v.resize(256);
        for (int t = 0; t < 256; ++t) {
            int x, y, li;
            tile_pixel(A, tx, ty, t, x, y, li);
            if ((unsigned)x < (unsigned)A.W && (unsigned)y < (unsigned)A.H) v[t] = trace_pixel(A, L, x, y);
        }
        return v;
    };
    Model M(A, C);
    const int nwg = 32 * wg_per_cu;
    std::vector<Wave> waves((size_t)nwg * 4);
    std::vector<std::pair<int, int>> wg_tile(nwg);
    size_t next = 0;
    auto start = [&](int g) {
        if (next >= items.size()) return false;
        const Item it = items[next++];
        auto& tr = tile_traces(it.tx, it.ty);
        for (int wv = 0; wv < 4; ++wv) {
            Wave& w = waves[(size_t)g * 4 + wv];
            w.lanes.clear();
            for (int l = 0; l < 64; ++l) {
                const auto& rd = tr[wv * 64 + l];
                if (rd.empty()) continue;
                w.lanes.push_back(Lane{rd, 0});
            }
            w.slice_lo = it.slice < 0 ? 0 : instr_lo(A, it.slice);
            w.slice_hi = it.slice < 0 ? ~0u : instr_lo(A, std::min(it.slice + C.per_item, A.nd));
            // a slice item after the first re-reads the centre depth and normal
            if (it.slice > 0)
                for (auto& l : w.lanes) l.pos = 0;
            w.active = !w.lanes.empty();
        }
        auto key = std::make_pair(it.tx, it.ty);
        if (--uses[key] == 0) wg_tile[g] = key;  // traces freed when this item is done
        else wg_tile[g] = {-1, -1};
        return true;
    };
    std::vector<bool> live(nwg, false);
    for (int g = 0; g < nwg; ++g) live[g] = start(g);
    bool any = true;
    while (any) {
        any = false;
        for (int g = 0; g < nwg; ++g) {
            if (!live[g]) continue;
            bool busy = false;
            for (int wv = 0; wv < 4; ++wv) busy |= issue(M, waves[(size_t)g * 4 + wv], g % 32);
            if (!busy) {
                if (wg_tile[g].first >= 0) traces.erase(wg_tile[g]);
                live[g] = start(g);
            }
            any |= live[g];
        }
    }
    host_read_observer = nullptr;
    const char* names[3] = {"depth", "normal", "radiance"};
    uint64_t acc = 0, miss = 0;
    printf("order %s layout %s tiles %u samples %llu\n", C.order.c_str(), C.layout.c_str(), take,
           (unsigned long long)M.samples);
    for (int k = 0; k < 3; ++k) {
        acc += M.l2_access[k];
        miss += M.l2_miss[k];
        printf("  %-8s instructions %llu lines/instr %.2f l2_requests/sample %.4f l2_misses/sample %.4f\n", names[k],
               (unsigned long long)M.instrs[k], M.instrs[k] ? (double)M.lines[k] / M.instrs[k] : 0.0,
               (double)M.l2_access[k] / M.samples, (double)M.l2_miss[k] / M.samples);
    }
    printf("total l2_hit %.4f l2_misses/sample %.4f l2_requests/sample %.4f bytes_past_l2_per_frame %.4g\n",
           1.0 - (double)miss / acc, (double)miss / M.samples, (double)acc / M.samples,
           (double)miss * 128.0 / M.samples * (double)A.W * A.H * A.nd * 2 * A.ns);
    return 0;
}
