// Host driver for the product planner's device code, compiled on the CPU by
// tests/test_planner_host.py: the planner section of product.hip is pasted above
// this file with one-thread launches emulated by loops.  It builds a plan for
// C = mask_C(A B) from three block-CSR patterns and checks that every (i, k, j)
// triple it schedules is a real one, with the right A, B and C slots, and that
// every C slot belongs to exactly one tile position.  Prints the number of
// triples scheduled; exits non-zero on any violation.
#include <cstdio>

struct HostPattern {
    int n = 0;
    std::vector<int> rp, cc, tm;
};

static int slot_of(const HostPattern &P, int i, int j)
{
    for (int p = P.rp[i]; p < P.rp[i + 1]; ++p)
        if (P.cc[p] == j) return p;
    return -1;
}

static HostPattern load(const char *fn)
{
    HostPattern P;
    FILE *f = fopen(fn, "rb");
    if (!f) exit(2);
    int hd[2];
    if (fread(hd, 4, 2, f) != 2) exit(2);
    P.n = hd[0];
    P.rp.resize(P.n + 1);
    P.cc.resize(hd[1]);
    if (fread(P.rp.data(), 4, P.n + 1, f) != (size_t)P.n + 1 || fread(P.cc.data(), 4, hd[1], f) != (size_t)hd[1])
        exit(2);
    fclose(f);
    P.tm.resize(hd[1]);
    for (int i = 0; i < P.n; ++i)
        for (int p = P.rp[i]; p < P.rp[i + 1]; ++p) P.tm[p] = slot_of(P, P.cc[p], i);
    return P;
}

int main(int argc, char **argv)
{
    if (argc != 10) return 2;
    const HostPattern A = load(argv[1]), Bp = load(argv[2]), C = load(argv[3]);
    const int G = atoi(argv[4]), JT = atoi(argv[5]), W = atoi(argv[6]), order = atoi(argv[7]), tr = atoi(argv[8]);
    const int nch = atoi(argv[9]);   // planner threads per tile
    const int n = C.n, jt = JT * W;
    const HostPattern &KA = tr ? Bp : A, &KB = tr ? A : Bp;   // the kernel's operands
    const int ng = (n + G - 1) / G;
    std::vector<int> ntile(ng);
    std::vector<int64_t> toff(ng + 1, 0);
    blockDim.x = 1;
    threadIdx.x = 0;
    for (int g = 0; g < ng; ++g) {
        blockIdx.x = g;
        k_group_union(n, G, C.rp.data(), C.cc.data(), jt, ntile.data());
        toff[g + 1] = toff[g] + ntile[g];
    }
    const int64_t nt = toff[ng];
    const int hs = G + G * jt, es = W * G + jt;
    std::vector<int> hdr(nt * hs, -9), tcols(nt * jt, -9), scr((5 + G) * nt * jt + 1, -5);
    for (int g = 0; g < ng; ++g) {
        blockIdx.x = g;
        k_group_tiles(n, G, jt, order, C.rp.data(), C.cc.data(), toff.data(), nt, hdr.data(), tcols.data(),
                      scr.data());
    }
    const int64_t ntc = nt * nch;
    std::vector<int64_t> nent(ntc), ebeg_tc(ntc + 1, 0), ebeg(nt + 1, 0);
    unsigned long long tri = 0, rw = 0;
    for (int64_t tc = 0; tc < ntc; ++tc) {
        blockIdx.x = (int)tc;
        k_tile_entries<0>(nt, nch, n, G, jt, W, tr, hdr.data(), tcols.data(), KA.rp.data(), KA.cc.data(),
                          KA.tm.data(), KB.rp.data(), KB.cc.data(), KB.tm.data(), nent.data(), &tri, &rw, nullptr,
                          nullptr);
    }
    for (int64_t t = 0; t < nt; ++t) {
        blockIdx.x = (int)t;
        k_pad_counts(nt, nch, nent.data());
    }
    for (int64_t tc = 0; tc < ntc; ++tc) ebeg_tc[tc + 1] = ebeg_tc[tc] + nent[tc];
    for (int64_t t = 0; t <= nt; ++t) {
        blockIdx.x = (int)t;
        k_tile_ebeg(nt, nch, ebeg_tc.data(), ebeg.data());
    }
    std::vector<int> ent((ebeg[nt] + 4) * es, -7);
    for (int64_t tc = 0; tc < ntc; ++tc) {
        blockIdx.x = (int)tc;
        k_tile_entries<1>(nt, nch, n, G, jt, W, tr, hdr.data(), tcols.data(), KA.rp.data(), KA.cc.data(),
                          KA.tm.data(), KB.rp.data(), KB.cc.data(), KB.tm.data(), nullptr, nullptr, nullptr,
                          ebeg_tc.data(), ent.data());
    }
    if (tr)
        for (int64_t t = 0; t < nt; ++t) {
            blockIdx.x = (int)t;
            k_map_cslots(nt, G, jt, C.tm.data(), hdr.data());
        }
    long bad = 0;
    // every C slot at exactly one (tile, row, column) position, at the right (row, column)
    std::vector<int> owner(C.cc.size(), 0);
    for (int64_t t = 0; t < nt; ++t)
        for (int a = 0; a < G; ++a)
            for (int x = 0; x < jt; ++x) {
                const int cs = hdr[t * hs + G + a * jt + x];
                if (cs == -9) ++bad;
                if (cs < 0) continue;
                const int i = hdr[t * hs + a], j = tcols[t * jt + x];
                if (i < 0 || j < 0 || cs != (tr ? slot_of(C, j, i) : slot_of(C, i, j))) ++bad;
                ++owner[cs];
            }
    for (int v : owner)
        if (v != 1) ++bad;
    // entries of a tile in strictly ascending k (padding entries, all slots -1, only at the end)
    for (int64_t t = 0; t < nt; ++t) {
        int last = -1;
        bool padded = false;
        for (int64_t q = ebeg[t]; q < ebeg[t + 1]; ++q) {
            int k = -1;
            for (int hf = 0; hf < W && k < 0; ++hf) {
                const int *e = &ent[q * es + hf * (G + JT)];
                for (int a = 0; a < G && k < 0; ++a)
                    if (e[a] >= 0) {
                        if (!tr) k = A.cc[e[a]];
                        else {
                            int r = 0;
                            while (!(e[a] >= Bp.rp[r] && e[a] < Bp.rp[r + 1])) ++r;
                            k = r;
                        }
                    }
            }
            if (k < 0) { padded = true; continue; }
            if (padded || k <= last) ++bad;
            last = k;
        }
    }
    // every scheduled triple real, with its A, B and C slots
    unsigned long long seen = 0;
    for (int64_t t = 0; t < nt; ++t) {
        if ((ebeg[t + 1] - ebeg[t]) % 2) ++bad;
        for (int64_t q = ebeg[t]; q < ebeg[t + 1]; ++q)
            for (int hf = 0; hf < W; ++hf) {
                const int *e = &ent[q * es + hf * (G + JT)];
                for (int a = 0; a < G; ++a) {
                    if (e[a] == -7) ++bad;
                    if (e[a] < 0) continue;
                    const int i = hdr[t * hs + a];
                    for (int x = 0; x < JT; ++x) {
                        const int bs = e[G + x], cs = hdr[t * hs + G + a * jt + hf * JT + x];
                        if (bs < 0 || cs < 0) continue;
                        const int j = tcols[t * jt + hf * JT + x];
                        if (!tr) {   // A slot (i, k), B slot (k, j)
                            const int k = A.cc[e[a]];
                            if (slot_of(A, i, k) != e[a] || slot_of(Bp, k, j) != bs) ++bad;
                        } else {     // B slot (k, i), A slot (j, k)
                            if (Bp.cc[e[a]] != i) { ++bad; continue; }
                            int k = 0;
                            while (!(e[a] >= Bp.rp[k] && e[a] < Bp.rp[k + 1])) ++k;
                            if (slot_of(A, j, k) != bs) ++bad;
                        }
                        ++seen;
                    }
                }
            }
    }
    if (seen != tri) ++bad;
    printf("%llu %ld\n", seen, bad);
    return bad != 0;
}
