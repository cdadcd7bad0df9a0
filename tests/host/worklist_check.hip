// Host-side check of the polarizability work list and batch sizes (no GPU
// needed): every lower-triangle tile of every plane exactly once, entries in
// range, the padding below one round per XCD, every XCD's run a whole number
// of rounds; batches within the buffer and taking no more waves than the
// fewest batches.  Exit status 0 on success.
#include "../../paper_2305_15955_amd/csrc/k_dense.hip"

#include <cstdio>
#include <set>

int main() {
    int bad = 0;
    for (int npad : {256, 512, 768, 1280, 2560, 5120, 6656})
        for (int nfb : {1, 2, 3, 7, 12, 16})
            for (int cu : {1, 16, 32, 38}) {
                const std::vector<int2> w = cdwac::pi_worklist(npad, nfb, cu);
                const int n = npad / 256;
                std::set<long> seen;
                for (const int2 e : w) {
                    if (e.x < 0) {
                        if (e.y != -1) ++bad;
                        continue;
                    }
                    const int fb = e.x >> 16, I = e.x & 0xffff, J = e.y;
                    if (fb >= nfb || I >= n || J < 0 || J > I || !seen.insert(((long)fb * n + I) * n + J).second)
                        ++bad;
                }
                const long want = (long)nfb * n * (n + 1) / 2;
                if ((long)seen.size() != want || w.size() % 8 != 0 || (w.size() / 8) % cu != 0 ||
                    (long)w.size() - want >= 8L * cu) {
                    ++bad;
                    std::printf("npad %d nfb %d cu %d: %zu entries for %ld tiles\n", npad, nfb, cu, w.size(), want);
                }
                if ((int)cdwac::pi_tile_count(npad) != n * (n + 1) / 2) ++bad;
            }
    // batch sizes: within the buffer, near-equal batches, never more waves of
    // workgroups than the fewest batches would take; 48 planes of 210 tiles on
    // 256 CUs split 4 x 12 (40 waves), not 3 x 16 (42)
    for (int np : {1, 7, 24, 48, 60, 88})
        for (int nb : {1, 5, 16, 100})
            for (int cu : {1, 256}) {
                const int per = cdwac::pi_batch_size(np, nb, 210, cu);
                const int minb = (np + nb - 1) / nb;
                const int per0 = (np + minb - 1) / minb;
                auto waves = [&](int p) {
                    long w = 0;
                    for (int f0 = 0; f0 < np; f0 += p) w += ((long)std::min(p, np - f0) * 210 + cu - 1) / cu;
                    return w;
                };
                if (per < 1 || per > nb || per > np || waves(per) > waves(per0)) {
                    ++bad;
                    std::printf("batch np %d nb %d cu %d -> %d\n", np, nb, cu, per);
                }
            }
    if (cdwac::pi_batch_size(48, 16, 210, 256) != 12) ++bad;
    // W tiles: every (row block I, column block J) of the grid exactly once,
    // row blocks from the last down (the contraction over Lambda's lower block
    // triangle makes row block I cost I + 1 chunks of 256)
    for (int npad : {256, 512, 1280, 5120, 6656})
        for (int cpad : {256, 768, 24064}) {
            const std::vector<int2> t = cdwac::w_tiles(npad, cpad);
            const int nI = npad / 256, nJ = cpad / 256;
            std::set<long> seen;
            int last_band = 0;
            for (const int2 e : t) {
                if (e.x < 0 || e.x >= nI || e.y < 0 || e.y >= nJ || !seen.insert((long)e.x * nJ + e.y).second) {
                    ++bad;
                    continue;
                }
                const int band = (nI - 1 - e.x) / 4;   // bands of 4 row blocks, counted from the last
                if (band < last_band) ++bad;
                last_band = band;
            }
            if ((long)seen.size() != (long)nI * nJ) {
                ++bad;
                std::printf("w_tiles npad %d cpad %d: %zu tiles\n", npad, cpad, seen.size());
            }
        }
    // tile order of the sweep's updates: every lower-triangle tile of an n x n
    // block grid exactly once, bands of 4 block rows in order, every 32
    // consecutive tiles of a full band within 4 row and 8 column blocks
    for (int n = 1; n <= 256; ++n) {
        const int T = n * (n + 1) / 2;
        std::set<long> seen;
        int last_band = 0;
        std::vector<int> ti(T), tj(T);
        for (int t = 0; t < T; ++t) {
            int I = -1, J = -1;
            cdwac::sweep_tile_order(t, n, I, J);
            ti[t] = I;
            tj[t] = J;
            if (I < 0 || I >= n || J < 0 || J > I || !seen.insert((long)I * n + J).second || I / 4 < last_band) {
                ++bad;
                std::printf("sweep order n %d t %d -> (%d, %d)\n", n, t, I, J);
                break;
            }
            last_band = I / 4;
        }
        if ((int)seen.size() != T) ++bad;
        for (int t0 = 0; t0 + 32 <= T; t0 += 32) {
            std::set<int> rows, cols;
            for (int t = t0; t < t0 + 32; ++t) {
                rows.insert(ti[t]);
                cols.insert(tj[t]);
            }
            // a run inside one full band, away from its diagonal, touches 4 x 8 blocks
            if (ti[t0] / 4 == ti[t0 + 31] / 4 && 4 * (ti[t0] / 4) + 3 < n && tj[t0 + 31] + 4 <= 4 * (ti[t0] / 4) &&
                (rows.size() > 4 || cols.size() > 16))
                ++bad;
        }
    }
    std::printf("%s\n", bad ? "FAIL" : "ok");
    return bad != 0;
}
