// Host check of the kernels' element offsets (built and run by
// tests/test_index_check.py; no GPU is involved).
//
// It walks the launch grid of the step and adjoint kernels -- the same block
// shape (block_x) and the same PullIndex code the kernels address with --
// over every block, lane and population, and checks each access the
// kernels make:
//   - in bounds: every offset lies in its buffer (Q * N state or adjoint
//     elements, (1 + D) * N seed values or, without a seed, the same offsets
//     of lambda, D * N force values), and each lane's
//     byte offset within a row fits the 32 bits the kernels add to the row's
//     base;
//   - a permutation where it must be one: the pull loads of the step (and the
//     adjoint), the step's stores, the in-place pull half's stores (the
//     adjoint's pushes are the pull loads themselves) each touch every
//     element exactly once.
// Usage: index_check D nx ny nz full|edges
//   full:  every block of the grid, with the permutation counts;
//   edges: bounds only, on the blocks of the first two and last two rows
//          along y and z (the wrap-around) and one interior row, for grids
//          too large to count every element.
// Prints "ok <accesses checked>" or the first failing access, exit status 0
// or 1.
#include "../paper_2203_12946_amd/csrc/internal.hpp"
#include "../paper_2203_12946_amd/csrc/lattice.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

using namespace eselbm;

static int fail(const char *what, long long off, long long lim, int x, int y, int z, int i)
{
    std::printf("FAIL %s offset %lld not in [0, %lld) at x=%d y=%d z=%d i=%d\n", what, off, lim, x, y, z, i);
    return 1;
}

template <int D>
static int run(int nx, int ny, int nz, bool full)
{
    constexpr int Q = Lat<D>::Q;
    const long long N = (long long)nx * ny * nz, QN = (long long)Q * N;
    const int bx = block_x(nx);
    const int gx = (nx + bx - 1) / bx;
    std::vector<unsigned char> pull, store, aa;
    if (full) {
        pull.assign((size_t)QN, 0);
        store.assign((size_t)QN, 0);
        aa.assign((size_t)QN, 0);
    }
    std::vector<int> ylist, zlist;
    auto rows = [&](int n, std::vector<int> &v) {
        if (full) {
            for (int k = 0; k < n; ++k) v.push_back(k);
        } else {
            const int cand[5] = {0, 1, n / 2, n - 2, n - 1};
            for (int k : cand)
                if (k >= 0 && k < n && (v.empty() || v.back() < k)) v.push_back(k);
        }
    };
    rows(ny, ylist);
    rows(nz, zlist);
    long long checked = 0;
    for (int z : zlist)
        for (int y : ylist)
            for (int b = 0; b < gx; ++b)
                for (int t = 0; t < bx; ++t) {
                    const int x = b * bx + t;
                    if (x >= nx) continue;  // the kernels' guard
                    const PullIndex<D> pix(x, y, z, nx, ny, nz);
                    const long long cell = pix.row0 + x;
                    if (cell < 0 || cell >= N) return fail("cell", cell, N, x, y, z, -1);
                    for (int i = 0; i < Q; ++i) {
                        // step and adjoint: the pull load (the adjoint's push
                        // writes the same element)
                        const long long rs = pix.src_row(i);
                        const unsigned xs = pix.src_x(i);
                        if ((unsigned long long)xs * 8ull >= (1ull << 32)) return fail("lane byte offset", xs, nx, x, y, z, i);
                        const long long lo = (long long)i * N + rs + xs;
                        if (lo < 0 || lo >= QN) return fail("pull", lo, QN, x, y, z, i);
                        // step store, adjoint lambda read: the cell's own slot
                        const long long so = (long long)i * N + pix.row0 + x;
                        if (so < 0 || so >= QN) return fail("store", so, QN, x, y, z, i);
                        // in-place pull half: slot opp(i) of the cell + c_i
                        const long long ao = (long long)(Q - 1 - i) * N + pix.dst_row(i) + pix.dst_x(i);
                        if (ao < 0 || ao >= QN) return fail("in-place store", ao, QN, x, y, z, i);
                        if (full) {
                            ++pull[(size_t)lo];
                            ++store[(size_t)so];
                            ++aa[(size_t)ao];
                        }
                        checked += 3;
                    }
                    for (int c = 0; c <= D; ++c) {
                        const long long o = (long long)c * N + pix.row0 + x;
                        if (o < 0 || o >= (long long)(1 + D) * N) return fail("seed", o, (1 + D) * N, x, y, z, c);
                        if (c < D && o >= (long long)D * N) return fail("force", o, D * N, x, y, z, c);
                        // without a seed the adjoint reads lambda at these
                        // offsets instead (and discards the values)
                        if (o >= QN) return fail("seed read of lambda", o, QN, x, y, z, c);
                        checked += 2 + (c < D);
                    }
                }
    if (full) {
        for (long long k = 0; k < QN; ++k) {
            if (pull[(size_t)k] != 1 || store[(size_t)k] != 1 || aa[(size_t)k] != 1) {
                std::printf("FAIL element %lld touched pull %d, store %d, in-place store %d times\n", k,
                            pull[(size_t)k], store[(size_t)k], aa[(size_t)k]);
                return 1;
            }
        }
    }
    std::printf("ok %lld\n", checked);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 6) {
        std::fprintf(stderr, "usage: index_check D nx ny nz full|edges\n");
        return 2;
    }
    const int D = std::atoi(argv[1]), nx = std::atoi(argv[2]), ny = std::atoi(argv[3]), nz = std::atoi(argv[4]);
    const bool full = std::strcmp(argv[5], "full") == 0;
    if (nx < 1 || ny < 1 || nz < 1 || (D == 2 && nz != 1) || (D != 2 && D != 3)) return 2;
    return D == 2 ? run<2>(nx, ny, nz, full) : run<3>(nx, ny, nz, full);
}
