// Driver for the host-sanitizer build of libadaptvqe's host-only entry points
// (the library's sources compiled with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side; no device call is made).
// Reads a pool of generators and an adjacency matrix on stdin, runs
// vqe_mf_describe, vqe_mf_pool_create/get/owner_rows/destroy and
// vqe_partition_greedy on them, checks that bad arguments are refused, and
// prints every result for comparison with the regular build.
//
// Input (text): n_qubits M; per generator "n_terms" and n_terms lines
// "x z re im"; then "K" and a K x K 0/1 adjacency matrix, row by row.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "adaptvqe.h"

static void need(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "check failed: %s\n", what);
        std::exit(2);
    }
}

static void print_desc(const char *tag, int j, int rc, const vqe_mf_desc &d)
{
    std::printf("%s %d rc %d", tag, j, rc);
    if (rc == VQE_OK) {
        std::printf(" x %llu zsign %llu v %.17g %.17g ncon %d kbits %u", (unsigned long long)d.x,
                    (unsigned long long)d.zsign, d.v_re, d.v_im, d.n_con, d.kbits);
        for (int i = 0; i < d.n_con; i++)
            std::printf(" %llu", (unsigned long long)d.beta[i]);
    }
    std::printf("\n");
}

int main()
{
    int nq = 0, M = 0;
    need(std::scanf("%d %d", &nq, &M) == 2 && nq >= 2 && nq <= 20 && M > 0, "header");
    std::vector<int64_t> off(1, 0);
    std::vector<uint64_t> x, z;
    std::vector<double> c;
    for (int j = 0; j < M; j++) {
        long long n = 0;
        need(std::scanf("%lld", &n) == 1 && n > 0, "term count");
        for (long long t = 0; t < n; t++) {
            unsigned long long a, b;
            double re, im;
            need(std::scanf("%llu %llu %lf %lf", &a, &b, &re, &im) == 4, "term");
            x.push_back(a);
            z.push_back(b);
            c.push_back(re);
            c.push_back(im);
        }
        off.push_back(off.back() + n);
    }
    int K = 0;
    need(std::scanf("%d", &K) == 1 && K >= 0, "adjacency size");
    std::vector<uint8_t> adj((size_t)K * K);
    for (auto &a : adj) {
        int v;
        need(std::scanf("%d", &v) == 1, "adjacency entry");
        a = (uint8_t)v;
    }

    // each generator alone
    for (int j = 0; j < M; j++) {
        vqe_mf_desc d{};
        const int rc = vqe_mf_describe(nq, off[j + 1] - off[j], &x[off[j]], &z[off[j]],
                                       &c[2 * off[j]], 1e-12, &d);
        print_desc("describe", j, rc, d);
    }
    // the pool
    vqe_mf_pool *pool = nullptr;
    int rc = vqe_mf_pool_create(nq, M, off.data(), x.data(), z.data(), c.data(), nullptr, &pool);
    std::printf("pool_create rc %d\n", rc);
    if (rc == VQE_OK) {
        const int64_t tile_rows = (int64_t)1 << (nq - 1);
        for (int j = 0; j < M; j++) {
            vqe_mf_desc d{};
            print_desc("get", j, vqe_mf_pool_get(pool, j, &d), d);
            for (int tile = -1; tile < 2; tile++) {
                int64_t n = -1;
                need(vqe_mf_owner_rows(pool, j, tile_rows, tile, &n, nullptr, nullptr) == VQE_OK,
                     "owner rows (count)");
                std::vector<uint32_t> rows(n > 0 ? n : 1), idx(n > 0 ? n : 1);
                need(vqe_mf_owner_rows(pool, j, tile_rows, tile, &n, rows.data(), idx.data()) ==
                         VQE_OK, "owner rows");
                std::printf("owner %d %d %lld", j, tile, (long long)n);
                for (int64_t i = 0; i < n; i++)
                    std::printf(" %u:%u", rows[i], idx[i]);
                std::printf("\n");
            }
        }
        vqe_mf_desc d{};
        need(vqe_mf_pool_get(pool, M, &d) == VQE_EINVAL, "get out of range");
        need(vqe_mf_pool_get(pool, -1, &d) == VQE_EINVAL, "get negative");
        int64_t n = 0;
        need(vqe_mf_owner_rows(pool, M, tile_rows, 0, &n, nullptr, nullptr) != VQE_OK,
             "owner rows out of range");
        need(vqe_mf_pool_destroy(pool) == VQE_OK, "destroy");
    }
    // refused arguments
    {
        vqe_mf_desc d{};
        const uint64_t bad = (uint64_t)1 << nq, zero = 0;
        const double one[2] = {1.0, 0.0};
        need(vqe_mf_describe(nq, 1, &bad, &zero, one, 1e-12, &d) == VQE_EINVAL, "mask bit >= n");
        need(vqe_mf_describe(nq, 1, nullptr, &zero, one, 1e-12, &d) == VQE_EINVAL, "null x");
        need(vqe_mf_describe(0, 1, &bad, &zero, one, 1e-12, &d) == VQE_EINVAL, "zero qubits");
        const uint64_t xs[2] = {1, 2}, zs[2] = {0, 0};
        const double cs[4] = {1.0, 0.0, 1.0, 0.0};
        need(vqe_mf_describe(nq, 2, xs, zs, cs, 1e-12, &d) == VQE_ENOTSUP, "two flip masks");
        vqe_mf_pool *p2 = nullptr;
        const int64_t o2[2] = {0, 1};
        need(vqe_mf_pool_create(nq, 1, o2, &bad, &zero, one, nullptr, &p2) == VQE_EINVAL && !p2,
             "pool with a bad mask");
        int32_t nf = 0, fam = 0;
        need(vqe_partition_greedy(-1, nullptr, &fam, &nf) == VQE_EINVAL, "negative M");
        need(vqe_partition_greedy(1, nullptr, &fam, &nf) == VQE_EINVAL, "null adjacency");
        need(vqe_partition_greedy(0, nullptr, nullptr, &nf) == VQE_OK && nf == 0, "empty graph");
    }
    // Alg. 1 on the given graph
    std::vector<int32_t> fam(K > 0 ? K : 1);
    int32_t nf = -1;
    need(vqe_partition_greedy(K, adj.data(), fam.data(), &nf) == VQE_OK, "partition");
    std::printf("families %d", nf);
    for (int i = 0; i < K; i++)
        std::printf(" %d", fam[i]);
    std::printf("\n");
    for (int s = 0; s >= -5; s--)
        std::printf("strerror %d %s\n", s, vqe_strerror(s));
    return 0;
}
