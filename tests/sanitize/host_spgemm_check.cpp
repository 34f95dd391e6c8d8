// Driver for the sanitizer builds of the library's host SpGEMM (host_spgemm.cpp):
// random CSC products of several shapes on 1 and 4 threads, each column
// compared bit for bit with a plain ordered-map accumulation in ascending k,
// plus the structure checks on malformed inputs.  Prints "ok" and exits 0
// when everything matches.
#include "host_spgemm.hpp"

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <random>
#include <vector>

namespace {

struct Mat {
    int64_t nrows = 0, ncols = 0;
    std::vector<int64_t> cp;
    std::vector<int32_t> ri;
    std::vector<double> v;
    mcl::host::CSC csc() const
    {
        return mcl::host::CSC{nrows, ncols, (int64_t)ri.size(), cp.data(), ri.data(), v.data()};
    }
};

Mat random_mat(int64_t nrows, int64_t ncols, double density, double empty_frac, uint64_t seed)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    Mat m;
    m.nrows = nrows;
    m.ncols = ncols;
    m.cp.push_back(0);
    for (int64_t j = 0; j < ncols; ++j) {
        if (u(rng) >= empty_frac)
            for (int64_t i = 0; i < nrows; ++i)
                if (u(rng) < density) {
                    m.ri.push_back((int32_t)i);
                    m.v.push_back(0.05 + u(rng));
                }
        m.cp.push_back((int64_t)m.ri.size());
    }
    return m;
}

// C = A*B one column at a time: products added in ascending k into an
// ordered map (first product of a row: 0.0 + product)
int check_product(const Mat &A, const Mat &B, int threads)
{
    mcl::host::Out o;
    mcl::host::spgemm(A.csc(), B.csc(), threads, o);
    int bad = 0;
    int64_t nnz = 0;
    for (int64_t j = 0; j < B.ncols; ++j) {
        std::map<int32_t, double> acc;
        for (int64_t t = B.cp[j]; t < B.cp[j + 1]; ++t) {
            const int32_t k = B.ri[t];
            const double b = B.v[t];
            for (int64_t p = A.cp[k]; p < A.cp[k + 1]; ++p) {
                const double prod = A.v[p] * b;
                auto it = acc.find(A.ri[p]);
                if (it == acc.end()) acc[A.ri[p]] = 0.0 + prod;
                else it->second = it->second + prod;
            }
        }
        if (o.colptr[j + 1] - o.colptr[j] != (int64_t)acc.size()) {
            ++bad;
            continue;
        }
        int64_t q = o.colptr[j];
        for (const auto &e : acc) {
            if (o.rowidx[q] != e.first || std::memcmp(&o.val[q], &e.second, sizeof(double)) != 0) ++bad;
            ++q;
        }
        nnz += (int64_t)acc.size();
    }
    if (o.nnz != nnz) ++bad;
    mcl::host::release(o);
    return bad;
}

}  // namespace

int main()
{
    int bad = 0;
    const Mat A1 = random_mat(300, 200, 0.03, 0.1, 1), B1 = random_mat(200, 150, 0.04, 0.2, 2);
    const Mat A2 = random_mat(2000, 2000, 0.004, 0.0, 3);
    const Mat Z = random_mat(50, 40, 0.0, 0.0, 4), E = random_mat(0, 30, 0.0, 0.0, 5);
    const Mat D = random_mat(64, 64, 0.9, 0.0, 6);  // dense columns: tables grow several times
    for (int threads : {1, 4}) {
        bad += check_product(A1, B1, threads);
        bad += check_product(A2, A2, threads);
        bad += check_product(random_mat(50, 50, 0.1, 0.0, 7), Z, threads);
        bad += check_product(random_mat(7, 0, 0.1, 0.0, 8), E, threads);
        bad += check_product(D, D, threads);
    }
    // malformed inputs are reported, not read
    Mat M = random_mat(20, 20, 0.2, 0.0, 9);
    if (!M.ri.empty()) {
        M.ri[0] = 20;
        if (std::strlen(mcl::host::check(M.csc())) == 0) ++bad;
    }
    Mat N = random_mat(20, 20, 0.2, 0.0, 10);
    N.cp[3] = N.cp[4] + 1;
    if (std::strlen(mcl::host::check(N.csc())) == 0) ++bad;
    if (std::strlen(mcl::host::check(A1.csc())) != 0) ++bad;
    std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
    return bad ? 1 : 0;
}
