// Test harness for the host-side dense step of the library (small_dense.cpp):
// reads one command and its matrices from stdin, writes the results to stdout
// as "name rows cols" followed by rows*cols column-major "re im" pairs.
// Built and driven by tests/test_host_small_dense.py (CPU only).
#include <complex>
#include <cstdio>
#include <iostream>
#include <string>

#include "small_dense.h"

using gplhr::small::Mat;
using cd = std::complex<double>;

static Mat read_mat(int r, int c) {
    Mat m(r, c);
    for (int j = 0; j < c; ++j)
        for (int i = 0; i < r; ++i) {
            double re, im;
            std::cin >> re >> im;
            m(i, j) = cd(re, im);
        }
    return m;
}

static void write_mat(const char *name, const Mat &m) {
    std::printf("%s %d %d\n", name, m.r, m.c);
    for (int j = 0; j < m.c; ++j)
        for (int i = 0; i < m.r; ++i) std::printf("%.17g %.17g\n", m(i, j).real(), m(i, j).imag());
}

int main() {
    std::string cmd;
    std::cin >> cmd;
    if (cmd == "schur") {
        int s, nsel;
        std::cin >> s >> nsel;
        Mat T = read_mat(s, s), Y;
        const bool ok = gplhr::small::schur(T, Y);
        if (nsel > 0) gplhr::small::reorder_desc_abs(T, Y, nsel);
        std::printf("ok %d\n", ok ? 1 : 0);
        write_mat("T", T);
        write_mat("Y", Y);
    } else if (cmd == "qr") {
        int r, c;
        std::cin >> r >> c;
        Mat X = read_mat(r, c), Q, R;
        gplhr::small::qr_thin(X, Q, R);
        std::printf("ok 1\n");
        write_mat("Q", Q);
        write_mat("R", R);
    } else if (cmd == "srr" || cmd == "eig") {
        int s, b, nkeep;
        double sr, si;
        std::cin >> s >> b >> nkeep >> sr >> si;
        Mat K = read_mat(s, s), G = read_mat(s, s);
        if (cmd == "srr") {
            gplhr::small::SrrResult r;
            const bool ok = gplhr::small::harmonic_srr(K, G, cd(sr, si), b, nkeep, r);
            std::printf("ok %d\n", ok ? 1 : 0);
            write_mat("YR", r.YR);
            write_mat("YL", r.YL);
            write_mat("RA", r.RA);
            write_mat("RB", r.RB);
            write_mat("MA", r.MA);
            write_mat("MB", r.MB);
        } else {
            Mat Yb;
            const bool ok = gplhr::small::harmonic_eig(K, G, nkeep, Yb);
            std::printf("ok %d\n", ok ? 1 : 0);
            write_mat("Ybar", Yb);
        }
    } else if (cmd == "qfree") {
        int b;
        std::cin >> b;
        Mat RA = read_mat(b, b), RB = read_mat(b, b), MA, MB;
        gplhr::small::q_free_factors(RA, RB, MA, MB);
        std::printf("ok 1\n");
        write_mat("MA", MA);
        write_mat("MB", MB);
    } else {
        std::printf("ok 0\n");
        return 2;
    }
    return 0;
}
