// shell.hpp -- the discrete contact shell of the WDLB force sums, usable at
// compile time (device kernels specialised for one sigma) and at run time
// (the host table of the generic kernels).  Both build every quad with the
// same function, so the two paths sum identical coefficients in the same
// order.
//
// Shell (Sec. 3, the sphere of contact): lattice offsets e with
// (sigma - 1/2)^2 <= |e|^2 < (sigma + 1/2)^2, each weighted 4 pi / |S|,
// direction k = e / |e|.  With s2 = 2 sigma (an integer for the specialised
// kernels) the test is (s2 - 1)^2 <= 4 |e|^2 < (s2 + 1)^2, exact in integers.
//
// Quads: the shell is visited in groups of mirror images (+-a, +-b, c),
// a, b >= 0, ordered by c, then b, then a.  A member with a = 0 or b = 0 is
// repeated in its group; the weight 1, 1/2 or 1/4 undoes the repetition.
#pragma once

namespace wdlb {

// square root by Newton's iteration from above (stops when the iterate no
// longer decreases: within an ulp of the rounded root)
constexpr double csqrt(double x)
{
    if (!(x > 0)) return 0;
    double y = x < 1 ? 1.0 : x;
    for (int i = 0; i < 2000; ++i) {
        const double n = 0.5 * (y + x / y);
        if (!(n < y)) break;
        y = n;
    }
    return y;
}

struct CQuad {
    int a, b, c, h;  // offset (a, b, c); h = parity sub-lattice (a&1) | (b&1)<<1 | (c&1)<<2
    // weight * k and weight * k_i k_j
    double px, py, pz, qxx, qyy, qzz, qxy, qxz, qyz;
};

constexpr CQuad make_cquad(int a, int b, int c)
{
    const double len = csqrt(double(a * a + b * b + c * c));
    const double ax = a / len, ay = b / len, az = c / len;
    const double w = (a > 0 ? 1.0 : 0.5) * (b > 0 ? 1.0 : 0.5);
    CQuad q{};
    q.a = a;
    q.b = b;
    q.c = c;
    q.h = (a & 1) | ((b & 1) << 1) | ((c & 1) << 2);
    q.px = w * ax;
    q.py = w * ay;
    q.pz = w * az;
    q.qxx = w * ax * ax;
    q.qyy = w * ay * ay;
    q.qzz = w * az * az;
    q.qxy = w * ax * ay;
    q.qxz = w * ax * az;
    q.qyz = w * ay * az;
    return q;
}

constexpr bool in_shell2(int s2, int r2) { return 4 * r2 >= (s2 - 1) * (s2 - 1) && 4 * r2 < (s2 + 1) * (s2 + 1); }
constexpr int shell_lim2(int s2) { return (s2 + 1) / 2 + 1; }

// largest offset component of the shell (at least 1)
constexpr int shell_reach2(int s2)
{
    int R = 1;
    const int L = shell_lim2(s2);
    for (int c = -L; c <= L; ++c)
        for (int b = -L; b <= L; ++b)
            for (int a = -L; a <= L; ++a)
                if (in_shell2(s2, a * a + b * b + c * c) && (a < 0 ? -a : a) > R) R = a < 0 ? -a : a;
    return R;
}

constexpr int shell_size2(int s2)
{
    int n = 0;
    const int L = shell_lim2(s2);
    for (int c = -L; c <= L; ++c)
        for (int b = -L; b <= L; ++b)
            for (int a = -L; a <= L; ++a) n += in_shell2(s2, a * a + b * b + c * c) ? 1 : 0;
    return n;
}

constexpr int shell_quads2(int s2)
{
    int n = 0;
    const int L = shell_lim2(s2);
    for (int c = -L; c <= L; ++c)
        for (int b = 0; b <= L; ++b)
            for (int a = 0; a <= L; ++a) n += in_shell2(s2, a * a + b * b + c * c) ? 1 : 0;
    return n;
}

// the quads of the shell 2 sigma = S2 and, per c = -R .. R, the start of its
// quads (qs[c + R] .. qs[c + R + 1])
template <int S2>
struct ShellTable {
    static constexpr int R = shell_reach2(S2);
    static constexpr int NQ = shell_quads2(S2);
    static constexpr int NS = shell_size2(S2);
    CQuad q[NQ];
    int qs[2 * R + 2];
    constexpr ShellTable() : q{}, qs{}
    {
        const int L = shell_lim2(S2);
        int n = 0;
        for (int c = -R; c <= R; ++c) {
            qs[c + R] = n;
            for (int b = 0; b <= L; ++b)
                for (int a = 0; a <= L; ++a)
                    if (in_shell2(S2, a * a + b * b + c * c)) q[n++] = make_cquad(a, b, c);
        }
        qs[2 * R + 1] = n;
    }
};

template <int S2>
struct Shell {
    static constexpr ShellTable<S2> T{};
    static constexpr int R = ShellTable<S2>::R;
    static constexpr int NQ = ShellTable<S2>::NQ;
};

// The ball of the smoothed density (Sec. 3): offsets with |e|^2 <= sigma^2/4
// (16 |e|^2 <= s2^2), each weighted 1/|B|, in the order z, then y, then x.
constexpr int ball_reach2(int s2)
{
    int r = 0;
    const int L = shell_lim2(s2);
    for (int z = -L; z <= L; ++z)
        for (int y = -L; y <= L; ++y)
            for (int x = -L; x <= L; ++x)
                if (16 * (x * x + y * y + z * z) <= s2 * s2 && (x < 0 ? -x : x) > r) r = x < 0 ? -x : x;
    return r;
}

constexpr int ball_size2(int s2)
{
    int n = 0;
    const int L = shell_lim2(s2);
    for (int z = -L; z <= L; ++z)
        for (int y = -L; y <= L; ++y)
            for (int x = -L; x <= L; ++x) n += 16 * (x * x + y * y + z * z) <= s2 * s2 ? 1 : 0;
    return n;
}

template <int S2>
struct BallTable {
    static constexpr int RB = ball_reach2(S2);
    static constexpr int NB = ball_size2(S2);
    int x[NB], y[NB], z[NB];
    constexpr BallTable() : x{}, y{}, z{}
    {
        int n = 0;
        for (int k = -RB; k <= RB; ++k)
            for (int j = -RB; j <= RB; ++j)
                for (int i = -RB; i <= RB; ++i)
                    if (16 * (i * i + j * j + k * k) <= S2 * S2) {
                        x[n] = i;
                        y[n] = j;
                        z[n] = k;
                        ++n;
                    }
    }
};

template <int S2>
struct Ball {
    static constexpr BallTable<S2> T{};
    static constexpr int RB = BallTable<S2>::RB;
    static constexpr int NB = BallTable<S2>::NB;
};

// The balls of MZ points stacked in z (point j at z = j) read together: every
// lattice offset (x, y, z) of their union once, in the order z, then y, then
// x, with the ball index k[j] it has for point j (its offset from that point
// is (x, y, z - j); -1 when outside that ball).  For each point the terms
// then arrive in its own ball order.
constexpr int ball_union_size2(int s2, int mz)
{
    const int rb = ball_reach2(s2);
    int n = 0;
    for (int z = -rb; z <= rb + mz - 1; ++z)
        for (int y = -rb; y <= rb; ++y)
            for (int x = -rb; x <= rb; ++x) {
                bool any = false;
                for (int j = 0; j < mz; ++j) {
                    const int zz = z - j;
                    any = any || 16 * (x * x + y * y + zz * zz) <= s2 * s2;
                }
                n += any ? 1 : 0;
            }
    return n;
}

template <int S2, int MZ>
struct BallColumn {
    static constexpr int NU = ball_union_size2(S2, MZ);
    int x[NU], y[NU], z[NU], k[NU][MZ];
    constexpr BallColumn() : x{}, y{}, z{}, k{}
    {
        const int rb = ball_reach2(S2), W = 2 * rb + 1;
        // ball index of each offset of the reach cube, in the ball's own order
        static_assert(ball_reach2(S2) <= 8, "ball reach of the index grid");
        int grid[17 * 17 * 17] = {};
        int idx = 0;
        for (int c = -rb; c <= rb; ++c)
            for (int b = -rb; b <= rb; ++b)
                for (int a = -rb; a <= rb; ++a)
                    grid[((c + rb) * W + (b + rb)) * W + (a + rb)] =
                        16 * (a * a + b * b + c * c) <= S2 * S2 ? idx++ : -1;
        int n = 0;
        for (int zz = -rb; zz <= rb + MZ - 1; ++zz)
            for (int yy = -rb; yy <= rb; ++yy)
                for (int xx = -rb; xx <= rb; ++xx) {
                    bool any = false;
                    int kk[MZ] = {};
                    for (int j = 0; j < MZ; ++j) {
                        const int zj = zz - j;
                        kk[j] = (zj < -rb || zj > rb) ? -1 : grid[((zj + rb) * W + (yy + rb)) * W + (xx + rb)];
                        any = any || kk[j] >= 0;
                    }
                    if (!any) continue;
                    x[n] = xx;
                    y[n] = yy;
                    z[n] = zz;
                    for (int j = 0; j < MZ; ++j) k[n][j] = kk[j];
                    ++n;
                }
    }
};

}  // namespace wdlb
