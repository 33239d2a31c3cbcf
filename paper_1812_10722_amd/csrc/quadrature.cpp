// Triangle and Gauss-Legendre rules of the library.
//
// The paper lists only the point counts of its triangle rules (section "Integral evaluation",
// Tables 1 and 4): 1, 3 or 4 points for far panels and 19, 25 or 37 for near-singular ones.
// These are the counts of Dunavant's symmetric rules (degrees 1, 2, 3, 9, 10, 13); the library
// carries the published degree-1, 2, 3, 9, 10 and 13 rules and Radon's 7-point degree-5 rule.
// Each rule is stored as symmetric orbits of barycentric coordinates.
#include <cmath>

#include "internal.hpp"

namespace lspr {

namespace {

struct Orbit {
    int kind;       // 1: centroid, 3: (a, b, b), 6: permutations of (a, b, 1 - a - b)
    double w, a, b;
};

const Orbit kRule1[] = {{1, 1.0, 0, 0}};
const Orbit kRule3[] = {{3, 1.0 / 3.0, 2.0 / 3.0, 1.0 / 6.0}};
const Orbit kRule4[] = {{1, -0.5625, 0, 0}, {3, 25.0 / 48.0, 0.6, 0.2}};
const Orbit kRule19[] = {
    {1, 0.097135796282799, 0, 0},
    {3, 0.031334700227139, 0.020634961602525, 0.489682519198738},
    {3, 0.077827541004774, 0.125820817014127, 0.437089591492937},
    {3, 0.079647738927210, 0.623592928761935, 0.188203535619033},
    {3, 0.025577675658698, 0.910540973211095, 0.044729513394453},
    {6, 0.043283539377289, 0.036838412054736, 0.221962989160766}};
const Orbit kRule25[] = {
    {1, 0.090817990382754, 0, 0},
    {3, 0.036725957756467, 0.028844733232685, 0.485577633383657},
    {3, 0.045321059435528, 0.781036849029926, 0.109481575485037},
    {6, 0.072757916845420, 0.141707219414880, 0.307939838764121},
    {6, 0.028327242531057, 0.025003534762686, 0.246672560639903},
    {6, 0.009421666963733, 0.009540815400299, 0.066803251012200}};
// degree 13: the strict near-singular rule of the paper's grid-convergence study
const Orbit kRule37[] = {
    {1, 0.052520923400802, 0, 0},
    {3, 0.011280145209330, 0.009903630120591, 0.495048184939705},
    {3, 0.031423518362454, 0.062566729780852, 0.468716635109574},
    {3, 0.047072502504194, 0.170957326397447, 0.414521336801277},
    {3, 0.047363586536355, 0.541200855914337, 0.229399572042831},
    {3, 0.031167529045794, 0.771151009607340, 0.114424495196330},
    {3, 0.007975771465074, 0.950377217273082, 0.024811391363459},
    {6, 0.036848402728732, 0.094853828379579, 0.268794997058761},
    {6, 0.017401463303822, 0.018100773278807, 0.291730066734288},
    {6, 0.015521786839045, 0.022233076674090, 0.126357385491669}};

void expand(const Orbit* o, int n_orbits, std::vector<double>& bary, std::vector<double>& w) {
    bary.clear();
    w.clear();
    auto put = [&](double x, double y, double z, double wt) {
        bary.push_back(x);
        bary.push_back(y);
        bary.push_back(z);
        w.push_back(wt);
    };
    for (int k = 0; k < n_orbits; ++k) {
        const Orbit& r = o[k];
        if (r.kind == 1) {
            put(1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, r.w);
        } else if (r.kind == 3) {
            const double a = r.a, b = 0.5 * (1.0 - r.a);
            put(a, b, b, r.w);
            put(b, a, b, r.w);
            put(b, b, a, r.w);
        } else {
            const double a = r.a, b = r.b, c = 1.0 - r.a - r.b;
            put(a, b, c, r.w);
            put(a, c, b, r.w);
            put(b, a, c, r.w);
            put(b, c, a, r.w);
            put(c, a, b, r.w);
            put(c, b, a, r.w);
        }
    }
}

}  // namespace

bool triangle_rule(int n, std::vector<double>& bary, std::vector<double>& w) {
    switch (n) {
        case 1: expand(kRule1, 1, bary, w); return true;
        case 3: expand(kRule3, 1, bary, w); return true;
        case 4: expand(kRule4, 2, bary, w); return true;
        case 7: {
            const double s = std::sqrt(15.0);
            const Orbit r7[] = {{1, 9.0 / 40.0, 0, 0},
                                {3, (155.0 - s) / 1200.0, (9.0 + 2.0 * s) / 21.0, 0},
                                {3, (155.0 + s) / 1200.0, (9.0 - 2.0 * s) / 21.0, 0}};
            expand(r7, 3, bary, w);
            return true;
        }
        case 19: expand(kRule19, 6, bary, w); return true;
        case 25: expand(kRule25, 6, bary, w); return true;
        case 37: expand(kRule37, 10, bary, w); return true;
        default: return false;
    }
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on P_n from the Chebyshev-like
// initial guess cos(pi (k - 1/4) / (n + 1/2)), P_n and P_n' from the three-term recurrence.
void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w) {
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < (n + 1) / 2; ++k) {
        double x = std::cos(pi * (k + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int m = 2; m <= n; ++m) {
                const double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            const double pn = n == 0 ? 1.0 : (n == 1 ? x : p1);
            const double pn1 = n == 1 ? 1.0 : p0;  // P_{n-1}
            dp = n * (x * pn - pn1) / (x * x - 1.0);
            const double dx = pn / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        // recompute the derivative at the converged node
        double p0 = 1.0, p1 = x;
        for (int m = 2; m <= n; ++m) {
            const double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        const double pn = n == 1 ? x : p1;
        const double pn1 = n == 1 ? 1.0 : p0;
        dp = n * (x * pn - pn1) / (x * x - 1.0);
        const double wk = 2.0 / ((1.0 - x * x) * dp * dp);
        t[k] = -x;
        t[n - 1 - k] = x;
        w[k] = wk;
        w[n - 1 - k] = wk;
    }
    if (n % 2 == 1) t[n / 2] = 0.0;
}

}  // namespace lspr
