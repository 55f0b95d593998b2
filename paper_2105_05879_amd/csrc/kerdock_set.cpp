// Host construction of the Kerdock set of Proposition 7 (Section 3).
//
// V = F_{2^{k-1}} x F_2 with basis B_i = (w^i, 0) for i < k-1 and
// B_{k-1} = (0, 1); bit i of a design coordinate is the coefficient on B_i.
// For s in F_{2^{k-1}} the matrix (M_s)_{ij} = B_i . L_s(B_j), with
// L_s(x, a) = (s^2 x + s tr(sx) + a s, tr(sx)) and (x,a).(y,b) = tr(xy) + ab,
// expands to
//   i, j < k-1:      tr(s^2 w^{i+j}) + tr(s w^i) tr(s w^j)
//   i < k-1 = j:     tr(s w^i)                       (and symmetrically)
//   i = j = k-1:     0.
// Only the strict upper triangle is kept: masks[s][i] has bit j (j > i) set
// when M_s[i][j] = 1, so that the quadratic form of Section 3 is
// Q_s(x) = parity( sum over set bits i of x of popcount(x & masks[s][i]) ).
//
// The field is F_2[w]/p(w) with p the smallest irreducible polynomial of
// degree k-1, chosen here with Rabin's irreducibility test.
#include <stdint.h>

#include <vector>

namespace kd {

namespace {

int degree(uint64_t p) { return p ? 63 - __builtin_clzll(p) : -1; }

// product of a and b modulo p (shift-and-add with interleaved reduction)
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) {
    const int D = degree(p);
    uint64_t r = 0;
    while (b) {
        if (b & 1) r ^= a;
        b >>= 1;
        a <<= 1;
        if ((a >> D) & 1) a ^= p;
    }
    return r;
}

// polynomial remainder and gcd over F_2
uint64_t pmod(uint64_t a, uint64_t b) {
    const int db = degree(b);
    for (int da = degree(a); da >= db; da = degree(a)) a ^= b << (da - db);
    return a;
}

uint64_t pgcd(uint64_t a, uint64_t b) {
    while (b) {
        uint64_t r = pmod(a, b);
        a = b;
        b = r;
    }
    return a;
}

// x^(2^e) mod p by repeated squaring of x
uint64_t frobenius_x(int e, uint64_t p) {
    uint64_t v = pmod(2, p);
    for (int i = 0; i < e; ++i) v = mulmod(v, v, p);
    return v;
}

// Rabin: p of degree D is irreducible iff x^(2^D) = x mod p and, for every
// prime q dividing D, gcd(x^(2^(D/q)) - x, p) = 1.
bool irreducible(uint64_t p) {
    const int D = degree(p);
    if (D < 1) return false;
    if (D == 1) return true;
    if (frobenius_x(D, p) != pmod(2, p)) return false;
    for (int q = 2; q <= D; ++q) {
        bool prime = true;
        for (int r = 2; r * r <= q; ++r)
            if (q % r == 0) prime = false;
        if (!prime || D % q) continue;
        if (pgcd(p, frobenius_x(D / q, p) ^ 2) != 1) return false;
    }
    return true;
}

}  // namespace

uint32_t field_polynomial(int D) {
    for (uint64_t p = 1ull << D; p < (2ull << D); ++p)
        if (irreducible(p)) return (uint32_t)p;
    return 0;
}

// masks: (2^{k-1}) x k entries, row-major by s.
std::vector<uint16_t> kerdock_masks(int k, uint32_t *poly_out) {
    const int D = k - 1;
    const uint64_t p = field_polynomial(D);
    if (poly_out) *poly_out = (uint32_t)p;
    const uint32_t q = 1u << D;

    // trace as a linear functional: tr(z) = parity(z & trmask), where bit t of
    // trmask is tr(w^t) = sum_{r<D} (w^t)^(2^r).
    uint64_t trmask = 0;
    for (int t = 0; t < D; ++t) {
        uint64_t z = (1ull << t), acc = 0;
        for (int r = 0; r < D; ++r) {
            acc ^= z;
            z = mulmod(z, z, p);
        }
        trmask |= (acc & 1ull) << t;
    }
    auto tr = [&](uint64_t z) { return (int)(__builtin_popcountll(z & trmask) & 1); };

    std::vector<uint16_t> masks((size_t)q * k, 0);
    std::vector<uint64_t> wpow(2 * D + 1);
    wpow[0] = 1;
    for (int e = 1; e <= 2 * D; ++e) wpow[e] = mulmod(wpow[e - 1], 2, p);
    for (uint32_t s = 0; s < q; ++s) {
        const uint64_t s2 = mulmod(s, s, p);
        std::vector<int> ts(D);
        for (int i = 0; i < D; ++i) ts[i] = tr(mulmod(s, wpow[i], p));
        uint16_t *row = &masks[(size_t)s * k];
        for (int i = 0; i < k; ++i) {
            uint16_t bits = 0;
            for (int j = i + 1; j < k; ++j) {
                int e;
                if (j < D) e = tr(mulmod(s2, wpow[i + j], p)) ^ (ts[i] & ts[j]);
                else e = ts[i];                          // j = k-1, i < k-1
                bits |= (uint16_t)(e << j);
            }
            row[i] = bits;
        }
    }
    return masks;
}

}  // namespace kd
