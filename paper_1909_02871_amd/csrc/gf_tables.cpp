// Host-side construction of the field tables that the kernels read.
//
// Fields (Sec. II: words of n bits, q = 2^n; addition is XOR, multiplication
// is reduction modulo a field polynomial): GF(4) x^2+x+1, GF(16) x^4+x+1,
// GF(256) x^8+x^4+x^3+x^2+1, all primitive, so x generates the multiplicative
// group.  Products are taken from exponent/logarithm tables of x; GF(2)
// multiplication is AND.
#include <string.h>

#include "gf_internal.h"

namespace gfnc {

namespace {

const int kBits[4] = {1, 2, 4, 8};
const int kPoly[4] = {0, 0x7, 0x13, 0x11D};

struct Builder {
    HostTables t;

    Builder()
    {
        memset(&t, 0, sizeof t);
        for (int f = 0; f < 4; f++)
            build_field(f);
    }

    void build_field(int f)
    {
        const int n = kBits[f], q = 1 << n;
        // element products
        if (n == 1) {
            for (int c = 0; c < 2; c++)
                for (int a = 0; a < 2; a++)
                    t.mul[f][c][a] = (uint8_t)(c & a);
        } else {
            int ex[512], lg[256];
            int e = 1;
            for (int i = 0; i < q - 1; i++) {
                ex[i] = ex[i + q - 1] = e;
                lg[e] = i;
                e <<= 1;              // multiply by x
                if (e & q)
                    e ^= kPoly[f];    // x^n = rest of the polynomial
            }
            for (int c = 0; c < q; c++)
                for (int a = 0; a < q; a++)
                    t.mul[f][c][a] = (uint8_t)((c && a) ? ex[lg[c] + lg[a]] : 0);
        }
        for (int a = 1; a < q; a++)
            for (int b = 1; b < q; b++)
                if (t.mul[f][a][b] == 1)
                    t.inv[f][a] = (uint8_t)b;
        // byte-permute tables: c times each byte whose set bits lie in one of
        // the three bit groups [0,3), [3,6), [6,8)
        const int mask = q - 1;
        for (int c = 0; c < q; c++) {
            auto prodbyte = [&](int b) {
                int r = 0;
                for (int k = 0; k < 8 / n; k++)
                    r |= t.mul[f][c][(b >> (n * k)) & mask] << (n * k);
                return (uint32_t)r;
            };
            uint32_t *d = t.ptab[f][c];
            for (int v = 0; v < 8; v++) {
                d[v >> 2] |= prodbyte(v) << (8 * (v & 3));
                d[2 + (v >> 2)] |= prodbyte(v << 3) << (8 * (v & 3));
            }
            for (int v = 0; v < 4; v++)
                d[4] |= prodbyte(v << 6) << (8 * v);
            // bit-matrix rows: column j is the product with the byte 1 << j
            for (int j = 0; j < 8; j++) {
                const uint32_t col = prodbyte(1 << j);
                for (int i = 0; i < 8; i++)
                    if ((col >> i) & 1u)
                        t.rows[f][c][i] |= (uint8_t)(1u << j);
            }
        }
    }
};

}  // namespace

const HostTables &host_tables()
{
    static Builder b;   // thread-safe static initialisation
    return b.t;
}

}  // namespace gfnc
