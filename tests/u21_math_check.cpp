// Host build of the library's FP64 uniform transcendentals (u21_ln, u21_sincos_turn), checked
// over every 21-bit argument b against long-double references, and against the double libm
// calls the oracle makes (log, sin, cos of the same u).  Prints the largest relative errors
// and exits non-zero when one exceeds the bound given on the command line.
#include "lb_rng.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int main(int argc, char **argv)
{
    const double bound = argc > 1 ? atof(argv[1]) : 4.5e-16;
    const long double pi = acosl(-1.0L);
    double eln = 0, esn = 0, ecs = 0, oln = 0, osn = 0, ocs = 0;
    for (uint32_t b = 0; b < (1u << 21); ++b) {
        const long double u = ((long double)b + 0.5L) / 2097152.0L;
        // the reference angle reduced exactly first: u - k/4 in [-1/8, 1/8], k its quarter turn
        const long double k = roundl(4 * u), th = 2 * pi * (u - k / 4);
        const long double s0 = sinl(th), c0 = cosl(th);
        const int q = (int)k & 3;
        const long double sr = q == 0 ? s0 : (q == 1 ? c0 : (q == 2 ? -s0 : -c0));
        const long double cr = q == 0 ? c0 : (q == 1 ? -s0 : (q == 2 ? -c0 : s0));
        const long double lr = logl(u);
        const double ln = lbf::u21_ln(b);
        double sn, cs;
        lbf::u21_sincos_turn(b, sn, cs);
        eln = fmax(eln, (double)fabsl((ln - lr) / lr));
        esn = fmax(esn, (double)fabsl((sn - sr) / sr));
        ecs = fmax(ecs, (double)fabsl((cs - cr) / cr));
        const double ud = ((double)b + 0.5) * 0x1p-21, td = 2.0 * M_PI * ud;
        // absolute for sine and cosine: 2 pi u rounded in double moves the oracle's values by
        // up to ~7e-16 where they pass through zero
        oln = fmax(oln, fabs((ln - log(ud)) / log(ud)));
        osn = fmax(osn, fabs(sn - sin(td)));
        ocs = fmax(ocs, fabs(cs - cos(td)));
    }
    printf("vs long double: ln %.3e sin %.3e cos %.3e\n", eln, esn, ecs);
    printf("vs double libm (the oracle's calls): ln %.3e (relative) sin %.3e cos %.3e (absolute)\n", oln, osn, ocs);
    return eln > bound || esn > bound || ecs > bound || osn > 2e-15 || ocs > 2e-15;
}
