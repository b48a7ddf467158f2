/* Oracle CNN switch: filled in with the regime classifier. */
#include "or_internal.h"

double or_cnn_switch(or_sim *s, const double *nmom, const double *u2mom, uint8_t *hot,
                     uint8_t *cold) {
    (void)s; (void)nmom; (void)u2mom; (void)hot; (void)cold;
    return 0.0;
}
void or_cnn_free(or_sim *s) { (void)s; }
