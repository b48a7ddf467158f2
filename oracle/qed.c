/* Oracle QED module: filled in with the photon-emission and pair-creation
 * rates; until then QED runs are rejected by the Python wrapper. */
#include "or_internal.h"

void or_qed_init(or_sim *s) { (void)s; }
void or_qed_free(or_sim *s) { (void)s; }
void or_qed_emit(or_sim *s, int sp, size_t i, const double e[3], const double b[3]) {
    (void)s; (void)sp; (void)i; (void)e; (void)b;
}
void or_photon_phase(or_sim *s) { (void)s; }
