// Session pieces the request server drives (session.hip): a session step
// as a state machine that never waits on the device. The server calls
// session_begin_step, then, each time the session's event has completed,
// session_advance until it reports the step done.
#pragma once

#include "kde_internal.hpp"

namespace kde {

double ad_upper_tail(double a2);
// Enqueue the fixed part of a step and record the session's event.
kde_status session_begin_step(kde_session* s);
// After the event completed: apply the update rule; either the step is done
// (*done = true; the next widths are enqueued) or a CV scan was enqueued and
// the event recorded again. KDE_E_NUMERIC (step counted) when a
// non-finite position or width reached the step.
kde_status session_advance(kde_session* s, bool* done);
hipEvent_t session_event(const kde_session* s);
size_t session_arena_bytes(const kde_session* s);
// Seconds since the current step began.
double session_step_seconds(const kde_session* s);

}  // namespace kde
