// ram_stream.h -- ordering of one context's work across the streams it is
// pointed at (host code only; no HIP types here, so that a host unit test can
// drive it with a recording stand-in for the runtime).
//
// Every call of a context reads and rewrites the context's device scratch
// (mesh tables, tile plan, ping-pong state) on the context's current stream.
// When the caller moves the context to another stream, the new stream first
// waits for everything already issued on the old one, so that calls made on
// different streams run one after the other on that scratch, in the order
// they were issued.  ram_destroy and the scratch's reallocation then only
// need to wait for the current stream.
//
// A stream under graph capture takes no part in the hand-off (an event
// recorded inside a capture cannot order work outside it, and a capturing
// stream cannot wait on work outside its capture): whoever captures orders
// the captured calls against the others.
#pragma once

namespace ram {

// Api supplies the runtime operations:
//   bool capturing(stream_t s)            s is capturing a graph now (or its
//                                         state cannot be read: treated alike)
//   int record(event_t ev, stream_t s)    mark the end of s's work so far
//   int wait(stream_t s, event_t ev)      s waits for that mark
// (record and wait return 0 on success).  On failure the context keeps its old
// stream and the error is returned.
template <class Api>
int switch_stream(Api &api, typename Api::stream_t &cur, typename Api::stream_t next,
                  typename Api::event_t ev)
{
    if (next == cur) return 0;
    if (!api.capturing(cur) && !api.capturing(next)) {
        int err = api.record(ev, cur);
        if (err != 0) return err;
        if ((err = api.wait(next, ev)) != 0) return err;
    }
    cur = next;
    return 0;
}

}  // namespace ram
